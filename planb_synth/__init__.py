"""Seeded synthetic FIBs and lookup traffic shaped like backbone IPv6 tables.

This module is the only code that both the GPU path's tests/bench and the CPU
oracle receive inputs from.  It holds none of the lookup method's arithmetic:
no range conversion, no interval partitioning, no tree layout and no
longest-prefix matching.  It only draws prefixes (with their host bits zero),
prefix lengths, next hops and destination addresses from numpy's PCG64.

Addresses and prefixes are numpy arrays of shape (n, 2) and dtype uint64,
column 0 = the high 64 bits (address bytes 0..7 read big-endian), column 1 =
the low 64 bits.  In memory each row is therefore the 16-byte record
{uint64 hi; uint64 lo;} that the C ABI takes.

Workload recipes (the paper's real RIPE/RouteViews tables and traces are not
available; these stand in for them, after the statistics of the paper's
Table 1 and its synthetic FIBs / traces in the evaluation section):

* ``tiny``      1,000 prefixes + ::/0; /32 20 %, /48 40 %, /40 10 %, /44 10 %,
                the other 20 % uniform over the remaining 45 lengths in /16-/64;
                ~15 % nested extensions up to depth 3; next hops 0..255.
* ``backbone``  200,000 prefixes; /48 45 %, /32 15 %, /44 10 %, /40 8 %,
                /36 5 %, /29-/31 5 %, /56-/64 12 %; ~12 % nested up to depth 4;
                next hops 0..65534.
* ``large``     1,000,000 prefixes; the backbone histogram x 0.95 plus 5 %
                /128 host routes.
* ``vrf``       a table of the ``tiny`` histogram with a given prefix count
                (log-uniform 50k..500k across 16 tables) plus ::/0.
* ``ipv4``      1,000,000 IPv4 prefixes shaped like a full BGP table: /24 58 %,
                /22 11 %, /23 9 %, /21 5 %, /20 4 %, /19 3 %, /16 2.5 %,
                /18 1.5 %, /17 1 %, /25-/32 4 % (uniform), and /8-/15 0.36 %
                (rising from 0.002 % at /8 to 0.15 % at /15: there are only
                2^L prefixes of length L); ~12 % nested up to depth 3; next
                hops 0..65534.  IPv4 rules and addresses are placed in the top
                32 bits of the 128-bit space (a 32-bit address a stands for
                a << 96).
* ``ipv4_tiny`` 2,000 prefixes of the ``ipv4`` histogram plus 0.0.0.0/0.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass

import numpy as np

U64 = np.uint64
ALL_ONES = np.uint64(0xFFFFFFFFFFFFFFFF)
NO_ROUTE = 0xFFFF


def _host_mask_tables():
    """HOST_HI[L], HOST_LO[L]: the bits of a 128-bit word below the top L bits."""
    hi = np.zeros(129, dtype=U64)
    lo = np.zeros(129, dtype=U64)
    for L in range(129):
        host = (1 << (128 - L)) - 1
        hi[L] = np.uint64(host >> 64)
        lo[L] = np.uint64(host & 0xFFFFFFFFFFFFFFFF)
    return hi, lo


HOST_HI, HOST_LO = _host_mask_tables()


# --------------------------------------------------------------------------
# prefix-length histograms
# --------------------------------------------------------------------------
def _hist(named: dict[int, float], rest_share: float = 0.0, rest_range=None):
    w = np.zeros(129, dtype=np.float64)
    for L, p in named.items():
        w[L] += p
    if rest_share:
        others = [L for L in range(rest_range[0], rest_range[1] + 1) if L not in named]
        for L in others:
            w[L] += rest_share / len(others)
    return w / w.sum()


TINY_HIST = _hist({32: 0.20, 48: 0.40, 40: 0.10, 44: 0.10}, 0.20, (16, 64))


def _backbone_weights():
    d = {48: 0.45, 32: 0.15, 44: 0.10, 40: 0.08, 36: 0.05}
    for L in (29, 30, 31):
        d[L] = d.get(L, 0.0) + 0.05 / 3
    for L in range(56, 65):
        d[L] = d.get(L, 0.0) + 0.12 / 9
    return _hist(d)


BACKBONE_HIST = _backbone_weights()


def _ipv4_weights():
    d = {24: 0.58, 22: 0.11, 23: 0.09, 21: 0.05, 20: 0.04, 19: 0.03, 16: 0.025, 18: 0.015, 17: 0.01}
    # short prefixes are few (there are only 2^L of each length L)
    for L, p in {8: 2e-5, 9: 2e-5, 10: 5e-5, 11: 1e-4, 12: 3e-4, 13: 6e-4, 14: 1e-3, 15: 1.5e-3}.items():
        d[L] = p
    for L in range(25, 33):
        d[L] = d.get(L, 0.0) + 0.04 / 8
    return _hist(d)


IPV4_HIST = _ipv4_weights()
LARGE_HIST = BACKBONE_HIST * 0.95
LARGE_HIST[128] += 0.05
LARGE_HIST = LARGE_HIST / LARGE_HIST.sum()


@dataclass(frozen=True)
class FibSpec:
    name: str
    n_prefixes: int          # not counting the default route
    hist: np.ndarray
    ext_share: float
    max_depth: int
    nh_max: int              # next hops drawn uniformly from 0..nh_max
    default_route: bool
    v4: bool = False         # IPv4 rules (lengths <= 32) in the top 32 bits


TINY = FibSpec("tiny", 1000, TINY_HIST, 0.15, 3, 255, True)
BACKBONE = FibSpec("backbone", 200_000, BACKBONE_HIST, 0.12, 4, 65534, False)
LARGE = FibSpec("large", 1_000_000, LARGE_HIST, 0.12, 4, 65534, False)
IPV4 = FibSpec("ipv4", 1_000_000, IPV4_HIST, 0.12, 3, 65534, False, True)
IPV4_TINY = FibSpec("ipv4_tiny", 2_000, IPV4_HIST, 0.15, 3, 255, True, True)


def vrf_spec(n_prefixes: int) -> FibSpec:
    return FibSpec(f"vrf{n_prefixes}", n_prefixes, TINY_HIST, 0.15, 3, 65534, True)


@dataclass
class Fib:
    prefixes: np.ndarray     # (n, 2) uint64, host bits zero
    lengths: np.ndarray      # (n,) uint8
    next_hops: np.ndarray    # (n,) uint16
    name: str = ""

    def __len__(self):
        return int(self.lengths.shape[0])


# --------------------------------------------------------------------------
# random 128-bit words
# --------------------------------------------------------------------------
def _rand_u64(rng, n):
    return rng.integers(0, np.iinfo(np.uint64).max, size=n, dtype=U64, endpoint=True)


def uniform_2000_3(rng, n):
    """n addresses uniform over 2000::/3 (top three bits 001)."""
    out = np.empty((n, 2), dtype=U64)
    out[:, 0] = (_rand_u64(rng, n) & np.uint64((1 << 61) - 1)) | np.uint64(1 << 61)
    out[:, 1] = _rand_u64(rng, n)
    return out


def uniform_v4(rng, n):
    """n IPv4 addresses uniform over the 32-bit space, placed in the top 32 bits."""
    out = np.zeros((n, 2), dtype=U64)
    out[:, 0] = rng.integers(0, 1 << 32, size=n, dtype=U64) << U64(32)
    return out


def _apply_len(hi, lo, lens):
    """Zero the host bits of (hi, lo) for prefix lengths ``lens``."""
    return hi & ~HOST_HI[lens], lo & ~HOST_LO[lens]


def _draw_lengths(rng, hist, n, above=None):
    """Lengths from ``hist``; with ``above`` given, conditioned on L > above."""
    cdf = np.cumsum(hist)
    cdf[-1] = 1.0
    if above is None:
        u = rng.random(n)
    else:
        lo = cdf[above]
        u = lo + (1.0 - lo) * rng.random(n)
    L = np.searchsorted(cdf, u, side="right")
    return np.minimum(L, 128).astype(np.uint8)


# --------------------------------------------------------------------------
# FIB generator
# --------------------------------------------------------------------------
def make_fib(spec: FibSpec, seed: int) -> Fib:
    """Draw a FIB of ``spec.n_prefixes`` unique (prefix, length) rules.

    Non-nested prefixes are uniform in 2000::/3 (IPv4 specs: uniform over
    the 32-bit space, in the top 32 bits).  A share ``spec.ext_share``
    are extensions: they copy a random existing prefix of depth < max_depth,
    draw their own length from the histogram conditioned on being longer, and
    randomise the bits between the two lengths.  Duplicates after masking are
    re-drawn.  ::/0 is appended when ``spec.default_route``.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    N = spec.n_prefixes
    hist = spec.hist
    maxlen = int(np.nonzero(hist)[0].max())
    n_ext = int(round(spec.ext_share * N))
    n_base = N - n_ext
    space = uniform_v4 if spec.v4 else uniform_2000_3

    def base(n):
        L = _draw_lengths(rng, hist, n)
        a = space(rng, n)
        hi, lo = _apply_len(a[:, 0], a[:, 1], L)
        return hi, lo, L

    hi, lo, L = base(n_base)
    depth = np.ones(n_base, dtype=np.int8)
    rounds = max(1, spec.max_depth - 1)
    per_round = np.full(rounds, n_ext // rounds)
    per_round[: n_ext % rounds] += 1
    for nr in per_round:
        if nr == 0:
            continue
        elig = np.nonzero((depth < spec.max_depth) & (L < maxlen))[0]
        par = elig[rng.integers(0, elig.size, size=nr)]
        Lp = L[par]
        Lc = _draw_lengths(rng, hist, nr, above=Lp)
        r = space(rng, nr)
        # keep the parent's top Lp bits, randomise bits Lp..Lc-1, zero the rest
        chi = (hi[par] & ~HOST_HI[Lp]) | (r[:, 0] & HOST_HI[Lp])
        clo = (lo[par] & ~HOST_LO[Lp]) | (r[:, 1] & HOST_LO[Lp])
        chi, clo = _apply_len(chi, clo, Lc)
        hi = np.concatenate([hi, chi])
        lo = np.concatenate([lo, clo])
        L = np.concatenate([L, Lc])
        depth = np.concatenate([depth, depth[par] + 1])

    # re-draw duplicates as fresh non-nested prefixes of the same length
    for _ in range(1000):
        rec = np.empty(hi.size, dtype=[("hi", U64), ("lo", U64), ("L", np.uint8)])
        rec["hi"], rec["lo"], rec["L"] = hi, lo, L
        _, first = np.unique(rec, return_index=True)
        dup = np.setdiff1d(np.arange(hi.size), first)
        if dup.size == 0:
            break
        a = space(rng, dup.size)
        hi[dup], lo[dup] = _apply_len(a[:, 0], a[:, 1], L[dup])
    else:  # pragma: no cover
        raise RuntimeError("could not draw a duplicate-free FIB")

    perm = rng.permutation(hi.size)
    prefixes = np.stack([hi[perm], lo[perm]], axis=1)
    lengths = L[perm].astype(np.uint8)
    nh = rng.integers(0, spec.nh_max + 1, size=hi.size).astype(np.uint16)
    if spec.default_route:
        prefixes = np.concatenate([prefixes, np.zeros((1, 2), dtype=U64)])
        lengths = np.concatenate([lengths, np.zeros(1, dtype=np.uint8)])
        nh = np.concatenate([nh, rng.integers(0, spec.nh_max + 1, size=1).astype(np.uint16)])
    return Fib(np.ascontiguousarray(prefixes), lengths, nh, spec.name)


def vrf_tables(n_tables: int = 16, seed: int = 5000, lo: int = 50_000, hi: int = 500_000):
    """``n_tables`` FIBs with prefix counts log-uniform over [lo, hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_tables))).astype(int)
    return [make_fib(vrf_spec(int(s)), seed + 1 + t) for t, s in enumerate(sizes)]


# --------------------------------------------------------------------------
# traffic generators
# --------------------------------------------------------------------------
def inside_prefixes(rng, fib: Fib, idx: np.ndarray) -> np.ndarray:
    """One address inside each prefix fib[idx]: the prefix plus a uniform suffix."""
    L = fib.lengths[idx]
    r = uniform_2000_3(rng, idx.size)
    out = np.empty((idx.size, 2), dtype=U64)
    out[:, 0] = fib.prefixes[idx, 0] | (r[:, 0] & HOST_HI[L])
    out[:, 1] = fib.prefixes[idx, 1] | (r[:, 1] & HOST_LO[L])
    return out


def mixed_traffic(fib: Fib, n: int, inside_share: float, seed: int,
                  chunk: int = 1 << 23, out: np.ndarray | None = None) -> np.ndarray:
    """``n`` addresses: a share ``inside_share`` falls inside a prefix chosen
    uniformly among the non-default prefixes, the rest is uniform over 2000::/3."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if out is None:
        out = np.empty((n, 2), dtype=U64)
    cand = np.nonzero(fib.lengths > 0)[0]
    for s in range(0, n, chunk):
        c = min(chunk, n - s)
        inside = rng.random(c) < inside_share
        blk = uniform_2000_3(rng, c)
        k = int(inside.sum())
        if k and cand.size:
            idx = cand[rng.integers(0, cand.size, size=k)]
            blk[inside] = inside_prefixes(rng, fib, idx)
        out[s:s + c] = blk
    return out


def tiny_traffic(fib: Fib, n: int = 1 << 20, seed: int = 1011) -> np.ndarray:
    return mixed_traffic(fib, n, 0.5, seed)


def backbone_traffic(fib: Fib, n: int = 1 << 28, seed: int = 1022, out=None) -> np.ndarray:
    return mixed_traffic(fib, n, 0.7, seed, out=out)


def zipf_traffic(fib: Fib, n: int, seed: int, s: float = 1.1, chunk: int = 1 << 21) -> np.ndarray:
    """Destinations Zipf(s) over a random ranking of the prefixes (bounded
    inverse-CDF over the N ranks), each with a uniform random suffix.  Chunks
    of ``chunk`` addresses draw from their own seeded streams (seed, chunk
    number) on a pool of host threads, so the result does not depend on the
    thread count."""
    from concurrent.futures import ThreadPoolExecutor
    rng = np.random.Generator(np.random.PCG64(seed))
    N = len(fib)
    rank_to_prefix = rng.permutation(N)
    w = np.arange(1, N + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    out = np.empty((n, 2), dtype=U64)

    def one(k):
        lo, hi = k * chunk, min(n, (k + 1) * chunk)
        g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, k + 1])))
        r = np.minimum(np.searchsorted(cdf, g.random(hi - lo), side="right"), N - 1)
        out[lo:hi] = inside_prefixes(g, fib, rank_to_prefix[r])

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(one, range((n + chunk - 1) // chunk)))
    return out


def ipv4_traffic(fib: Fib, n: int, inside_share: float, seed: int, chunk: int = 1 << 23) -> np.ndarray:
    """``n`` 32-bit IPv4 addresses (uint32) for an IPv4 FIB: a share
    ``inside_share`` inside a prefix chosen uniformly among the non-default
    prefixes (prefix plus a uniform suffix), the rest uniform over 2^32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty(n, dtype=np.uint32)
    cand = np.nonzero(fib.lengths > 0)[0]
    top = (fib.prefixes[:, 0] >> U64(32)).astype(np.uint32)
    for s in range(0, n, chunk):
        c = min(chunk, n - s)
        blk = rng.integers(0, 1 << 32, size=c, dtype=np.uint64).astype(np.uint32)
        inside = rng.random(c) < inside_share
        k = int(inside.sum())
        if k and cand.size:
            idx = cand[rng.integers(0, cand.size, size=k)]
            host = (np.uint64(1) << (32 - fib.lengths[idx].astype(np.uint64))) - np.uint64(1)
            blk[inside] = top[idx] | (blk[inside] & host.astype(np.uint32))
        out[s:s + c] = blk
    return out


def v4_as_128(addrs: np.ndarray) -> np.ndarray:
    """32-bit addresses as the (n, 2) uint64 records of the 128-bit space (a << 96)."""
    out = np.zeros((addrs.shape[0], 2), dtype=U64)
    out[:, 0] = addrs.astype(U64) << U64(32)
    return out


def log_uniform_sizes(rng, n: int, lo: int, hi: int) -> np.ndarray:
    return np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi + 1), size=n))).astype(np.int64).clip(lo, hi)


def uneven_batches(fib: Fib, n_batches: int = 512, lo: int = 64, hi: int = 1 << 22,
                   seed: int = 1033):
    """Batch sizes log-uniform over [lo, hi] and Zipf(1.1) destinations,
    returned as (sizes, addresses concatenated in batch order)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = log_uniform_sizes(rng, n_batches, lo, hi)
    addrs = zipf_traffic(fib, int(sizes.sum()), seed + 1)
    return sizes, addrs


def poisson_bursts(tables, n_bursts: int, rate_per_s: float, seed: int,
                   lo: int = 32, hi: int = 4096):
    """Burst arrivals: exponential inter-arrival times (Poisson process of rate
    ``rate_per_s``), sizes log-uniform over [lo, hi], table ids uniform; each
    burst's addresses follow the tiny-config mix (50 % inside a prefix)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.cumsum(rng.exponential(1.0 / rate_per_s, size=n_bursts))
    sizes = log_uniform_sizes(rng, n_bursts, lo, hi)
    tid = rng.integers(0, len(tables), size=n_bursts)
    addrs = []
    for b in range(n_bursts):
        addrs.append(mixed_traffic(tables[tid[b]], int(sizes[b]), 0.5,
                                   int(rng.integers(0, 2**62))))
    return t, sizes, tid, addrs


# --------------------------------------------------------------------------
# small helpers for tests (conversion only)
# --------------------------------------------------------------------------
def to_int(row) -> int:
    return (int(row[0]) << 64) | int(row[1])


def from_ints(vals) -> np.ndarray:
    vals = list(vals)
    out = np.empty((len(vals), 2), dtype=U64)
    for i, v in enumerate(vals):
        out[i, 0] = (v >> 64) & 0xFFFFFFFFFFFFFFFF
        out[i, 1] = v & 0xFFFFFFFFFFFFFFFF
    return out
