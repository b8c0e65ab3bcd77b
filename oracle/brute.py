"""Brute-force longest-prefix match: the definition written out.

Test infrastructure only (see the package docstring).  Follows the problem
statement of the paper's Background section (the router picks the rule with
the longest matching prefix) and the Design section's default route for
uncovered space.
"""
from __future__ import annotations

import numpy as np

NO_ROUTE = 0xFFFF
_M128 = (1 << 128) - 1


def _as_int(row) -> int:
    return (int(row[0]) << 64) | int(row[1])


def lpm_one(x: int, rules) -> int:
    """rules: iterable of (prefix_int, length, next_hop).  Pure Python ints."""
    best_len, best = -1, NO_ROUTE
    for P, L, nh in rules:
        shift = 128 - L
        if (x >> shift) == (P >> shift) and L > best_len:
            best_len, best = L, nh
    return best


def rules_of(prefixes: np.ndarray, lengths: np.ndarray, next_hops: np.ndarray):
    return [(_as_int(prefixes[i]), int(lengths[i]), int(next_hops[i]))
            for i in range(lengths.shape[0])]


def lpm_bruteforce(prefixes, lengths, next_hops, addrs) -> np.ndarray:
    """Pure-Python scan of every rule for every address (small cases only)."""
    rules = rules_of(prefixes, lengths, next_hops)
    out = np.empty(addrs.shape[0], dtype=np.uint16)
    for i in range(addrs.shape[0]):
        out[i] = lpm_one(_as_int(addrs[i]), rules)
    return out


def lpm_bruteforce_np(prefixes, lengths, next_hops, addrs) -> np.ndarray:
    """The same scan, vectorised over the rules with numpy (medium cases)."""
    n = lengths.shape[0]
    out = np.full(addrs.shape[0], NO_ROUTE, dtype=np.uint16)
    if n == 0:
        return out
    net_hi = np.empty(n, dtype=np.uint64)
    net_lo = np.empty(n, dtype=np.uint64)
    for i in range(n):
        net = (_M128 << (128 - int(lengths[i]))) & _M128
        net_hi[i] = net >> 64
        net_lo[i] = net & 0xFFFFFFFFFFFFFFFF
    p_hi = prefixes[:, 0] & net_hi
    p_lo = prefixes[:, 1] & net_lo
    L = lengths.astype(np.int32)
    for j in range(addrs.shape[0]):
        hit = ((addrs[j, 0] & net_hi) == p_hi) & ((addrs[j, 1] & net_lo) == p_lo)
        if hit.any():
            cand = np.nonzero(hit)[0]
            out[j] = next_hops[cand[np.argmax(L[cand])]]
    return out
