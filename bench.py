"""Benchmark: batched IPv6 longest-prefix-match lookups on one MI355X.

Workload (the headline): a backbone-shaped synthetic FIB of 200,000 prefixes
and 2^28 synthetic destination addresses (70 % inside a prefix, 30 % uniform in
2000::/3), resident in HBM before timing.  A step is one lookup pass over the
whole batch.  Prints ONE JSON line on stdout; progress goes to stderr.

Legs (all on the same FIB and address batch unless stated):
  plain      autotuned tree descent (fanout 8/16/32 and launch shape), the
             headline value; also the same with 128-bit key slots forced
  learned    the MLP-guided bounded search (trained here), exact, with its
             fallback rate and its speedup over the plain lookup
  batches    uneven batches (log-uniform 64..2^22) replayed one at a time:
             per-batch latency p50/p99 for plain launches and graph replays
  uneven     the 1M-prefix FIB with /128 host routes (128-bit keys): 512
             Zipf batches of 64..2^22, autotuned per size bucket; eager,
             persistent and graph throughput, one-at-a-time latency, and
             0 mismatches against the oracle over every batch
  serving    16 VRF-style tables (50k..500k prefixes) behind the serving
             runtime, Poisson bursts of 32..4096 at 25/50/80 % of capacity
  cpu        the binary-trie oracle over the whole batch on the host cores
             (also the full-size parity check: mismatches must be 0)
Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "lookups/sec (GLPS) on 200k-prefix FIB, plain vs learned; p99 batch latency"
HBM_PEAK_GBS = 8000.0
BYTES_PER_LOOKUP = 18  # 16-byte address read + 2-byte next hop written
KERNEL_SOURCES = ["paper_2604_14650_amd/csrc/lookup.hip", "paper_2604_14650_amd/csrc/descent.hpp",
                  "paper_2604_14650_amd/csrc/device.hpp", "paper_2604_14650_amd/csrc/leaf_format.hpp"]
TRAFFIC_FILE = "profiles/lookup_backbone_2e28_traffic.txt"
TRACE_FILE = "profiles/lookup_backbone_2e28_trace.txt"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--addresses", type=int, default=28, help="log2 of the batch size")
    ap.add_argument("--quick", action="store_true", help="headline plain lookup only (for profiling)")
    ap.add_argument("--copy-probe", action="store_true", help="also run a 1 GiB device copy (PMC scaling)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the autotuner legs (the headline always runs the fixed launch shapes; fewer launches to profile)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-learned", action="store_true")
    ap.add_argument("--learned-epochs", type=int, default=0,
                    help="training passes for the learned leg (0: the library default); short runs for profiling")
    ap.add_argument("--skip-batches", action="store_true")
    ap.add_argument("--skip-uneven", action="store_true", help="skip the 1M-prefix uneven-batch leg")
    ap.add_argument("--skip-ablation", action="store_true")
    ap.add_argument("--skip-rebuild", action="store_true")
    ap.add_argument("--skip-ipv4", action="store_true")
    ap.add_argument("--skip-serving", action="store_true")
    ap.add_argument("--size-sweep", action="store_true",
                    help="also time FIBs of 25k..1M prefixes with the backbone's length mix (not in the default run)")
    return ap.parse_args()


def upload(addrs: np.ndarray, chunk: int = 1 << 24):
    import torch
    n = addrs.shape[0]
    d = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        d[s:e].copy_(torch.from_numpy(addrs[s:e].view(np.int64)))
    torch.cuda.synchronize()
    return d


def time_steps(fn, steps: int, warmup: int):
    """Per-step seconds, timed with events on torch's current stream -- the
    stream every lookup here is launched on (each step is one launch)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    evs[0].record()
    for i in range(steps):
        fn()
        evs[i + 1].record()
    torch.cuda.synchronize()
    return [evs[i].elapsed_time(evs[i + 1]) / 1e3 for i in range(steps)]


def kernel_hash() -> str:
    """SHA-1 (12 hex digits) of the headline kernel's sources with comments and
    blank lines removed: a comment-only edit keeps a profile summary valid."""
    import re
    h = hashlib.sha1()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), encoding="utf-8") as f:
            src = re.sub(r"/\*.*?\*/", "", f.read(), flags=re.S)
        for line in src.splitlines():
            code = line.split("//", 1)[0].rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:12]


def _profile_fields(path: str, per_launch_lookups: int, config: str):
    """key = value fields of a committed rocprofv3 summary, if it was taken with
    the current kernel sources and the same kernel configuration (else None)."""
    path = os.path.join(ROOT, path)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if (kv.get("kernel_sources_sha1") != kernel_hash() or int(kv.get("lookups_per_launch", -1)) != per_launch_lookups
            or kv.get("kernel_config") != config):
        return None
    return kv


def measured_traffic(per_launch_lookups: int, config: str):
    """HBM bytes per launch from the committed PMC summary (or None)."""
    kv = _profile_fields(TRAFFIC_FILE, per_launch_lookups, config)
    return None if kv is None else float(kv["hbm_bytes_per_launch"])


def profiled_kernel_ns(per_launch_lookups: int, config: str):
    """The headline kernel's average duration in the committed kernel-trace
    summary over the dispatches of its timed steps (warm-up and the parity check
    excluded), else over all its dispatches; None without a matching summary."""
    kv = _profile_fields(TRACE_FILE, per_launch_lookups, config)
    if kv is None:
        return None
    return float(kv.get("kernel_timed_avg_ns", kv["kernel_avg_ns"]))


# Launch shapes the autotuner chose for this workload on MI355X (used with --no-autotune).
KNOWN_TUNING = {0: {"fanout": 8, "tuning": (2, 5, 2, 1024, 2)}, 128: {"fanout": 8, "tuning": (2, 5, 1, 1024, 1)}}
# the tiny FIB (2,003 intervals): every level in LDS, one lane group per lookup
TINY_TUNING = {"fanout": 8, "tuning": (2, -1, 2, 1024, 1)}


def plain_leg(P, fib, d, n, out, args):
    """The headline runs the fixed launch configuration above (the one the
    committed rocprofv3 summaries were taken with); the autotuner's pick on
    this GPU is timed on the same batch and reported beside it."""
    from paper_2604_14650_amd import autotune
    sample = min(n, 1 << 24)
    res, handles, times = {}, {}, {}
    for kb in (0, 128):
        k = KNOWN_TUNING[kb]
        h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, fanout=k["fanout"], key_bits=kb)
        P.planb_set_tuning(h, *k["tuning"])
        rec = {"fanout": k["fanout"], "tuning": P.planb_get_tuning(h)}
        if kb == 0:
            times[kb] = time_steps(lambda: P.planb_lookup(h, d, n, out), args.steps, args.warmup)
        else:
            times[kb] = time_steps(lambda: P.planb_lookup(h, d, n, out), max(3, args.steps // 2), 1)
        if not args.no_autotune:
            ht, tr = autotune.tune(fib.prefixes, fib.lengths, fib.next_hops, d, sample, key_bits=kb,
                                   cache_path=None, reps=3, log=log)
            tt = time_steps(lambda: P.planb_lookup(ht, d, n, out), max(3, args.steps // 2), 1)
            rec["autotuned"] = {"fanout": tr["fanout"], "tuning": tr["tuning"],
                                "glps": round(n / (sum(tt) / len(tt)) / 1e9, 3), "fanout_sweep_glps": tr["fanout_glps"]}
            del ht
        handles[kb] = h
        res[kb] = rec
        log(f"key_bits={kb}: {rec}")
    return handles[0], res, times[0], times[128]


def learned_on(P, fib, d, n, out, tuning, steps, want=None, epochs=0, keep=None):
    """Plain and learned lookups on one FIB and resident batch: both timed with
    events over `steps` launches, the learned results compared with the plain
    ones (and with the oracle's, when given), the fallback rate counted.  With
    a list as `keep`, the learned results (host array) are appended to it."""
    import torch
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, fanout=tuning["fanout"])
    P.planb_set_tuning(h, *tuning["tuning"])
    tp = time_steps(lambda: P.planb_lookup(h, d, n, out), steps, 2)
    torch.cuda.synchronize()
    plain_out = out.clone()
    t0 = time.time()
    rep = P.planb_train(h, epochs=epochs, seed=1)
    train_s = time.time() - t0
    eps = P.planb_model_get_eps(h, 1 << 16).astype(np.int64)
    used = eps[eps != 0xFFFFFFFF]
    fb = torch.zeros(1, dtype=torch.int32, device="cuda")
    lout = torch.empty_like(out)
    P.planb_lookup_learned(h, d, n, lout, fb)
    torch.cuda.synchronize()
    fallbacks = int(fb.item())
    same = bool(torch.equal(lout, plain_out))
    mism = None if want is None else int((lout.cpu().numpy().view(np.uint16) != want).sum())
    if keep is not None:
        keep.append(lout.cpu().numpy().view(np.uint16))
    tl = time_steps(lambda: P.planb_lookup_learned(h, d, n, lout), steps, 2)
    plain_glps = n / (sum(tp) / len(tp)) / 1e9
    glps = n / (sum(tl) / len(tl)) / 1e9
    achieved = BYTES_PER_LOOKUP * glps  # GB/s of algorithmic bytes (16 B in, 2 B out per lookup)
    info = P.planb_get_info(h)
    h.close()
    return {"glps": round(glps, 3), "ms_per_step": round(sum(tl) / len(tl) * 1e3, 4),
            "plain_glps": round(plain_glps, 3), "speedup_vs_plain": round(glps / plain_glps, 4),
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4)},
            "fallback_rate": round(fallbacks / n, 6), "identical_to_plain": same, "mismatches_vs_oracle": mism,
            "addresses": n, "intervals": info["intervals"], "fanout": info["fanout"], "key_bits": info["key_bits"],
            "eps_per_segment": {"segments": int(eps.size), "empty": int(eps.size - used.size),
                                "p50": float(np.median(used)) if used.size else None,
                                "p90": float(np.percentile(used, 90)) if used.size else None,
                                "max": int(used.max()) if used.size else None},
            "train_seconds": round(train_s, 2), "train_steps": rep["steps"], "final_loss": rep["final_loss"]}


def learned_leg(P, fib, d, n, out, args, keep=None):
    """The learned position model on the two FIBs it is specified for: the
    backbone FIB with the headline batch (its results appended to `keep`, for
    the oracle's check once the oracle has run), and the tiny FIB with its 2^20
    addresses (checked against the oracle here)."""
    import torch
    import planb_synth as S
    from oracle.trie import Trie
    res = {"backbone": learned_on(P, fib, d, n, out, KNOWN_TUNING[0], max(3, args.steps // 2),
                                  epochs=args.learned_epochs, keep=keep)}
    log(f"learned backbone: {res['backbone']}")
    tiny = S.make_fib(S.TINY, 11)
    ta = S.tiny_traffic(tiny, 1 << 20, seed=1011)
    want = Trie(tiny.prefixes, tiny.lengths, tiny.next_hops).lookup(ta)
    td = upload(ta)
    tout = torch.empty(ta.shape[0], dtype=torch.int16, device="cuda")
    res["tiny"] = learned_on(P, tiny, td, ta.shape[0], tout, TINY_TUNING, 50, want, epochs=args.learned_epochs)
    log(f"learned tiny: {res['tiny']}")
    return res


def batches_leg(P, h, d, n, out, seed=1044, count=96):
    """Uneven batches (log-uniform 64..2^22) drawn as slices of the resident
    batch, each run alone: latency of a plain launch and of a graph replay
    (enqueue to completion, host clock), and lookups/s over the set."""
    import torch
    import planb_synth as S
    rng = np.random.default_rng(seed)
    top = min(1 << 22, n // 2)
    sizes = S.log_uniform_sizes(rng, count, 64, top)
    starts = rng.integers(0, n - top + 1, size=count)
    g = P.Graph(h, 4)
    lat = {"plain": [], "graph": []}
    stream = torch.cuda.current_stream()
    for k in range(count):
        a, o, m = d[starts[k]:], out[starts[k]:], int(sizes[k])
        for mode in ("plain", "graph", "plain", "graph"):  # first of each is a warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if mode == "plain":
                P.planb_lookup(h, a, m, o)
            else:
                g.launch([(a, o, m)])
            stream.synchronize()
            lat[mode].append((time.perf_counter() - t0) * 1e6)
    g.close()
    res = {}
    for mode, v in lat.items():
        v = np.array(v[1::2])  # the timed runs
        res[mode] = {"p50_us": round(float(np.percentile(v, 50)), 2), "p99_us": round(float(np.percentile(v, 99)), 2),
                     "glps": round(float(sizes.sum() / (v.sum() / 1e6) / 1e9), 3)}
    res["batches"] = int(count)
    res["sizes"] = "log-uniform 64..4194304"
    return res


def uneven_leg(P, log_fn, n_batches=512, seed=1033, buckets=(256, 4096, 1 << 16, 1 << 20, 1 << 22)):
    """Uneven batches on the 1M-prefix FIB with 5 % /128 host routes (so 128-bit
    keys): 512 batches, sizes log-uniform over 64..2^22, Zipf(1.1) destinations.
    Launch shapes are autotuned per batch-size bucket (fanout by the summed
    bucket times).  Timed: every batch as its own planb_lookup back to back,
    all of them in one persistent launch, and in one graph replay; then each
    batch alone (enqueue to completion, host clock) as a plain launch and as a
    graph replay of its bucket's shape, and empty graph replays (the replay's
    own cost).  The persistent launch and the graph over every batch take the
    shape, of the two largest buckets' picks, that runs this batch set fastest
    (autotune.tune_batches).  Every mode's output is compared with the trie
    oracle over all batches."""
    import torch
    import planb_synth as S
    from oracle.trie import Trie, default_threads
    from paper_2604_14650_amd import autotune
    t0 = time.time()
    fib = S.make_fib(S.LARGE, 33)
    sizes, addrs = S.uneven_batches(fib, n_batches, 64, 1 << 22, seed)
    total = int(sizes.sum())
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    log_fn(f"uneven: {len(fib)} prefixes, {n_batches} batches, {total} lookups ({time.time() - t0:.1f} s)")
    t0 = time.time()
    want = Trie(fib.prefixes, fib.lengths, fib.next_hops).lookup(addrs, default_threads())
    log_fn(f"uneven: oracle over every batch ({time.time() - t0:.1f} s)")
    d = upload(addrs)
    del addrs
    out = torch.empty(total, dtype=torch.int16, device="cuda")
    h, rec = autotune.tune_sizes(fib.prefixes, fib.lengths, fib.next_hops, d, list(buckets), cache_path=None, reps=3,
                                 log=log_fn)
    info = P.planb_get_info(h)
    table = P.planb_get_size_tunings(h)
    mism = {}

    def check(name):
        torch.cuda.synchronize()
        mism[name] = int((out.cpu().numpy().view(np.uint16) != want).sum())
        out.fill_(-1)

    def every_batch():
        for i in range(n_batches):
            P.planb_lookup(h, d[offs[i]:], int(sizes[i]), out[offs[i]:])

    res = {"prefixes": len(fib), "intervals": info["intervals"], "key_bits": info["key_bits"], "depth": info["depth"],
           "fanout": rec["fanout"], "batches": n_batches, "lookups": total,
           "sizes": "log-uniform 64..4194304", "autotuned_buckets": rec["buckets"],
           "fanout_sweep": rec["fanout_sweep"]}
    ts = time_steps(every_batch, 5, 1)
    res["eager_glps"] = round(total / (sum(ts) / len(ts)) / 1e9, 3)
    check("eager")
    desc = torch.from_numpy(np.frombuffer(bytes(P.batch_array(
        [(d[offs[i]:], out[offs[i]:], int(sizes[i])) for i in range(n_batches)])), dtype=np.uint8).copy()).cuda()
    cnt = torch.tensor([n_batches], dtype=torch.int32, device="cuda")
    # launches over every batch: the shape, among the two largest buckets' picks, that runs this batch set fastest
    cands = []
    for _, tu in table[-2:]:
        if tu not in cands:
            cands.append(tu)
    shape, shape_ms = autotune.tune_batches(h, desc, cnt, n_batches, cands)
    res["persistent_shape"] = {"tuning": shape, "candidates_ms": {json.dumps(c): shape_ms[k] for k, c in enumerate(cands)}}
    ts = time_steps(lambda: P.planb_lookup_batches(h, desc, cnt, n_batches), 5, 1)
    res["persistent_glps"] = round(total / (sum(ts) / len(ts)) / 1e9, 3)
    check("persistent")
    g = P.Graph(h, n_batches)
    every = [(d[offs[i]:], out[offs[i]:], int(sizes[i])) for i in range(n_batches)]
    ts = time_steps(lambda: g.launch(every), 5, 1)
    res["graph_glps"] = round(total / (sum(ts) / len(ts)) / 1e9, 3)
    check("graph")
    g.close()
    # one batch at a time: plain launch (its bucket's shape) and a replay of a graph of its bucket's shape
    graphs = []
    for lo, tu in table:
        P.planb_set_tuning(h, **tu)
        graphs.append((lo, P.Graph(h, 1)))
    stream = torch.cuda.current_stream()
    lat = {"plain": [], "graph": []}
    for i in range(n_batches):
        a, o, m = d[offs[i]:], out[offs[i]:], int(sizes[i])
        gi = max(k for k, (lo, _) in enumerate(graphs) if lo <= m)
        for mode in ("plain", "graph", "plain", "graph"):  # the first of each is a warm-up
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            if mode == "plain":
                P.planb_lookup(h, a, m, o)
            else:
                graphs[gi][1].launch([(a, o, m)])
            stream.synchronize()
            lat[mode].append((time.perf_counter() - t1) * 1e6)
    check("one_at_a_time")
    empty = []
    for _ in range(200):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        graphs[0][1].launch([])
        stream.synchronize()
        empty.append((time.perf_counter() - t1) * 1e6)
    for _, g in graphs:
        g.close()
    bucket_of = np.searchsorted([lo for lo, _ in table], sizes, side="right") - 1
    for mode, v in lat.items():
        v = np.array(v[1::2])
        r = {"p50_us": round(float(np.percentile(v, 50)), 2), "p99_us": round(float(np.percentile(v, 99)), 2),
             "glps": round(float(total / (v.sum() / 1e6) / 1e9), 3)}
        r["p50_us_by_bucket"] = {str(table[k][0]): round(float(np.percentile(v[bucket_of == k], 50)), 2)
                                 for k in range(len(table)) if np.any(bucket_of == k)}
        res[mode] = r
    res["empty_graph_replay_p50_us"] = round(float(np.percentile(empty, 50)), 2)
    res["mismatches_vs_oracle"] = mism
    del d, desc
    torch.cuda.empty_cache()
    return res


def pcie_bandwidth(nbytes=1 << 28, reps=5):
    """Pinned host <-> device copy bandwidth (GB/s), each direction alone and
    both at once on two streams, timed with events."""
    import torch
    h_src = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
    h_dst = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
    d_a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    d_b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    res = {}
    for name, fn in (("h2d", lambda: d_a.copy_(h_src, non_blocking=True)),
                     ("d2h", lambda: h_dst.copy_(d_b, non_blocking=True))):
        ts = time_steps(fn, reps, 1)
        res[f"{name}_GBps"] = round(nbytes / (sum(ts) / len(ts)) / 1e9, 2)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        with torch.cuda.stream(s1):
            d_a.copy_(h_src, non_blocking=True)
        with torch.cuda.stream(s2):
            h_dst.copy_(d_b, non_blocking=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    res["duplex_GBps_each_way"] = round(nbytes / dt / 1e9, 2)
    del h_src, h_dst, d_a, d_b
    return res


def serving_leg(P, log_fn, n_tables=16, bursts_per_level=3000):
    """16 VRF tables behind the serving runtime, plain and learned: capacity
    (every burst at once, after an untimed warm-up pass that pays one-time
    costs such as first touches of pinned staging), then open-loop Poisson
    arrivals at 25/50/80 % of the plain capacity, the same arrival sequences
    for both modes."""
    import planb_synth as S
    from paper_2604_14650_amd import serve
    t0 = time.time()
    tabs = S.vrf_tables(n_tables, seed=5000)
    log_fn(f"serving: {n_tables} tables, {sum(len(t) for t in tabs)} prefixes ({time.time() - t0:.1f} s)")
    rng = np.random.default_rng(77)
    sizes = S.log_uniform_sizes(rng, bursts_per_level, 32, 4096)
    tids = rng.integers(0, n_tables, size=bursts_per_level)
    addrs = [S.mixed_traffic(tabs[t], int(m), 0.5, int(rng.integers(0, 2**62))) for t, m in zip(tids, sizes)]
    mean_burst = float(np.mean(sizes))
    res = {"tables": n_tables, "prefixes": int(sum(len(t) for t in tabs))}
    arrivals = {}
    for mode in ("plain", "learned"):
        srv = P.Server(max_tables=n_tables, streams=3, max_bursts=256, max_lookups=1 << 18, fanout=16, key_bits=64,
                       learned=(mode == "learned"))
        t1 = time.time()
        for k, t in enumerate(tabs):
            srv.set_table(k, t.prefixes, t.lengths, t.next_hops)
            srv.admit(k)  # builds (and, learned, trains) the table
        admit_s = time.time() - t1
        serve.replay_native(srv, np.zeros(len(sizes)), tids, addrs)
        lat, wall, outs = serve.replay_native(srv, np.zeros(len(sizes)), tids, addrs)
        # capacity: the burst list five times over, all at once, so that launches
        # overlap in steady state rather than the first launch's latency dominating
        reps = 5
        lat5, wall5, _ = serve.replay_native(srv, np.zeros(reps * len(sizes)), np.tile(tids, reps), addrs * reps)
        cap = serve.summary(lat5, np.tile(sizes, reps), wall5)
        r = {"capacity_glps": round(cap["glps"], 4), "admit_seconds": round(admit_s, 2),
             "capacity_one_pass_glps": round(serve.summary(lat, sizes, wall)["glps"], 4)}
        if mode == "plain":
            plain_outs = outs
            for load in (0.25, 0.5, 0.8):
                rate = load * cap["glps"] * 1e9 / mean_burst  # bursts per second
                arrivals[load] = np.cumsum(np.random.default_rng(int(load * 100)).exponential(1.0 / rate, size=len(sizes)))
        else:
            r["identical_to_plain"] = all(np.array_equal(a, b) for a, b in zip(outs, plain_outs))
        for load, arr in arrivals.items():
            lat, wall, _ = serve.replay_native(srv, arr, tids, addrs)
            sm = serve.summary(lat, sizes, wall)
            r[f"load_{int(load * 100)}"] = {k: round(v, 3) if isinstance(v, float) else v for k, v in sm.items()}
        r["stats"] = srv.stats()
        srv.close()
        res[mode] = r
        log_fn(f"serving {mode}: {r}")
    # zero-copy: the bursts sit in registered pinned memory (as packets in a NIC's
    # DMA buffers) and the kernels read and write them over PCIe directly
    io = serve.pinned_io(addrs)
    for mode in ("plain", "learned"):
        try:
            srv = P.Server(max_tables=n_tables, streams=3, max_bursts=256, max_lookups=1 << 18, fanout=16,
                           key_bits=64, learned=(mode == "learned"), zero_copy=True)
            for k, t in enumerate(tabs):
                srv.set_table(k, t.prefixes, t.lengths, t.next_hops)
                srv.admit(k)
            serve.replay_zero_copy(srv, np.zeros(len(sizes)), tids, io)
            reps = 5
            io5 = serve.pinned_io(addrs * reps)
            lat5, wall5, _ = serve.replay_zero_copy(srv, np.zeros(reps * len(sizes)), np.tile(tids, reps), io5)
            del io5
            lat, wall, outs = serve.replay_zero_copy(srv, np.zeros(len(sizes)), tids, io)
            r = {"capacity_glps": round(serve.summary(lat5, np.tile(sizes, reps), wall5)["glps"], 4),
                 "identical_to_plain": all(np.array_equal(a, b) for a, b in zip(outs, plain_outs))}
            for load, arr in arrivals.items():
                lat, wall, _ = serve.replay_zero_copy(srv, arr, tids, io)
                sm = serve.summary(lat, sizes, wall)
                r[f"load_{int(load * 100)}"] = {k: round(v, 3) if isinstance(v, float) else v for k, v in sm.items()}
            srv.close()
        except P.PlanbError as e:  # e.g. a platform where pinned memory is not device-addressable as it is
            r = {"error": str(e)}
        res[f"{mode}_zero_copy"] = r
        log_fn(f"serving {mode} zero-copy: {r}")
    res["capacity_glps"] = res["plain"]["capacity_glps"]
    # bursts come from host memory: 16 B of addresses cross PCIe per lookup
    # (and 2 B of next hops back), so the link, not HBM, bounds serving
    pcie = pcie_bandwidth()
    res["pcie"] = pcie
    achieved = res["capacity_glps"] * 16
    res["roofline"] = {"bound": "pcie_h2d", "achieved": round(achieved, 2), "peak": pcie["h2d_GBps"], "unit": "GB/s",
                       "frac": round(achieved / pcie["h2d_GBps"], 4), "bytes_per_lookup": 16}
    zc = res["plain_zero_copy"].get("capacity_glps")
    if zc:
        res["roofline_zero_copy"] = {"bound": "pcie_h2d", "achieved": round(zc * 16, 2), "peak": pcie["h2d_GBps"],
                                     "unit": "GB/s", "frac": round(zc * 16 / pcie["h2d_GBps"], 4),
                                     "bytes_per_lookup": 16}
    return res


def cpu_leg(fib, addrs, got):
    from oracle.trie import Trie, default_threads
    t = Trie(fib.prefixes, fib.lengths, fib.next_hops)
    thr = default_threads()
    t0 = time.perf_counter()
    want = t.lookup(addrs, thr)
    dt = time.perf_counter() - t0
    return ({"value": round(addrs.shape[0] / dt / 1e9, 5), "unit": "GLPS", "cores": thr, "kind": "oracle",
             "sample": f"the whole batch ({addrs.shape[0]} addresses), binary-trie oracle, {thr} threads, "
                       f"{dt:.1f} s"}, int((got != want).sum()), want)


def size_sweep_leg(P, log_fn, n_log=26):
    """FIBs of 25k..1M prefixes with the backbone FIB's length mix and the same
    traffic recipe: the autotuner's pick per size (fanout 8 or 16, every
    launch shape, tuned on the timed batch itself) timed on 2^n_log
    addresses, a 2^20 sample checked against the oracle's trie."""
    import dataclasses
    import torch
    import planb_synth as S
    from oracle.trie import Trie, default_threads
    from paper_2604_14650_amd import autotune
    n = 1 << n_log
    res = []
    for k in (25_000, 50_000, 100_000, 200_000, 400_000, 1_000_000):
        fib = S.make_fib(dataclasses.replace(S.BACKBONE, name=f"backbone_{k}", n_prefixes=k), 22)
        addrs = S.backbone_traffic(fib, n, seed=1022)
        d = upload(addrs)
        out = torch.empty(n, dtype=torch.int16, device="cuda")
        h, rec = autotune.tune(fib.prefixes, fib.lengths, fib.next_hops, d, n, fanouts=(8, 16),
                               cache_path=None, reps=3)
        ts = time_steps(lambda: P.planb_lookup(h, d, n, out), 10, 2)
        info = P.planb_get_info(h)
        m = 1 << 20
        P.planb_lookup(h, d, m, out)
        torch.cuda.synchronize()
        got = out[:m].cpu().numpy().view(np.uint16)
        want = Trie(fib.prefixes, fib.lengths, fib.next_hops).lookup(addrs[:m], default_threads())
        r = {"prefixes": k, "intervals": info["intervals"], "depth": info["depth"], "fanout": rec["fanout"],
             "tree_bytes": info["key_bytes"] + info["value_bytes"], "tuning": rec["tuning"],
             "glps": round(n / (sum(ts) / len(ts)) / 1e9, 2), "mismatches_2e20": int((got != want).sum())}
        log_fn(f"size sweep: {r}")
        res.append(r)
        del h, d, out
        torch.cuda.empty_cache()
    return {"addresses": n, "sizes": res}


def ablation_leg(P, fib, d, n, out, got, steps=3):
    """The design ladder on the headline FIB and batch (the GPU analogue of the
    paper's Section 4 ablation): binary search over the sorted starts, then
    the tree with one lane per lookup and no LDS, lane groups per lookup,
    LDS-staged top levels, binary search by one lane in the LDS levels, the
    bottom internal level in LDS as 32-bit key tops (the headline shape), and
    the persistent kernel replayed from a graph in the last two shapes.  Every
    rung's output is checked against the headline result."""
    import torch
    rungs = []
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, fanout=8)
    o = torch.empty_like(out)

    def timed(name, fn, note):
        o.fill_(0)
        ts = time_steps(fn, steps, 1)
        torch.cuda.synchronize()
        same = bool(np.array_equal(o.cpu().numpy().view(np.uint16), got))
        rungs.append({"rung": name, "glps": round(n / (sum(ts) / len(ts)) / 1e9, 3), "identical": same, "shape": note})
        log(f"ablation {name}: {rungs[-1]}")

    timed("sorted-array binary search", lambda: P.planb_lookup_bsearch(h, d, n, o), "one lane per lookup")
    for name, tu in (("tree, one lane per lookup, no LDS", (8, 0, 2, 512, 0)),
                     ("tree, 4 lanes per lookup, no LDS", (2, 0, 2, 512, 0)),
                     ("+ top 5 levels in LDS", (2, 5, 2, 512, 0)),
                     ("+ one-lane binary search in the LDS levels", (2, 5, 2, 512, 1)),
                     ("+ bottom internal level in LDS as 32-bit key tops (headline)", (2, 5, 2, 1024, 2))):
        P.planb_set_tuning(h, *tu)
        timed(name, lambda: P.planb_lookup(h, d, n, o), dict(zip(("keys_per_lane", "lds_levels", "lookups_per_group",
                                                                   "block_threads", "lds_search"), tu)))
    for tu, note in (((2, 5, 2, 512, 1), "whole keys in the top 5 LDS levels (lds_search 1)"),
                     ((2, 5, 2, 1024, 2), "the headline shape (key tops)")):
        P.planb_set_tuning(h, *tu)
        g = P.Graph(h, 4)
        timed("persistent kernel, graph replay, one batch", lambda: g.launch([(d, o, n)]), note)
        g.close()
    return rungs


def ipv4_leg(P, n, steps):
    """IPv4: the 1M-prefix BGP-shaped table, n 4-byte addresses (70 % inside
    prefixes, 30 % uniform) through planb_lookup_v4 (32-bit key slots).  Per
    fanout the autotuner picks the launch shape on a 2^24 sample, the whole
    batch is timed, and a 2^22 sample is checked against the oracle."""
    import torch
    import planb_synth as S
    from oracle.trie import Trie
    from paper_2604_14650_amd import autotune
    t0 = time.time()
    fib = S.make_fib(S.IPV4, 44)
    a4 = S.ipv4_traffic(fib, n, 0.7, 1044)
    log(f"ipv4: {len(fib)} prefixes, {n} addresses ({time.time() - t0:.1f} s)")
    d4 = torch.from_numpy(a4.view(np.int32)).cuda()
    sample = torch.from_numpy(S.v4_as_128(a4[:1 << 24]).view(np.int64)).cuda()
    out = torch.empty(n, dtype=torch.int16, device="cuda")
    sweep, best = {}, None
    for b in (8, 16, 32):
        h, rec = autotune.tune(fib.prefixes, fib.lengths, fib.next_hops, sample, fanouts=(b,), cache_path=None,
                               reps=3, log=log)
        ts = time_steps(lambda: P.planb_lookup_v4(h, d4, n, out), steps, 1)
        g = n / (sum(ts) / len(ts)) / 1e9
        sweep[str(b)] = round(g, 3)
        if best is None or g > best[0]:
            best = (g, b, rec["tuning"], sum(ts) / len(ts), P.planb_get_info(h))
    del sample
    g, b, tu, step_s, info = best
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, fanout=b)
    P.planb_set_tuning(h, tu["keys_per_lane"], tu["lds_levels"], tu["lookups_per_group"], tu["block_threads"],
                       tu["lds_search"])
    m = 1 << 22
    P.planb_lookup_v4(h, d4, m, out)
    torch.cuda.synchronize()
    got = out[:m].cpu().numpy().view(np.uint16)
    want = Trie(fib.prefixes, fib.lengths, fib.next_hops).lookup(S.v4_as_128(a4[:m]))
    achieved = 6 * n / step_s / 1e9  # 4-byte address in, 2-byte next hop out
    return {"glps": round(g, 3), "ms_per_step": round(step_s * 1e3, 4), "addresses": n, "prefixes": len(fib),
            "intervals": info["intervals"], "fanout": b, "key_bits": info["key_bits"], "depth": info["depth"],
            "tuning": tu, "fanout_sweep_glps": sweep,
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4), "bytes_per_lookup": 6},
            "mismatches_vs_oracle_on_2e22": int((got != want).sum())}


def rebuild_leg(P, reps=3):
    """Full rebuild of a FIB from its rules (Section 3.6 rebuilds the whole
    structure on every update; the paper reports 850 ms for 1M prefixes on
    its CPU): the host build (rules in host memory, tree uploaded) and the
    device build (rules already in device memory), median of `reps`."""
    import torch
    import planb_synth as S
    res = {}
    for name, spec, seed in (("backbone_200k", S.BACKBONE, 22), ("large_1m", S.LARGE, 33)):
        fib = S.make_fib(spec, seed)
        dp = torch.from_numpy(np.ascontiguousarray(fib.prefixes).view(np.int64)).cuda()
        dL = torch.from_numpy(np.ascontiguousarray(fib.lengths)).cuda()
        dn = torch.from_numpy(np.ascontiguousarray(fib.next_hops).view(np.int16)).cuda()
        th, td = [], []
        for r in range(reps + 1):  # the first of each is a warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            hb = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, fanout=16)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            db = P.planb_build_device(dp, dL, dn, fanout=16)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            if r:
                th.append(t1 - t0)
                td.append(t2 - t1)
            same = bool(np.array_equal(P.planb_export_image(hb), P.planb_export_image(db)))
            hb.close()
            db.close()
        res[name] = {"prefixes": len(fib), "host_ms": round(1e3 * float(np.median(th)), 2),
                     "device_ms": round(1e3 * float(np.median(td)), 2), "identical_image": same}
        log(f"rebuild {name}: {res[name]}")
    res["paper_cpu_ms_1m"] = 850
    return res


def host_cpu() -> dict:
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"model": model, "nproc": usable}


def cpu_btree_leg(fib, addrs, got, warmup=3, reps=20, single_sample=1 << 24):
    """The method on the host cores in the paper's own CPU design
    (planb_cpu_tree_*: fanout 9, 8 keys per 64-byte node, vector compare +
    popcount, batched and fully unrolled descent): 64-bit keys (the paper's
    width, exact on this FIB) and 128-bit keys, over the whole batch on every
    usable core and on one core over a 2^24-address sample; 3 warm-ups and 20
    timed repetitions each, as in the paper's measurements.  Results are
    compared with the GPU's."""
    from paper_2604_14650_amd import planb as P
    cpu = host_cpu()
    thr = cpu["nproc"]
    res = {"kind": "linearized B+-tree in the paper's CPU design (planb_cpu_tree_*: fanout 9, 8 keys per node, "
                   "vector compare + popcount, batched, unrolled)", "cpu": cpu["model"], "nproc": thr,
           "warmup": warmup, "reps": reps}
    out = np.empty(addrs.shape[0], dtype=np.uint16)
    for kb in (64, 128):
        tree = P.PaperCpuTree(fib.prefixes, fib.lengths, fib.next_hops, key_bits=kb)
        r = {"isa": tree.isa, "depth": tree.depth}
        for label, a, threads in (("all_cores", addrs, thr), ("one_core", addrs[:single_sample], 1)):
            o = out[:a.shape[0]]
            for _ in range(warmup):
                tree.lookup(a, threads, out=o)
            t0 = time.perf_counter()
            for _ in range(reps):
                tree.lookup(a, threads, out=o)
            dt = (time.perf_counter() - t0) / reps
            r[label] = {"glps": round(a.shape[0] / dt / 1e9, 4), "threads": threads, "addresses": int(a.shape[0]),
                        "mismatches_vs_gpu": int((o != got[:a.shape[0]]).sum())}
        tree.close()
        res[f"keys_{kb}"] = r
        log(f"cpu paper-design B+-tree, {kb}-bit keys: {r}")
    res["value"] = res["keys_64"]["all_cores"]["glps"]
    res["unit"] = "GLPS"
    res["cores"] = thr
    res["single_core_mlps"] = round(res["keys_64"]["one_core"]["glps"] * 1e3, 1)
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU (got --gpus {args.gpus}); across GPUs the lookup would replicate "
              "the FIB on each and split the batch between them, with no exchange", file=sys.stderr)
        sys.exit(2)
    import torch

    import planb_synth as S
    from paper_2604_14650_amd import planb as P

    n = 1 << args.addresses
    t0 = time.time()
    fib = S.make_fib(S.BACKBONE, 22)
    addrs = S.backbone_traffic(fib, n, seed=1022)
    log(f"workload: {len(fib)} prefixes, {n} addresses ({time.time() - t0:.1f} s)")
    d = upload(addrs)
    out = torch.empty(n, dtype=torch.int16, device="cuda")

    if args.copy_probe:  # a plain copy of known size, for scaling the PMC byte counters
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    t0 = time.perf_counter()
    hb = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops)
    build_s = time.perf_counter() - t0
    hb.close()

    h, tuned, ts, ts128 = plain_leg(P, fib, d, n, out, args)
    step_s = sum(ts) / len(ts)
    glps = n / step_s / 1e9
    glps128 = n / (sum(ts128) / len(ts128)) / 1e9
    info = P.planb_get_info(h)
    achieved = BYTES_PER_LOOKUP * n / step_s / 1e9
    P.planb_lookup(h, d, n, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint16).copy()
    tu = P.planb_get_tuning(h)
    kconf = (f"fanout={info['fanout']} key_bits={info['key_bits']} keys_per_lane={tu['keys_per_lane']} "
             f"lds_levels={tu['lds_levels']} lookups_per_group={tu['lookups_per_group']} "
             f"block_threads={tu['block_threads']} lds_search={tu['lds_search']}")
    traffic = measured_traffic(n, kconf)
    prof_ns = profiled_kernel_ns(n, kconf)

    result = {
        "metric": METRIC, "value": round(glps, 3), "unit": "GLPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(step_s * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "backbone-shaped FIB of 200,000 prefixes; 2^%d destination addresses "
                               "(70%% inside prefixes, 30%% uniform in 2000::/3)" % args.addresses,
                   "fib_prefixes": len(fib), "intervals": info["intervals"], "addresses": n,
                   "fanout": info["fanout"], "key_bits": info["key_bits"], "depth": info["depth"],
                   "tuning": P.planb_get_tuning(h),
                   "autotuned": tuned[0].get("autotuned"),
                   "tree_bytes": info["key_bytes"] + info["value_bytes"],
                   "build_seconds": round(build_s, 3)},
        "plain_128bit_keys": {"glps": round(glps128, 3), "fanout": tuned[128]["fanout"],
                              "tuning": tuned[128]["tuning"], "autotuned": tuned[128].get("autotuned")},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic / step_s / 1e9, 1),
                     # achieved and frac come from this run's HIP events (the mean step);
                     # the committed kernel-trace summary's average kernel time is shown beside them
                     "source": "hip events over the timed steps",
                     "profiled_ms_per_launch": None if prof_ns is None else round(prof_ns / 1e6, 4),
                     "frac_profiled": None if prof_ns is None else
                     round(BYTES_PER_LOOKUP * n / (prof_ns * 1e-9) / 1e9 / HBM_PEAK_GBS, 4)},
        "paper_cpu_context": {"single_core_mlps": 390, "all_core_blps": 3.4,
                              "cpu": "AMD Ryzen 9 370HX, 12 cores (paper's figures, 64-bit keys, real FIBs)"},
    }
    if traffic is not None:
        result["roofline"]["traffic_bytes_per_launch"] = int(traffic)
    log(f"plain: {glps:.2f} GLPS ({info})")
    if args.size_sweep:
        result["size_sweep"] = size_sweep_leg(P, log)
    learned_out = []  # the learned lookup's results on the headline batch, for the oracle's check
    if not args.quick:
        if not args.skip_learned:
            result["learned"] = learned_leg(P, fib, d, n, out, args, keep=learned_out)
        if not args.skip_ablation:
            result["ablation"] = ablation_leg(P, fib, d, n, out, got)
        if not args.skip_rebuild:
            result["rebuild"] = rebuild_leg(P)
        if not args.skip_batches:
            result["batch_latency"] = batches_leg(P, h, d, n, out)
            log(f"batches: {result['batch_latency']}")
        del d  # the IPv6 batch is no longer needed on the device
        torch.cuda.empty_cache()
        if not args.skip_uneven:
            result["uneven_batches"] = uneven_leg(P, log)
            # batch latency as a user would submit: one plain launch per batch, enqueue to completion
            result["p99_batch_latency_us"] = result["uneven_batches"]["plain"]["p99_us"]
            result["p50_batch_latency_us"] = result["uneven_batches"]["plain"]["p50_us"]
            log(f"uneven batches: {result['uneven_batches']}")
        if not args.skip_ipv4:
            result["ipv4"] = ipv4_leg(P, n, max(3, args.steps // 2))
            log(f"ipv4: {result['ipv4']}")
        if not args.skip_serving:
            result["serving"] = serving_leg(P, log)
            log(f"serving: {result['serving']}")
    if not args.no_cpu_baseline:
        cb, mism, want = cpu_leg(fib, addrs, got)
        result["cpu_baseline"] = cb
        result["mismatches_vs_oracle"] = mism
        if learned_out:  # the learned lookup's results on the same batch, against the oracle's
            result["learned"]["backbone"]["mismatches_vs_oracle"] = int((learned_out[0] != want).sum())
        del want, learned_out[:]
        result["cpu_btree_baseline"] = cpu_btree_leg(fib, addrs, got)
        log(f"cpu B+-tree: {result['cpu_btree_baseline']}")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
