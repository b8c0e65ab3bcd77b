"""Autotuner: picks the fanout (a build parameter) and the lookup tuning.

For each fanout it builds the FIB and lets the native planb_autotune time
every compiled-in launch shape on a device-resident sample; the fastest
(fanout, tuning) wins.  ``tune_sizes`` does the same per batch-size bucket
(native planb_autotune_sizes): the fanout with the least summed time over the
buckets' sizes wins, and its per-bucket launch shapes are installed on the
handle.  Results are cached in a JSON file keyed by a hash of the FIB, the key
width requested and the sample's size bucket (log2) or the bucket sizes, so a
rerun on the same FIB skips the trials.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np

from . import planb as P

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "planb", "autotune.json")


def fib_fingerprint(prefixes, lengths, next_hops) -> str:
    h = hashlib.sha1()
    for a in (prefixes, lengths, next_hops):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:16]


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(path, data):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(prefixes, lengths, next_hops, sample, n: int | None = None, fanouts=(8, 16, 32), key_bits: int = 0,
         cache_path: str | None = DEFAULT_CACHE, reps: int = 3, log=None):
    """Returns (fib handle with the best tuning applied, record dict)."""
    n = sample.shape[0] if n is None else n
    key = f"{fib_fingerprint(prefixes, lengths, next_hops)}:k{key_bits}:n{max(n, 1).bit_length()}:" \
          f"f{','.join(map(str, fanouts))}"
    cache = _load(cache_path) if cache_path else {}
    rec = cache.get(key)
    if rec:
        h = P.planb_build(prefixes, lengths, next_hops, fanout=rec["fanout"], key_bits=key_bits)
        t = rec["tuning"]
        P.planb_set_tuning(h, t["keys_per_lane"], t["lds_levels"], t["lookups_per_group"], t["block_threads"],
                           t.get("lds_search", 0))
        return h, dict(rec, cached=True)
    best = None
    trials = {}
    t0 = time.time()
    for b in fanouts:
        h = P.planb_build(prefixes, lengths, next_hops, fanout=b, key_bits=key_bits)
        r = P.planb_autotune(h, sample, n, reps)
        trials[str(b)] = round(r["glps"], 3)
        if log:
            log(f"autotune fanout {b}: {r}")
        if best is None or r["glps"] > best[1]["glps"]:
            if best is not None:
                best[0].close()
            best = (h, r, b)
        else:
            h.close()
    h, r, b = best
    rec = {"fanout": b, "key_bits": P.planb_get_info(h)["key_bits"],
           "tuning": {k: r[k] for k in ("keys_per_lane", "lds_levels", "lookups_per_group", "block_threads",
                                        "lds_search")},
           "glps": round(r["glps"], 3), "fanout_glps": trials, "sample": n,
           "seconds": round(time.time() - t0, 2)}
    if cache_path:
        cache = _load(cache_path)
        cache[key] = rec
        _save(cache_path, cache)
    return h, dict(rec, cached=False)


def tune_sizes(prefixes, lengths, next_hops, sample, sizes, fanouts=(8, 16, 32), key_bits: int = 0,
               cache_path: str | None = DEFAULT_CACHE, reps: int = 3, log=None):
    """Per batch-size bucket launch shapes.  Returns (fib handle whose size
    tunings are installed, record dict with the fanout and per-bucket picks)."""
    sizes = [int(x) for x in sizes]
    key = f"{fib_fingerprint(prefixes, lengths, next_hops)}:k{key_bits}:sizes{','.join(map(str, sizes))}:" \
          f"f{','.join(map(str, fanouts))}"
    cache = _load(cache_path) if cache_path else {}
    rec = cache.get(key)
    if rec:
        h = P.planb_build(prefixes, lengths, next_hops, fanout=rec["fanout"], key_bits=key_bits)
        P.planb_set_size_tunings(h, [(e["min_lookups"], e["tuning"]) for e in rec["buckets"]])
        return h, dict(rec, cached=True)
    best = None
    sweep = {}
    t0 = time.time()
    for b in fanouts:
        h = P.planb_build(prefixes, lengths, next_hops, fanout=b, key_bits=key_bits)
        res = P.planb_autotune_sizes(h, sample, sizes, reps)
        total_ms = sum(r["ms_per_call"] for r in res)
        sweep[str(b)] = {"total_ms": round(total_ms, 4), "glps": [round(r["glps"], 3) for r in res]}
        if log:
            log(f"autotune sizes fanout {b}: {sweep[str(b)]}")
        if best is None or total_ms < best[1]:
            if best is not None:
                best[0].close()
            best = (h, total_ms, b, res)
        else:
            h.close()
    h, total_ms, b, res = best
    table = P.planb_get_size_tunings(h)
    rec = {"fanout": b, "key_bits": P.planb_get_info(h)["key_bits"],
           "buckets": [{"size": sizes[i], "min_lookups": table[i][0], "tuning": table[i][1],
                        "glps": round(res[i]["glps"], 3)} for i in range(len(sizes))],
           "fanout_sweep": sweep, "seconds": round(time.time() - t0, 2)}
    if cache_path:
        cache = _load(cache_path)
        cache[key] = rec
        _save(cache_path, cache)
    return h, dict(rec, cached=False)


def tune_batches(h, batches, n_batches, max_batches: int, candidates, reps: int = 2, stream=None):
    """The launch shape for persistent multi-batch launches (planb_lookup_batches
    and the graphs built on the handle afterwards): each candidate tuning is
    timed on the caller's own batch set (one warm-up, then `reps` launches,
    HIP events on `stream`) and the fastest is applied.  Returns (tuning,
    {candidate index: ms per launch}).  The shape that wins one batch size
    need not win a launch over many uneven batches, where the tiles of every
    batch share the grid."""
    import torch
    stream = torch.cuda.current_stream() if stream is None else stream
    times = {}
    best = None
    for k, tu in enumerate(candidates):
        P.planb_set_tuning(h, **tu)
        P.planb_lookup_batches(h, batches, n_batches, max_batches, stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            P.planb_lookup_batches(h, batches, n_batches, max_batches, stream)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        times[k] = round(ms, 4)
        if best is None or ms < best[0]:
            best = (ms, tu)
    P.planb_set_tuning(h, **best[1])
    return best[1], times
