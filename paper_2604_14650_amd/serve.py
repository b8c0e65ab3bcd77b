"""Serving driver: replays burst arrivals against the native server
(planb_server_*) and reports latency percentiles and throughput.

The server does admission, continuous batching, streams and completion
tracking; this module only feeds it arrivals at their scheduled times (an open
loop: a burst's latency runs from its scheduled arrival to the moment the
server reports it complete, so time spent queued behind a slow driver or a
busy GPU counts) and summarises the completions.
"""
from __future__ import annotations

import numpy as np

from . import planb as P


def replay(server: "P.Server", arrivals_s, tables, addrs, outs, timeout_s: float = 120.0):
    """arrivals_s: sorted arrival offsets (seconds); tables / addrs / outs per
    burst.  Returns per-burst latencies (microseconds) and the wall time."""
    n = len(arrivals_s)
    lat = np.zeros(n)
    t0 = P.planb_server_now_us() + 1000.0  # start 1 ms from now
    sched = t0 + np.asarray(arrivals_s) * 1e6
    nxt = 0
    done = 0
    while done < n:
        now = P.planb_server_now_us()
        while nxt < n and sched[nxt] <= now:
            server.submit(int(tables[nxt]), addrs[nxt], outs[nxt], nxt)
            nxt += 1
        for tag, _, _, _, done_us, _ in server.poll(block=(nxt == n)):
            lat[tag] = done_us - sched[tag]
            done += 1
        if now - t0 > timeout_s * 1e6:
            raise TimeoutError(f"serving replay did not finish: {done} of {n} bursts done")
    wall = (P.planb_server_now_us() - t0) / 1e6
    return lat, wall


def replay_native(server: "P.Server", arrivals_s, tables, addrs_list):
    """The same open-loop replay run by the native planb_server_replay (no
    Python in the submit/poll loop).  Returns (latency_us, wall_s, outputs)."""
    sizes = np.array([len(a) for a in addrs_list], dtype=np.uint64)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    flat = np.concatenate(addrs_list) if len(addrs_list) else np.zeros((0, 2), np.uint64)
    out = np.zeros(max(1, flat.shape[0]), dtype=np.uint16)
    lat, wall = server.replay(np.asarray(arrivals_s) * 1e6, tables, offsets, flat, out)
    return lat, wall, [out[offsets[k]:offsets[k + 1]] for k in range(len(addrs_list))]


def pinned_io(addrs_list):
    """The bursts' addresses gathered once into pinned host memory (as packets
    sit in a NIC's DMA buffers) with a pinned output area: (offsets, addrs
    tensor, out tensor), both to be registered with a zero-copy server."""
    import torch
    sizes = np.array([len(a) for a in addrs_list], dtype=np.uint64)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    total = max(1, int(offsets[-1]))
    a = torch.empty((total, 2), dtype=torch.int64, pin_memory=True)
    if len(addrs_list):
        a.numpy()[:int(offsets[-1])] = np.concatenate(addrs_list).view(np.int64)
    out = torch.zeros(total, dtype=torch.int16, pin_memory=True)
    return offsets, a, out


def replay_zero_copy(server: "P.Server", arrivals_s, tables, io):
    """replay_native for a zero-copy server over pinned_io buffers (registered
    here once per server).  Returns (latency_us, wall_s, outputs)."""
    offsets, a, out = io
    key = (a.data_ptr(), out.data_ptr())
    if key not in getattr(server, "_io_registered", set()):
        server.register_io(a.data_ptr(), a.numel() * 8)
        server.register_io(out.data_ptr(), out.numel() * 2)
        server._io_registered = getattr(server, "_io_registered", set()) | {key}
    lat, wall = server.replay_raw(np.asarray(arrivals_s) * 1e6, tables, offsets, a.data_ptr(), out.data_ptr())
    o = out.numpy().view(np.uint16)
    return lat, wall, [o[int(offsets[k]):int(offsets[k + 1])].copy() for k in range(len(offsets) - 1)]


def summary(lat_us, sizes, wall_s) -> dict:
    return {"bursts": int(len(lat_us)), "lookups": int(np.sum(sizes)),
            "p50_us": float(np.percentile(lat_us, 50)), "p99_us": float(np.percentile(lat_us, 99)),
            "mean_us": float(np.mean(lat_us)), "glps": float(np.sum(sizes) / wall_s / 1e9), "seconds": wall_s}
