"""Shared test helpers: device transfer and seeded workloads (no method arithmetic)."""
from __future__ import annotations

import functools
import sys

import numpy as np

import planb_synth as S


def say(*a):
    """Print and flush: names the case before each GPU step."""
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(addrs: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(addrs).view(np.int64)).cuda()


def out_u16(n: int):
    import torch
    return torch.full((max(n, 1),), -1, dtype=torch.int16, device="cuda")


def host_u16(t, n: int) -> np.ndarray:
    return t[:n].cpu().numpy().view(np.uint16)


@functools.lru_cache(maxsize=None)
def fib_of(kind: str, seed: int):
    spec = {"tiny": S.TINY, "backbone": S.BACKBONE, "large": S.LARGE}[kind]
    return S.make_fib(spec, seed)


@functools.lru_cache(maxsize=None)
def oracle_trie(kind: str, seed: int):
    from oracle.trie import Trie
    f = fib_of(kind, seed)
    return Trie(f.prefixes, f.lengths, f.next_hops)
