"""The C ABI from a C99 program with no Python between (tests/c_abi_client.c,
built by __graft_entry__.build()): reading raw rule and address files, it
resolves every address through include/planb.h alone.  Its next hops equal
the oracle's: host-only calls (planb_build_intervals, planb_build_image,
planb_cpu_lookup) on the CPU, planb_build and planb_lookup on a HIP stream of
its own on the GPU."""
import os
import subprocess

import numpy as np
import pytest

import planb_synth as S
from helpers import fib_of, oracle_trie, say

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "c_abi_client")


def run_client(mode, prefixes, lengths, hops, addrs, tmp_path):
    assert os.path.exists(EXE), "tests/c_abi_client is missing: run __graft_entry__.build() first"
    paths = []
    for name, arr, dt in (("prefixes", prefixes, np.uint64), ("lengths", lengths, np.uint8),
                          ("hops", hops, np.uint16), ("addrs", addrs, np.uint64)):
        p = str(tmp_path / f"{name}.bin")
        np.ascontiguousarray(arr, dtype=dt).tofile(p)
        paths.append(p)
    out = str(tmp_path / "out.bin")
    r = subprocess.run([EXE, mode, *paths, out], capture_output=True, text=True, timeout=120)
    say(r.stdout.strip() or r.stderr.strip())
    assert r.returncode == 0, r.stderr
    got = np.fromfile(out, dtype=np.uint16)
    assert got.shape[0] == addrs.shape[0]
    return got


def test_c_client_host_only_matches_oracle(tmp_path):
    fib = fib_of("tiny", 11)
    addrs = S.tiny_traffic(fib, 1 << 16, seed=1011)
    got = run_client("host", fib.prefixes, fib.lengths, fib.next_hops, addrs, tmp_path)
    assert np.array_equal(got, oracle_trie("tiny", 11).lookup(addrs))


def test_c_client_empty_rule_set(tmp_path):
    """No rules: every address resolves to PLANB_NO_ROUTE."""
    addrs = np.array([[0, 0], [0x2001_0db8_0000_0000, 1], [2**64 - 1, 2**64 - 1]], dtype=np.uint64)
    got = run_client("host", np.zeros((0, 2), np.uint64), np.zeros(0, np.uint8), np.zeros(0, np.uint16), addrs,
                     tmp_path)
    assert np.all(got == 0xFFFF)


def test_c_client_reports_a_refused_rule_set(tmp_path):
    """A rule whose next hop is the reserved 0xFFFF: the client exits non-zero
    with the library's message."""
    fib = fib_of("tiny", 11)
    hops = fib.next_hops.copy()
    hops[3] = 0xFFFF
    paths = []
    for name, arr, dt in (("prefixes", fib.prefixes, np.uint64), ("lengths", fib.lengths, np.uint8),
                          ("hops", hops, np.uint16), ("addrs", np.zeros((4, 2)), np.uint64)):
        p = str(tmp_path / f"{name}.bin")
        np.ascontiguousarray(arr, dtype=dt).tofile(p)
        paths.append(p)
    r = subprocess.run([EXE, "host", *paths, str(tmp_path / "out.bin")], capture_output=True, text=True, timeout=60)
    assert r.returncode != 0 and "planb_build_intervals" in r.stderr


@pytest.mark.gpu
@pytest.mark.parametrize("kind,seed,n", [("tiny", 11, 1 << 16), ("backbone", 22, 1 << 20)])
def test_c_client_gpu_matches_oracle(tmp_path, kind, seed, n):
    fib = fib_of(kind, seed)
    addrs = S.tiny_traffic(fib, n, seed=1011) if kind == "tiny" else S.backbone_traffic(fib, n, seed=2023)
    got = run_client("gpu", fib.prefixes, fib.lengths, fib.next_hops, addrs, tmp_path)
    assert np.array_equal(got, oracle_trie(kind, seed).lookup(addrs))
