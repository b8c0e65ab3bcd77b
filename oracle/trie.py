"""ctypes wrapper of the C binary-trie oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle_trie.so")
SRC_PATH = os.path.join(_HERE, "trie.c")


def build_oracle() -> str:
    """Compile trie.c with gcc into liboracle_trie.so (always recompiles)."""
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                           "-o", LIB_PATH + ".tmp", SRC_PATH])
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build_oracle()
        lib = ctypes.CDLL(LIB_PATH)
        lib.oracle_trie_new.restype = ctypes.c_void_p
        lib.oracle_trie_new.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]
        lib.oracle_trie_free.argtypes = [ctypes.c_void_p]
        lib.oracle_trie_nodes.restype = ctypes.c_size_t
        lib.oracle_trie_nodes.argtypes = [ctypes.c_void_p]
        lib.oracle_trie_lookup.restype = ctypes.c_int
        lib.oracle_trie_lookup.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                           ctypes.c_void_p, ctypes.c_int]
        _lib = lib
    return _lib


def default_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


class Trie:
    def __init__(self, prefixes, lengths, next_hops):
        lib = _load()
        self._p = np.ascontiguousarray(prefixes, dtype=np.uint64)
        L = np.ascontiguousarray(lengths, dtype=np.uint8)
        nh = np.ascontiguousarray(next_hops, dtype=np.uint16)
        n = L.shape[0]
        self._h = lib.oracle_trie_new(self._p.ctypes.data if n else None,
                                      L.ctypes.data if n else None,
                                      nh.ctypes.data if n else None, n)
        if not self._h:
            raise ValueError("oracle trie: bad rule length or out of memory")

    @property
    def nodes(self) -> int:
        return int(_load().oracle_trie_nodes(self._h))

    def lookup(self, addrs, nthreads: int | None = None) -> np.ndarray:
        a = np.ascontiguousarray(addrs, dtype=np.uint64)
        out = np.empty(a.shape[0], dtype=np.uint16)
        if a.shape[0] == 0:
            return out
        rc = _load().oracle_trie_lookup(self._h, a.ctypes.data, a.shape[0], out.ctypes.data,
                                        nthreads or default_threads())
        if rc != 0:
            raise RuntimeError("oracle trie lookup failed")
        return out

    def close(self):
        if getattr(self, "_h", None):
            _load().oracle_trie_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lpm_trie(prefixes, lengths, next_hops, addrs, nthreads=None) -> np.ndarray:
    t = Trie(prefixes, lengths, next_hops)
    try:
        return t.lookup(addrs, nthreads)
    finally:
        t.close()
