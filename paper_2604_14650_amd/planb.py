"""Thin ctypes binding of ``libplanb.so`` (include/planb.h), same names as the C ABI.

Argument marshalling only: every step of building and searching runs in the
native library (host C++ for the build, HIP kernels for lookups).  PyTorch is
used for device memory (``torch.Tensor.data_ptr()``) and streams
(``torch.cuda.current_stream().cuda_stream``).  There is no fallback: if the
library is missing this module raises at import.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libplanb.so")

PLANB_OK = 0
PLANB_EINVAL = -1
PLANB_EDUP = -2
PLANB_ENOMEM = -3
PLANB_EDEVICE = -4
PLANB_ERANGE = -5
PLANB_NO_ROUTE = 0xFFFF
PLANB_FLAG_MERGE_EQUAL_NH = 1
PLANB_MAX_LEVELS = 16
PLANB_SERVER_ZERO_COPY = 1

# torch bundles its own libamdhip64.so.7.  Loading torch first makes the
# dynamic linker resolve this library's libamdhip64.so.7 to that same, already
# loaded runtime, so torch's device pointers and stream handles are valid here.
import torch  # noqa: E402,F401

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                      "(or python paper_2604_14650_amd/build.py) first")

_lib = ctypes.CDLL(LIB_PATH)


class planb_params_t(ctypes.Structure):
    _fields_ = [("fanout", ctypes.c_uint32), ("keys_per_lane", ctypes.c_uint32),
                ("lds_levels", ctypes.c_int32), ("flags", ctypes.c_uint32), ("key_bits", ctypes.c_uint32)]


class planb_tuning_t(ctypes.Structure):
    _fields_ = [("keys_per_lane", ctypes.c_uint32), ("lds_levels", ctypes.c_int32),
                ("lookups_per_group", ctypes.c_uint32), ("block_threads", ctypes.c_uint32),
                ("lds_search", ctypes.c_uint32)]


class planb_info_t(ctypes.Structure):
    _fields_ = [("intervals", ctypes.c_uint64), ("fanout", ctypes.c_uint32), ("slots", ctypes.c_uint32),
                ("depth", ctypes.c_uint32), ("key_bits", ctypes.c_uint32),
                ("level_nodes", ctypes.c_uint64 * PLANB_MAX_LEVELS),
                ("level_offset", ctypes.c_uint64 * (PLANB_MAX_LEVELS + 1)),
                ("key_bytes", ctypes.c_uint64), ("value_bytes", ctypes.c_uint64),
                ("leaf_keys", ctypes.c_uint32), ("leaf_slots", ctypes.c_uint32), ("leaf_base", ctypes.c_uint64)]


class planb_batch_t(ctypes.Structure):
    _fields_ = [("addrs", ctypes.c_void_p), ("out", ctypes.c_void_p), ("n", ctypes.c_uint64)]


class planb_autotune_result_t(ctypes.Structure):
    _fields_ = [("tuning", planb_tuning_t), ("ms_per_call", ctypes.c_float), ("glps", ctypes.c_float),
                ("candidates", ctypes.c_uint32)]


class planb_train_cfg_t(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_uint32), ("batch", ctypes.c_uint32), ("lr", ctypes.c_float),
                ("segments", ctypes.c_uint32), ("seed", ctypes.c_uint64)]


class planb_train_report_t(ctypes.Structure):
    _fields_ = [("final_loss", ctypes.c_float), ("steps", ctypes.c_uint32), ("seconds", ctypes.c_float),
                ("max_eps", ctypes.c_uint32), ("mean_eps", ctypes.c_float), ("empty_segments", ctypes.c_uint32)]


class planb_burst_t(ctypes.Structure):
    _fields_ = [("table", ctypes.c_uint32), ("n", ctypes.c_uint32), ("addrs", ctypes.c_void_p),
                ("out", ctypes.c_void_p)]


class planb_server_cfg_t(ctypes.Structure):
    _fields_ = [("max_tables", ctypes.c_uint32), ("streams", ctypes.c_uint32), ("max_bursts", ctypes.c_uint32),
                ("max_lookups", ctypes.c_uint32), ("fanout", ctypes.c_uint32), ("key_bits", ctypes.c_uint32),
                ("memory_budget", ctypes.c_uint64), ("learned", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class planb_completion_t(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_int64), ("table", ctypes.c_uint32), ("n", ctypes.c_uint32),
                ("submit_us", ctypes.c_double), ("done_us", ctypes.c_double), ("status", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class planb_server_stats_t(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_uint64), ("bursts", ctypes.c_uint64), ("lookups", ctypes.c_uint64),
                ("admissions", ctypes.c_uint64), ("evictions", ctypes.c_uint64), ("resident_bytes", ctypes.c_uint64),
                ("resident_tables", ctypes.c_uint32), ("queued", ctypes.c_uint32)]


_vp = ctypes.c_void_p
_sz = ctypes.c_size_t


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_sig("planb_build", _vp, _vp, _vp, _vp, _sz)
_sig("planb_build_ex", _vp, _vp, _vp, _vp, _sz, ctypes.POINTER(planb_params_t))
_sig("planb_build_device", _vp, _vp, _vp, _vp, _sz, ctypes.POINTER(planb_params_t), _vp)
_sig("planb_lookup", ctypes.c_int, _vp, _vp, _sz, _vp, _vp)
_sig("planb_lookup_index", ctypes.c_int, _vp, _vp, _sz, _vp, _vp)
_sig("planb_lookup_bsearch", ctypes.c_int, _vp, _vp, _sz, _vp, _vp)
_sig("planb_lookup_v4", ctypes.c_int, _vp, _vp, _sz, _vp, _vp)
_sig("planb_free", None, _vp)
_sig("planb_last_error", ctypes.c_char_p)
_sig("planb_last_status", ctypes.c_int)
_sig("planb_num_intervals", _sz, _vp)
_sig("planb_export_intervals", ctypes.c_longlong, _vp, _vp, _vp, _sz)
_sig("planb_get_info", ctypes.c_int, _vp, ctypes.POINTER(planb_info_t))
_sig("planb_set_tuning", ctypes.c_int, _vp, ctypes.POINTER(planb_tuning_t))
_sig("planb_get_tuning", ctypes.c_int, _vp, ctypes.POINTER(planb_tuning_t))
_sig("planb_build_intervals", ctypes.c_longlong, _vp, _vp, _vp, _sz, ctypes.c_uint32, _vp, _vp, _sz)
_sig("planb_build_keys", ctypes.c_longlong, _vp, _sz, ctypes.c_uint32, _vp, _sz, ctypes.POINTER(planb_info_t))
_sig("planb_cpu_lookup", ctypes.c_int, _vp, ctypes.POINTER(planb_info_t), _vp, _sz, _vp, ctypes.c_int)
_sig("planb_export_image", ctypes.c_longlong, _vp, _vp, _sz)
_sig("planb_build_image", ctypes.c_longlong, _vp, _vp, _sz, ctypes.c_uint32, ctypes.c_uint32, _vp, _sz,
     ctypes.POINTER(planb_info_t))
_sig("planb_lookup_batches", ctypes.c_int, _vp, _vp, _vp, ctypes.c_uint32, _vp)
_sig("planb_graph_create", _vp, _vp, ctypes.c_uint32)
_sig("planb_graph_launch", ctypes.c_int, _vp, _vp, ctypes.c_uint32, _vp)
_sig("planb_graph_free", None, _vp)
_sig("planb_autotune", ctypes.c_int, _vp, _vp, _sz, ctypes.c_uint32, _vp, ctypes.POINTER(planb_autotune_result_t))
_sig("planb_set_size_tunings", ctypes.c_int, _vp, _vp, _vp, ctypes.c_uint32)
_sig("planb_get_size_tunings", ctypes.c_int, _vp, _vp, _vp, ctypes.c_uint32)
_sig("planb_autotune_sizes", ctypes.c_int, _vp, _vp, _sz, _vp, ctypes.c_uint32, ctypes.c_uint32, _vp,
     _vp)
_sig("planb_train", ctypes.c_int, _vp, ctypes.POINTER(planb_train_cfg_t), _vp, ctypes.POINTER(planb_train_report_t))
_sig("planb_lookup_learned", ctypes.c_int, _vp, _vp, _sz, _vp, _vp, _vp)
_sig("planb_lookup_learned_noalloc", ctypes.c_int, _vp, _vp, _sz, _vp, _vp, _vp)
_sig("planb_model_num_params", ctypes.c_int)
_sig("planb_model_set_params", ctypes.c_int, _vp, _vp, ctypes.c_uint32)
_sig("planb_model_get_params", ctypes.c_int, _vp, _vp)
_sig("planb_model_predict", ctypes.c_int, _vp, _vp, _sz, _vp, _vp)
_sig("planb_model_grad", ctypes.c_int, _vp, _vp, _vp, _sz, _vp, _vp)
_sig("planb_model_adam", ctypes.c_int, _vp, _vp, ctypes.c_float, _vp)
_sig("planb_model_build_eps", ctypes.c_int, _vp, _vp)
_sig("planb_model_get_eps", ctypes.c_int, _vp, _vp, ctypes.c_uint32)
_sig("planb_model_set_eps", ctypes.c_int, _vp, _vp, ctypes.c_uint32)
_sig("planb_tableset_create", _vp, ctypes.c_uint32)
_sig("planb_tableset_set", ctypes.c_int, _vp, ctypes.c_uint32, _vp)
_sig("planb_tableset_set_tuning", ctypes.c_int, _vp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32)
_sig("planb_lookup_multi", ctypes.c_int, _vp, _vp, _vp, ctypes.c_uint32, _vp)
_sig("planb_lookup_multi_learned", ctypes.c_int, _vp, _vp, _vp, ctypes.c_uint32, _vp, _vp)
_sig("planb_tableset_free", None, _vp)
_sig("planb_server_create", _vp, ctypes.POINTER(planb_server_cfg_t))
_sig("planb_server_register_io", ctypes.c_int, _vp, _vp, _sz)
_sig("planb_server_free", None, _vp)
_sig("planb_server_set_table", ctypes.c_int, _vp, ctypes.c_uint32, _vp, _vp, _vp, _sz)
_sig("planb_server_submit", ctypes.c_int, _vp, ctypes.c_uint32, _vp, ctypes.c_uint32, _vp, ctypes.c_int64)
_sig("planb_server_poll", ctypes.c_int, _vp, ctypes.POINTER(planb_completion_t), ctypes.c_uint32, ctypes.c_int)
_sig("planb_server_stats", ctypes.c_int, _vp, ctypes.POINTER(planb_server_stats_t))
_sig("planb_server_now_us", ctypes.c_double)
_sig("planb_server_admit", ctypes.c_int, _vp, ctypes.c_uint32)
_sig("planb_server_replay", ctypes.c_int, _vp, ctypes.c_uint32, _vp, _vp, _vp, _vp, _vp, _vp,
     ctypes.POINTER(ctypes.c_double))
_sig("planb_layout", ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
     ctypes.POINTER(planb_info_t))


class PlanbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"planb error {code}: {msg}")
        self.code = code


def planb_last_error() -> str:
    return (_lib.planb_last_error() or b"").decode()


def _check(rc: int) -> int:
    if rc < 0:
        raise PlanbError(rc, planb_last_error())
    return rc


def lib_handle():
    return _lib


class Fib:
    """Owner of one ``planb_fib_t*``; frees it when garbage-collected."""

    def __init__(self, ptr: int):
        self.ptr = ptr

    def close(self):
        if self.ptr:
            _lib.planb_free(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def _as_parameter_(self):
        if not self.ptr:
            raise ValueError("FIB handle already freed")
        return ctypes.c_void_p(self.ptr)


def _host(a, dtype, shape_tail=()):
    a = np.ascontiguousarray(a, dtype=dtype)
    if shape_tail and a.shape[1:] != shape_tail:
        raise ValueError(f"expected shape (n, {shape_tail}), got {a.shape}")
    return a


def planb_last_status() -> int:
    return int(_lib.planb_last_status())


def planb_build(prefixes, lengths, next_hops, fanout: int = 16, keys_per_lane: int = 0,
                lds_levels: int = 0, flags: int = 0, key_bits: int = 0) -> Fib:
    """prefixes: (n, 2) uint64 {hi, lo}; lengths: (n,) uint8; next_hops: (n,) uint16."""
    p = _host(prefixes, np.uint64, (2,)) if len(lengths) else np.zeros((0, 2), np.uint64)
    L = _host(lengths, np.uint8)
    nh = _host(next_hops, np.uint16)
    if not (p.shape[0] == L.shape[0] == nh.shape[0]):
        raise ValueError("prefixes, lengths and next_hops differ in length")
    params = planb_params_t(fanout, keys_per_lane, lds_levels, flags, key_bits)
    n = L.shape[0]
    ptr = _lib.planb_build_ex(p.ctypes.data if n else None, L.ctypes.data if n else None,
                              nh.ctypes.data if n else None, n, ctypes.byref(params))
    if not ptr:
        raise PlanbError(planb_last_status(), planb_last_error())
    return Fib(ptr)


def planb_build_device(prefixes, lengths, next_hops, n: int | None = None, fanout: int = 16, keys_per_lane: int = 0,
                       lds_levels: int = 0, flags: int = 0, key_bits: int = 0, stream=None) -> Fib:
    """Device-side build: prefixes (n, 2) int64, lengths (n,) uint8 and
    next_hops (n,) int16/uint16 are device tensors (or device pointers with n)."""
    if n is None:
        n = lengths.shape[0]
    params = planb_params_t(fanout, keys_per_lane, lds_levels, flags, key_bits)
    ptr = _lib.planb_build_device(_dev_ptr(prefixes, "prefixes") if n else None,
                                  _dev_ptr(lengths, "lengths") if n else None,
                                  _dev_ptr(next_hops, "next_hops") if n else None, n, ctypes.byref(params),
                                  _stream_handle(stream))
    if not ptr:
        raise PlanbError(planb_last_status(), planb_last_error())
    return Fib(ptr)


def _stream_handle(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dev_ptr(t, what):
    if hasattr(t, "data_ptr"):
        if not t.is_cuda:
            raise ValueError(f"{what} must be a device tensor")
        if not t.is_contiguous():
            raise ValueError(f"{what} must be contiguous")
        return t.data_ptr()
    return int(t)


def _records(t) -> int | None:
    """Records a tensor holds (None for a raw pointer)."""
    if not hasattr(t, "data_ptr"):
        return None
    return t.shape[0] if t.dim() > 0 else 0


def _check_io(addrs, out, n, rec_bytes: int, out_bytes: int, what: str = "out"):
    """When tensors are passed, n must fit both of them and their element
    layout must be the one the C call reads and writes; raw pointers are the
    caller's responsibility."""
    if n is None:
        if not hasattr(addrs, "data_ptr"):
            raise ValueError("n is required when addrs is a raw pointer")
        n = addrs.shape[0]
    if n < 0:
        raise ValueError("n must be >= 0")
    if hasattr(addrs, "data_ptr"):
        if rec_bytes == 16:
            if addrs.dim() != 2 or addrs.shape[1] != 2 or addrs.element_size() != 8:
                raise ValueError(f"addrs must be an (n, 2) tensor of 64-bit words, got {tuple(addrs.shape)} "
                                 f"of {addrs.dtype}")
        elif addrs.dim() != 1 or addrs.element_size() != rec_bytes:
            raise ValueError(f"addrs must be a 1-D tensor of {rec_bytes}-byte addresses")
        if n > addrs.shape[0]:
            raise ValueError(f"n = {n} exceeds the {addrs.shape[0]} address records passed")
    if out is None:
        raise ValueError(f"{what} is required")
    if hasattr(out, "data_ptr"):
        if out.element_size() != out_bytes:
            raise ValueError(f"{what} must hold {out_bytes}-byte elements, got {out.dtype}")
        if n > out.numel():
            raise ValueError(f"n = {n} exceeds the {out.numel()} elements of {what}")
    return n


def planb_lookup(fib: Fib, addrs, n: int | None = None, out=None, stream=None):
    """addrs: device tensor (n, 2) int64 (the {hi, lo} records); out: device
    tensor (n,) int16/uint16 receiving next hops.  Asynchronous on ``stream``."""
    n = _check_io(addrs, out, n, 16, 2)
    _check(_lib.planb_lookup(fib, _dev_ptr(addrs, "addrs"), n, _dev_ptr(out, "out"), _stream_handle(stream)))
    return out


def planb_lookup_index(fib: Fib, addrs, n: int | None = None, out=None, stream=None):
    """Like planb_lookup, but out (n,) int32 receives interval indices."""
    n = _check_io(addrs, out, n, 16, 4)
    _check(_lib.planb_lookup_index(fib, _dev_ptr(addrs, "addrs"), n, _dev_ptr(out, "out"),
                                   _stream_handle(stream)))
    return out


def planb_lookup_v4(fib: Fib, addrs, n: int | None = None, out=None, stream=None):
    """addrs: device tensor (n,) int32 of IPv4 addresses; the FIB must hold 32-bit keys."""
    n = _check_io(addrs, out, n, 4, 2)
    _check(_lib.planb_lookup_v4(fib, _dev_ptr(addrs, "addrs"), n, _dev_ptr(out, "out"), _stream_handle(stream)))
    return out


def planb_lookup_bsearch(fib: Fib, addrs, n: int | None = None, out=None, stream=None):
    """Binary search over the sorted interval starts (ablation baseline); same results as planb_lookup."""
    n = _check_io(addrs, out, n, 16, 2)
    _check(_lib.planb_lookup_bsearch(fib, _dev_ptr(addrs, "addrs"), n, _dev_ptr(out, "out"),
                                     _stream_handle(stream)))
    return out


def planb_num_intervals(fib: Fib) -> int:
    return int(_lib.planb_num_intervals(fib))


def planb_export_intervals(fib: Fib):
    m = planb_num_intervals(fib)
    starts = np.empty((m, 2), dtype=np.uint64)
    nh = np.empty(m, dtype=np.uint16)
    got = _check(_lib.planb_export_intervals(fib, starts.ctypes.data, nh.ctypes.data, m))
    return starts[:got], nh[:got]


def _info_dict(info: planb_info_t) -> dict:
    D = info.depth
    return {"intervals": info.intervals, "fanout": info.fanout, "slots": info.slots, "depth": D,
            "key_bits": info.key_bits,
            "level_nodes": [int(info.level_nodes[i]) for i in range(D)],
            "level_offset": [int(info.level_offset[i]) for i in range(D + 1)],
            "key_bytes": int(info.key_bytes), "value_bytes": int(info.value_bytes),
            "leaf_keys": int(info.leaf_keys), "leaf_slots": int(info.leaf_slots), "leaf_base": int(info.leaf_base)}


def planb_get_info(fib: Fib) -> dict:
    info = planb_info_t()
    _check(_lib.planb_get_info(fib, ctypes.byref(info)))
    return _info_dict(info)


def planb_set_tuning(fib: Fib, keys_per_lane: int, lds_levels: int = -1, lookups_per_group: int = 2,
                     block_threads: int = 512, lds_search: int = 0):
    t = planb_tuning_t(keys_per_lane, lds_levels, lookups_per_group, block_threads, lds_search)
    _check(_lib.planb_set_tuning(fib, ctypes.byref(t)))


def _tuning_dict(t) -> dict:
    return {"keys_per_lane": t.keys_per_lane, "lds_levels": t.lds_levels,
            "lookups_per_group": t.lookups_per_group, "block_threads": t.block_threads, "lds_search": t.lds_search}


def _tuning_struct(d: dict):
    return planb_tuning_t(d["keys_per_lane"], d["lds_levels"], d["lookups_per_group"], d["block_threads"],
                          d.get("lds_search", 0))


def planb_get_tuning(fib: Fib) -> dict:
    t = planb_tuning_t()
    _check(_lib.planb_get_tuning(fib, ctypes.byref(t)))
    return _tuning_dict(t)


def planb_set_size_tunings(fib: Fib, entries):
    """entries: [(min_lookups, tuning dict), ...] with ascending min_lookups ([] clears)."""
    k = len(entries)
    lo = (ctypes.c_uint64 * max(k, 1))(*[int(e[0]) for e in entries])
    tu = (planb_tuning_t * max(k, 1))(*[_tuning_struct(e[1]) for e in entries])
    _check(_lib.planb_set_size_tunings(fib, lo, tu, k))


def planb_get_size_tunings(fib: Fib) -> list:
    k = _lib.planb_get_size_tunings(fib, None, None, 0)
    if k < 0:
        _check(k)
    lo = (ctypes.c_uint64 * max(k, 1))()
    tu = (planb_tuning_t * max(k, 1))()
    _check(min(0, _lib.planb_get_size_tunings(fib, lo, tu, k)))
    return [(int(lo[i]), _tuning_dict(tu[i])) for i in range(k)]


def planb_autotune_sizes(fib: Fib, sample, sizes, reps: int = 3, stream=None) -> list:
    """Autotunes each size on the sample's first addresses and installs the winners as size tunings."""
    k = len(sizes)
    sz = (ctypes.c_uint64 * max(k, 1))(*[int(x) for x in sizes])
    res = (planb_autotune_result_t * max(k, 1))()
    _check(_lib.planb_autotune_sizes(fib, _dev_ptr(sample, "sample"), int(sample.shape[0]), sz, k, reps,
                                     _stream_handle(stream), res))
    return [dict(_tuning_dict(r.tuning), size=int(sizes[i]), ms_per_call=r.ms_per_call, glps=r.glps,
                 candidates=r.candidates) for i, r in enumerate(res[:k])]


def planb_layout(m: int, fanout: int, slots: int, trimmed: bool = True) -> dict:
    info = planb_info_t()
    _check(_lib.planb_layout(m, fanout, slots, 1 if trimmed else 0, ctypes.byref(info)))
    return _info_dict(info)


def planb_build_intervals(prefixes, lengths, next_hops, flags: int = 0):
    """Host-only interval partitioning: returns (starts (m, 2) uint64, next hops (m,) uint16)."""
    n = len(lengths)
    p = _host(prefixes, np.uint64, (2,)) if n else np.zeros((0, 2), np.uint64)
    L = _host(lengths, np.uint8)
    nh = _host(next_hops, np.uint16)
    args = (p.ctypes.data if n else None, L.ctypes.data if n else None, nh.ctypes.data if n else None, n, flags)
    m = _check(_lib.planb_build_intervals(*args, None, None, 0))
    starts = np.empty((m, 2), dtype=np.uint64)
    out_nh = np.empty(m, dtype=np.uint16)
    _check(_lib.planb_build_intervals(*args, starts.ctypes.data, out_nh.ctypes.data, m))
    return starts, out_nh


def planb_build_keys(starts, fanout: int = 16):
    """Host-only key array of the tree over ``starts``: returns (keys (slots, 2) uint64, info)."""
    s = _host(starts, np.uint64, (2,))
    info = planb_info_t()
    need = _check(_lib.planb_build_keys(s.ctypes.data, s.shape[0], fanout, None, 0, ctypes.byref(info)))
    keys = np.empty((need, 2), dtype=np.uint64)
    _check(_lib.planb_build_keys(s.ctypes.data, s.shape[0], fanout, keys.ctypes.data, need, None))
    return keys, _info_dict(info)


def planb_export_image(fib: Fib) -> np.ndarray:
    """The FIB's device slot array, copied to host memory (uint8)."""
    need = _check(_lib.planb_export_image(fib, None, 0))
    img = np.empty(need, dtype=np.uint8)
    _check(_lib.planb_export_image(fib, img.ctypes.data, need))
    return img


def planb_build_image(starts, next_hops, fanout: int = 16, key_bits: int = 0):
    """Host-only device image of the tree over ``starts`` / ``next_hops``: returns (bytes (uint8), info)."""
    s = _host(starts, np.uint64, (2,))
    nh = _host(next_hops, np.uint16)
    if nh.shape[0] != s.shape[0]:
        raise ValueError("starts and next_hops differ in length")
    info = planb_info_t()
    args = (s.ctypes.data, nh.ctypes.data, s.shape[0], fanout, key_bits)
    need = _check(_lib.planb_build_image(*args, None, 0, ctypes.byref(info)))
    img = np.empty(need, dtype=np.uint8)
    _check(_lib.planb_build_image(*args, img.ctypes.data, need, None))
    return img, _info_dict(info)


class CpuTree:
    """Host-core linearized B+-tree baseline over a FIB's device image (planb_cpu_lookup)."""

    def __init__(self, prefixes, lengths, next_hops, fanout: int = 8, key_bits: int = 0):
        starts, nh = planb_build_intervals(prefixes, lengths, next_hops)
        self.image, info = planb_build_image(starts, nh, fanout, key_bits)
        self.info = planb_info_t()
        _check(_lib.planb_build_image(starts.ctypes.data, nh.ctypes.data, starts.shape[0], fanout, key_bits,
                                      None, 0, ctypes.byref(self.info)))
        self.shape = info

    def lookup(self, addrs, threads: int = 0) -> np.ndarray:
        a = _host(addrs, np.uint64, (2,))
        out = np.empty(a.shape[0], dtype=np.uint16)
        _check(_lib.planb_cpu_lookup(self.image.ctypes.data, ctypes.byref(self.info), a.ctypes.data, a.shape[0],
                                     out.ctypes.data, threads))
        return out


_sig("planb_cpu_tree_build", _vp, _vp, _vp, _sz, ctypes.c_uint32)
_sig("planb_cpu_tree_lookup", ctypes.c_int, _vp, _vp, _sz, _vp, ctypes.c_int)
_sig("planb_cpu_tree_isa", ctypes.c_char_p, _vp)
_sig("planb_cpu_tree_depth", ctypes.c_int, _vp)
_sig("planb_cpu_tree_free", None, _vp)


class PaperCpuTree:
    """Host-core baseline in the paper's CPU design (fanout 9, 8 keys per node,
    vector compare + popcount, batched, unrolled): planb_cpu_tree_*."""

    def __init__(self, prefixes, lengths, next_hops, key_bits: int = 64):
        starts, nh = planb_build_intervals(prefixes, lengths, next_hops)
        s = np.ascontiguousarray(starts, dtype=np.uint64)
        h = np.ascontiguousarray(nh, dtype=np.uint16)
        self.ptr = _lib.planb_cpu_tree_build(s.ctypes.data, h.ctypes.data, s.shape[0], key_bits)
        if not self.ptr:
            raise PlanbError(PLANB_EINVAL, f"planb_cpu_tree_build failed (key_bits {key_bits})")
        self.key_bits = key_bits
        self.isa = _lib.planb_cpu_tree_isa(self.ptr).decode()
        self.depth = int(_lib.planb_cpu_tree_depth(self.ptr))

    def lookup(self, addrs, threads: int = 0, out=None) -> np.ndarray:
        a = _host(addrs, np.uint64, (2,))
        if out is None:
            out = np.empty(a.shape[0], dtype=np.uint16)
        _check(_lib.planb_cpu_tree_lookup(self.ptr, a.ctypes.data, a.shape[0], out.ctypes.data, threads))
        return out

    def close(self):
        if getattr(self, "ptr", None):
            _lib.planb_cpu_tree_free(self.ptr)
            self.ptr = None

    def __del__(self):
        self.close()


def batch_array(batches):
    """[(addrs_tensor_or_ptr, out_tensor_or_ptr, n), ...] -> ctypes array of planb_batch_t."""
    arr = (planb_batch_t * max(1, len(batches)))()
    for i, (a, o, n) in enumerate(batches):
        arr[i].addrs = _dev_ptr(a, "addrs") if n else 0
        arr[i].out = _dev_ptr(o, "out") if n else 0
        arr[i].n = n
    return arr


def planb_lookup_batches(fib: Fib, batches_dev, n_batches_dev, max_batches: int, stream=None):
    """batches_dev: device buffer of planb_batch_t records; n_batches_dev: device uint32."""
    _check(_lib.planb_lookup_batches(fib, _dev_ptr(batches_dev, "batches"), _dev_ptr(n_batches_dev, "n_batches"),
                                     max_batches, _stream_handle(stream)))


class Graph:
    """Owner of a planb_graph_t* (captured persistent batch lookups)."""

    def __init__(self, fib: Fib, max_batches: int):
        self.fib = fib  # keeps the FIB alive while the graph exists
        self.max_batches = max_batches
        self.ptr = _lib.planb_graph_create(fib, max_batches)
        if not self.ptr:
            raise PlanbError(planb_last_status(), planb_last_error())

    def launch(self, batches, stream=None):
        arr = batch_array(batches)
        _check(_lib.planb_graph_launch(self.ptr, arr, len(batches), _stream_handle(stream)))

    def close(self):
        if self.ptr:
            _lib.planb_graph_free(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def planb_graph_create(fib: Fib, max_batches: int) -> Graph:
    return Graph(fib, max_batches)


def planb_graph_launch(graph: Graph, batches, stream=None):
    graph.launch(batches, stream)


def planb_graph_free(graph: Graph):
    graph.close()


def planb_autotune(fib: Fib, sample, n: int | None = None, reps: int = 3, stream=None) -> dict:
    if n is None:
        n = sample.shape[0]
    r = planb_autotune_result_t()
    _check(_lib.planb_autotune(fib, _dev_ptr(sample, "sample"), n, reps, _stream_handle(stream), ctypes.byref(r)))
    t = r.tuning
    return {"keys_per_lane": t.keys_per_lane, "lds_levels": t.lds_levels, "lookups_per_group": t.lookups_per_group,
            "block_threads": t.block_threads, "lds_search": t.lds_search, "ms_per_call": r.ms_per_call,
            "glps": r.glps, "candidates": r.candidates}


def planb_train(fib: Fib, epochs: int = 0, batch: int = 0, lr: float = 0.0, segments: int = 0, seed: int = 0,
                stream=None) -> dict:
    cfg = planb_train_cfg_t(epochs, batch, lr, segments, seed)
    r = planb_train_report_t()
    _check(_lib.planb_train(fib, ctypes.byref(cfg), _stream_handle(stream), ctypes.byref(r)))
    return {k: getattr(r, k) for k, _ in planb_train_report_t._fields_}


def planb_lookup_learned(fib: Fib, addrs, n: int | None = None, out=None, fallback_count=None, stream=None):
    n = _check_io(addrs, out, n, 16, 2)
    fb = _dev_ptr(fallback_count, "fallback_count") if fallback_count is not None else None
    _check(_lib.planb_lookup_learned(fib, _dev_ptr(addrs, "addrs"), n, _dev_ptr(out, "out"), fb,
                                     _stream_handle(stream)))
    return out


def planb_lookup_learned_noalloc(fib: Fib, addrs, n: int | None = None, out=None, fallback_count=None, stream=None):
    n = _check_io(addrs, out, n, 16, 2)
    fb = _dev_ptr(fallback_count, "fallback_count") if fallback_count is not None else None
    _check(_lib.planb_lookup_learned_noalloc(fib, _dev_ptr(addrs, "addrs"), n, _dev_ptr(out, "out"), fb,
                                             _stream_handle(stream)))
    return out


def planb_model_num_params() -> int:
    return int(_lib.planb_model_num_params())


def planb_model_set_params(fib: Fib, params, segments: int = 4096):
    p = np.ascontiguousarray(params, dtype=np.float32)
    if p.shape != (planb_model_num_params(),):
        raise ValueError("wrong parameter count")
    _check(_lib.planb_model_set_params(fib, p.ctypes.data, segments))


def planb_model_get_params(fib: Fib) -> np.ndarray:
    p = np.empty(planb_model_num_params(), dtype=np.float32)
    _check(_lib.planb_model_get_params(fib, p.ctypes.data))
    return p


def planb_model_predict(fib: Fib, addrs, n=None, y=None, stream=None):
    n = _check_io(addrs, y, n, 16, 4, "y")
    _check(_lib.planb_model_predict(fib, _dev_ptr(addrs, "addrs"), n, _dev_ptr(y, "y"), _stream_handle(stream)))
    return y


def planb_model_grad(fib: Fib, samples, targets, n=None, grad=None, stream=None):
    n = _check_io(samples, targets, n, 16, 4, "targets")
    if hasattr(grad, "data_ptr") and (grad.element_size() != 4 or grad.numel() < planb_model_num_params()):
        raise ValueError("grad must hold planb_model_num_params() float32 values")
    _check(_lib.planb_model_grad(fib, _dev_ptr(samples, "samples"), _dev_ptr(targets, "targets"), n,
                                 _dev_ptr(grad, "grad"), _stream_handle(stream)))
    return grad


def planb_model_adam(fib: Fib, grad, lr: float, stream=None):
    _check(_lib.planb_model_adam(fib, _dev_ptr(grad, "grad"), lr, _stream_handle(stream)))


def planb_model_build_eps(fib: Fib, stream=None):
    _check(_lib.planb_model_build_eps(fib, _stream_handle(stream)))


def planb_model_get_eps(fib: Fib, segments: int) -> np.ndarray:
    e = np.empty(segments, dtype=np.uint32)
    got = _check(_lib.planb_model_get_eps(fib, e.ctypes.data, segments))
    return e[:got]


def planb_model_set_eps(fib: Fib, eps):
    e = np.ascontiguousarray(eps, dtype=np.uint32)
    _check(_lib.planb_model_set_eps(fib, e.ctypes.data, e.shape[0]))


class TableSet:
    """Owner of a planb_tableset_t* (slot -> FIB descriptors on the device)."""

    def __init__(self, max_tables: int):
        self.ptr = _lib.planb_tableset_create(max_tables)
        if not self.ptr:
            raise PlanbError(planb_last_status(), planb_last_error())
        self.fibs = {}

    def set(self, slot: int, fib: Fib | None):
        _check(_lib.planb_tableset_set(self.ptr, slot, fib if fib is not None else None))
        self.fibs[slot] = fib  # keeps the FIB alive while the slot points at it

    def set_tuning(self, keys_per_lane: int, lookups_per_group: int = 2, block_threads: int = 512):
        _check(_lib.planb_tableset_set_tuning(self.ptr, keys_per_lane, lookups_per_group, block_threads))

    def close(self):
        if self.ptr:
            _lib.planb_tableset_free(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def burst_array(bursts):
    """[(slot, addrs_tensor_or_ptr, out_tensor_or_ptr, n), ...] -> ctypes array of planb_burst_t."""
    arr = (planb_burst_t * max(1, len(bursts)))()
    for i, (slot, a, o, n) in enumerate(bursts):
        arr[i].table = slot
        arr[i].n = n
        arr[i].addrs = _dev_ptr(a, "addrs") if n else 0
        arr[i].out = _dev_ptr(o, "out") if n else 0
    return arr


def planb_lookup_multi(ts: TableSet, bursts_dev, n_bursts_dev, max_bursts: int, stream=None):
    _check(_lib.planb_lookup_multi(ts.ptr, _dev_ptr(bursts_dev, "bursts"), _dev_ptr(n_bursts_dev, "n_bursts"),
                                   max_bursts, _stream_handle(stream)))


def planb_lookup_multi_learned(ts: TableSet, bursts_dev, n_bursts_dev, max_bursts: int, fallback_count=None,
                               stream=None):
    fb = _dev_ptr(fallback_count, "fallback_count") if fallback_count is not None else None
    _check(_lib.planb_lookup_multi_learned(ts.ptr, _dev_ptr(bursts_dev, "bursts"), _dev_ptr(n_bursts_dev, "n_bursts"),
                                           max_bursts, fb, _stream_handle(stream)))


class Server:
    """Owner of a planb_server_t* (see planb.h for the semantics)."""

    def __init__(self, max_tables=16, streams=2, max_bursts=1024, max_lookups=1 << 20, fanout=16, key_bits=128,
                 memory_budget=0, learned=False, zero_copy=False):
        self.cfg = planb_server_cfg_t(max_tables, streams, max_bursts, max_lookups, fanout, key_bits, memory_budget,
                                      1 if learned else 0, PLANB_SERVER_ZERO_COPY if zero_copy else 0)
        self.ptr = _lib.planb_server_create(ctypes.byref(self.cfg))
        if not self.ptr:
            raise PlanbError(planb_last_status(), planb_last_error())
        self._comp = (planb_completion_t * 4096)()
        self._keep = {}

    def set_table(self, table_id, prefixes, lengths, next_hops):
        n = len(lengths)
        p = _host(prefixes, np.uint64, (2,)) if n else np.zeros((0, 2), np.uint64)
        L = _host(lengths, np.uint8)
        nh = _host(next_hops, np.uint16)
        _check(_lib.planb_server_set_table(self.ptr, table_id, p.ctypes.data if n else None,
                                           L.ctypes.data if n else None, nh.ctypes.data if n else None, n))

    def submit(self, table_id, addrs: np.ndarray, out: np.ndarray, tag: int):
        """addrs (n, 2) uint64 host; out (n,) uint16 host array written before completion."""
        a = _host(addrs, np.uint64, (2,))
        if out.dtype != np.uint16 or not out.flags.c_contiguous or out.shape[0] < a.shape[0]:
            raise ValueError("out must be a contiguous uint16 array of at least n elements")
        self._keep[tag] = (a, out)  # both must outlive the burst
        _check(_lib.planb_server_submit(self.ptr, table_id, a.ctypes.data, a.shape[0], out.ctypes.data, tag))

    def poll(self, block: bool = False):
        k = _check(_lib.planb_server_poll(self.ptr, self._comp, len(self._comp), 1 if block else 0))
        res = []
        for i in range(k):
            c = self._comp[i]
            self._keep.pop(c.tag, None)
            res.append((c.tag, c.table, c.n, c.submit_us, c.done_us, c.status))
        return res

    def admit(self, table_id: int):
        _check(_lib.planb_server_admit(self.ptr, table_id))

    def replay(self, arrival_us, tables, offsets, addrs, out):
        """Native open-loop replay (planb_server_replay); returns (latency_us, wall_s)."""
        arr = np.ascontiguousarray(arrival_us, dtype=np.float64)
        tb = np.ascontiguousarray(tables, dtype=np.uint32)
        off = np.ascontiguousarray(offsets, dtype=np.uint64)
        a = _host(addrs, np.uint64, (2,))
        if out.dtype != np.uint16 or not out.flags.c_contiguous or out.shape[0] < a.shape[0]:
            raise ValueError("out must be a contiguous uint16 array covering every address")
        lat = np.zeros(arr.shape[0], dtype=np.float64)
        wall = ctypes.c_double(0.0)
        _check(_lib.planb_server_replay(self.ptr, arr.shape[0], arr.ctypes.data, tb.ctypes.data, off.ctypes.data,
                                        a.ctypes.data, out.ctypes.data, lat.ctypes.data, ctypes.byref(wall)))
        return lat, wall.value

    def register_io(self, ptr: int, nbytes: int):
        """Registers pinned host memory [ptr, ptr + nbytes) for zero-copy bursts."""
        _check(_lib.planb_server_register_io(self.ptr, ptr, nbytes))

    def replay_raw(self, arrival_us, tables, offsets, addrs_ptr: int, out_ptr: int):
        """planb_server_replay over raw host pointers (e.g. pinned tensors); returns (latency_us, wall_s)."""
        arr = np.ascontiguousarray(arrival_us, dtype=np.float64)
        tb = np.ascontiguousarray(tables, dtype=np.uint32)
        off = np.ascontiguousarray(offsets, dtype=np.uint64)
        lat = np.zeros(arr.shape[0], dtype=np.float64)
        wall = ctypes.c_double(0.0)
        _check(_lib.planb_server_replay(self.ptr, arr.shape[0], arr.ctypes.data, tb.ctypes.data, off.ctypes.data,
                                        addrs_ptr, out_ptr, lat.ctypes.data, ctypes.byref(wall)))
        return lat, wall.value

    def stats(self) -> dict:
        st = planb_server_stats_t()
        _check(_lib.planb_server_stats(self.ptr, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in planb_server_stats_t._fields_}

    def close(self):
        if self.ptr:
            _lib.planb_server_free(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def planb_server_now_us() -> float:
    return float(_lib.planb_server_now_us())


def exported_symbols() -> list[str]:
    """Names of the planb_* functions the header declares, for ABI checks."""
    return [n for n in dir(_lib) if n.startswith("planb_")]
