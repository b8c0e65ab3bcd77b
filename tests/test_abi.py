"""The C-ABI library loads and exports every function include/*.h declares;
argument errors are reported without touching a GPU."""
import ctypes
import glob
import os
import re

import pytest

from paper_2604_14650_amd import planb as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(planb_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_core_calls():
    names = declared_functions()
    for core in ("planb_build", "planb_lookup", "planb_free", "planb_last_error"):
        assert core in names


@pytest.mark.parametrize("name", declared_functions())
def test_symbol_exported(name):
    lib = ctypes.CDLL(P.LIB_PATH)
    assert hasattr(lib, name), name


def test_lookup_argument_errors_need_no_gpu():
    lib = P.lib_handle()
    assert lib.planb_lookup(None, None, 10, None, None) == P.PLANB_EINVAL
    assert "NULL fib" in P.planb_last_error()
    assert lib.planb_lookup_index(None, None, 0, None, None) == P.PLANB_EINVAL
    assert lib.planb_num_intervals(None) == 0
    lib.planb_free(None)


def test_layout_argument_errors():
    with pytest.raises(P.PlanbError):
        P.planb_layout(0, 16, 16)
    with pytest.raises(P.PlanbError):
        P.planb_layout(10, 16, 4)


def test_binding_checks_sizes_and_layouts():
    """The wrappers refuse an n beyond the tensors passed, or a record or
    element layout the C call does not read, before any device call."""
    import torch
    from paper_2604_14650_amd import planb as P
    a = torch.zeros((10, 2), dtype=torch.int64)
    o = torch.zeros(10, dtype=torch.int16)
    assert P._check_io(a, o, None, 16, 2) == 10
    assert P._check_io(a, o, 7, 16, 2) == 7
    for bad in [lambda: P._check_io(a, o, 11, 16, 2),                       # n beyond addrs
                lambda: P._check_io(a, o[:5], 8, 16, 2),                    # n beyond out
                lambda: P._check_io(a, torch.zeros(10, dtype=torch.int32), 10, 16, 2),  # 4-byte outputs
                lambda: P._check_io(a.view(-1), o, 10, 16, 2),              # not (n, 2) records
                lambda: P._check_io(a.to(torch.int32), o, 10, 16, 2),       # 32-bit words
                lambda: P._check_io(a, o, 10, 16, 4),                       # index output needs 4 bytes
                lambda: P._check_io(torch.zeros(10, dtype=torch.int64), o, 10, 4, 2),  # IPv4 takes 4-byte words
                lambda: P._check_io(a, None, 10, 16, 2)]:
        with pytest.raises(ValueError):
            bad()
