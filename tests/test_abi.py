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
