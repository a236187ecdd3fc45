"""The C ABI library builds, loads and exports every function include/arrow.h declares (no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "arrow.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:int|size_t)\s+([a-z0-9_]+)\s*\(", src, flags=re.M)
    assert names
    return names


@pytest.fixture(scope="module")
def libarrow():
    from paper_1302_7203_amd import build as B
    if B.stale():
        B.build()
    return ctypes.CDLL(B.LIB)


def test_header_declares_the_documented_entry_points():
    names = set(declared_functions())
    for f in ("arrow_create", "arrow_destroy", "arrow_set_stream", "arrow_set_option",
              "arrow_workspace_size", "arrow_eig", "arrow_eig_herm", "dpr1_eig", "arrow_svd"):
        assert f in names


def test_every_declared_symbol_is_exported(libarrow):
    for name in declared_functions():
        assert hasattr(libarrow, name), name


def test_workspace_size_is_host_only(libarrow):
    f = libarrow.arrow_workspace_size
    f.argtypes = [ctypes.c_int64]
    f.restype = ctypes.c_size_t
    assert f(0) == 0
    assert f(1) > 0
    assert f(16384) >= 16384 * 15 * 8


def test_binding_loads_the_built_library():
    from paper_1302_7203_amd import binding
    L = binding.lib()
    assert L is not None and os.path.samefile(binding.LIB_PATH, os.path.join(ROOT, "paper_1302_7203_amd", "libarrow.so"))


def test_null_handle_is_rejected(libarrow):
    f = libarrow.arrow_eig
    f.restype = ctypes.c_int
    assert f(None, ctypes.c_int64(4), None, None, ctypes.c_double(0.0), None, None, ctypes.c_int64(4),
             None, None, None) == -1


def test_order_cap_is_host_side(libarrow):
    """Orders above ARROW_N_MAX (where n * 64 lanes would pass 2^31) are refused
    before any device work: the workspace query, host-only, says 0 there."""
    src = open(HEADER).read()
    cap = int(re.search(r"#define ARROW_N_MAX (\d+)", src).group(1))
    assert cap * 64 <= 2 ** 31
    f = libarrow.arrow_workspace_size
    f.argtypes = [ctypes.c_int64]
    f.restype = ctypes.c_size_t
    assert f(cap) > 0 and f(cap + 1) == 0 and f(2 ** 28) == 0 and f(-1) == 0
