"""The C-ABI library loads and exports every function include/mspfmm.h declares;
host-side argument checks answer with status codes (no GPU work is launched)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2301_10570_amd", "libmspfmm.so")
HEADER = os.path.join(ROOT, "include", "mspfmm.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(msp_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import importlib.util
        spec = importlib.util.spec_from_file_location(
            "_mspfmm_build", os.path.join(ROOT, "paper_2301_10570_amd", "build.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build()
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 12
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings(lib):
    lib.msp_status_string.restype = ctypes.c_char_p
    assert lib.msp_status_string(0) == b"ok"
    assert lib.msp_status_string(-1) == b"invalid argument"
    assert lib.msp_status_string(-2) == b"size limit exceeded"
    assert lib.msp_status_string(-6) == b"handle not ready"
    assert lib.msp_status_string(-99) == b"unknown status"


def test_argument_checks_without_device(lib):
    lib.msp_last_error.restype = ctypes.c_char_p
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.msp_octree_build.argtypes = [vp, vp, vp, vp, i64, i32, i32, vp]
    assert lib.msp_octree_build(None, None, None, None, 10, 64, 21, None) == -1
    assert b"NULL" in lib.msp_last_error()
    lib.msp_direct_sum.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, i64, ctypes.c_float, vp, vp]
    assert lib.msp_direct_sum(None, None, None, -1, None, None, None, None, 0, 1.0, None, None) == -1
    assert lib.msp_direct_sum(None, None, None, 3, None, None, None, None, 0, 1.0, None, None) == -1
    assert lib.msp_direct_sum(None, None, None, 1 << 40, None, None, None, None, 0, 1.0, None, None) == -3
    lib.msp_tree_get_info.argtypes = [vp, vp]
    assert lib.msp_tree_get_info(None, None) == -1
    lib.msp_fgt_debug_buffer.argtypes = [vp, i32, vp, ctypes.c_size_t, vp, vp]
    assert lib.msp_fgt_debug_buffer(None, 0, None, 0, None, None) == -1
