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
    lib.msp_tree_set_work_counting.argtypes = [vp, ctypes.c_int]
    assert lib.msp_tree_set_work_counting(None, 1) == -1
    lib.msp_tree_get_work_counts.argtypes = [vp, vp, ctypes.c_int]
    assert lib.msp_tree_get_work_counts(None, None, 0) == -1


class _Params(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("level", ctypes.c_int32), ("sigma", ctypes.c_float),
                ("cutoff_sigmas", ctypes.c_float), ("route", ctypes.c_int32), ("flags", ctypes.c_uint32)]


def _build_query(lib, n, leaf_max=64, max_depth=21):
    sz = ctypes.c_size_t
    lib.msp_octree_build_query.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.POINTER(sz), ctypes.POINTER(sz)]
    tb, wb = sz(), sz()
    rc = lib.msp_octree_build_query(n, leaf_max, max_depth, ctypes.byref(tb), ctypes.byref(wb))
    return rc, tb.value, wb.value


def test_build_query_sizes(lib):
    rc, tb, wb = _build_query(lib, 0)
    assert rc == 0 and tb > 0 and wb > 0
    # per point the tree keeps keys (8 B), permutation (4), two packed position
    # arrays (2 x 16) and the inverse permutation (4); the scratch holds at least a
    # second key and index array
    for n in (1000, 100000, 4194304):
        rc, tb, wb = _build_query(lib, n)
        assert rc == 0
        assert tb >= 48 * n and wb >= 12 * n
    assert _build_query(lib, -1)[0] == -1
    assert _build_query(lib, 1 << 31)[0] == -3
    assert _build_query(lib, 10, 0)[0] == -1
    assert _build_query(lib, 10, 64, 22)[0] == -1


def test_build_query_node_bound_holds_for_oracle_trees(lib):
    """The tree buffer from the query holds the node table of every tree the oracle
    builds, including nested clusters that make long single-child chains."""
    import numpy as np

    from oracle import octree
    rng = np.random.default_rng(7)
    cases = []
    cases.append(rng.random((5000, 3)).astype(np.float32) * 1000)
    # 65 points at each of 12 nested scales: every level has one full cell
    pts = [rng.random((65, 3)) * (0.5 ** k) for k in range(12)]
    cases.append((np.concatenate(pts) * 1000).astype(np.float32))
    # duplicates: a depth-21 leaf holding more than leaf_max points
    cases.append(np.repeat(rng.random((3, 3)).astype(np.float32), 200, axis=0))
    per_node = 10 * 4 + 4 + 8   # node table, list length, list offset
    for leaf in (1, 8, 64):
        for p in cases:
            n = p.shape[0]
            tr = octree.build(p[:, 0], p[:, 1], p[:, 2], leaf_max=leaf)
            nn = int(tr.first.size)
            rc, tb, _ = _build_query(lib, n, leaf)
            assert rc == 0
            rc0, tb_points, _ = _build_query(lib, n, n)   # leaf_max = n: the root alone
            assert tb - tb_points >= per_node * (nn - 1), (leaf, n, nn)


def test_new_entry_points_check_arguments(lib):
    vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    lib.msp_last_error.restype = ctypes.c_char_p
    lib.msp_octree_build_ws.argtypes = [vp, vp, vp, vp, i64, i32, i32, vp, sz, vp, sz, vp]
    assert lib.msp_octree_build_ws(None, None, None, None, 10, 64, 21, None, 0, None, 0, None) == -1
    lib.msp_fgt_forward_query.argtypes = [vp, ctypes.POINTER(_Params), ctypes.POINTER(sz), vp]
    out = sz()
    prm = _Params(8, -1, 100.0, 4.5, 0, 0)
    assert lib.msp_fgt_forward_query(None, ctypes.byref(prm), ctypes.byref(out), None) == -1
    lib.msp_fgt_forward_ws.argtypes = [vp, vp, vp, ctypes.POINTER(_Params), vp, vp, sz, vp]
    assert lib.msp_fgt_forward_ws(None, None, None, ctypes.byref(prm), None, None, 0, None) == -1
    lib.msp_batch_pair_count.argtypes = [vp, vp, vp, vp]
    assert lib.msp_batch_pair_count(None, None, None, None) == -1
    assert b"NULL" in lib.msp_last_error()


def test_batch_refuses_flags_it_does_not_honour(lib):
    """The batched kernels translate on the matrix cores on one level (fp32, or
    split bf16 at p = 8): the vector and two-level flags, split bf16 at other p and
    the staging flags are refused, not silently ignored."""
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    lib.msp_last_error.restype = ctypes.c_char_p
    lib.msp_batch_forward.argtypes = [vp, vp, vp, vp, ctypes.POINTER(_Params), vp, i32, vp]
    lib.msp_batch_backward.argtypes = [vp, vp, vp, vp, ctypes.POINTER(_Params), vp, vp, vp, vp, vp, vp,
                                       i32, vp]
    for p_, flag in ((8, 2), (8, 4), (6, 8), (8, 16), (8, 32)):   # M2L_VALU, TWO_LEVEL, M2L_BF16X3 at
        prm = _Params(p_, -1, 100.0, 4.5, 0, flag)                 # p != 8, WEIGHTS_STAGED, STAGE_WEIGHTS
        assert lib.msp_batch_forward(None, None, None, None, ctypes.byref(prm), None, 1, None) == -5
        assert b"not supported" in lib.msp_last_error()
        assert lib.msp_batch_backward(None, None, None, None, ctypes.byref(prm), None, None, None, None, None,
                                      None, 0, None) == -5
    for flag in (1, 8):   # EXCLUDE_SELF and (at p = 8) M2L_BF16X3 are honoured
        prm = _Params(8, -1, 100.0, 4.5, 0, flag)
        assert lib.msp_batch_forward(None, None, None, None, ctypes.byref(prm), None, 1, None) == -1
