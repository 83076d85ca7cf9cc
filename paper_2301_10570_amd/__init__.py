"""Python binding of libmspfmm (include/mspfmm.h): argument marshalling only.

Every step of the computation runs in the HIP kernels of the shared library;
this module checks tensors, passes their device pointers and the current torch
stream, and turns status codes into exceptions.  PyTorch supplies device memory
and streams.  The library must have been built (python -m
paper_2301_10570_amd/build.py); importing without it raises ImportError.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmspfmm.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "mspfmm.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing; build it with `python paper_2301_10570_amd/build.py`")

_lib = ctypes.CDLL(LIB_PATH)

MSP_OK, MSP_EINVAL, MSP_ENOSPC, MSP_EOVERFLOW, MSP_EHIP, MSP_ENOTSUP, MSP_ESTATE = 0, -1, -2, -3, -4, -5, -6
ROUTES = {"auto": 0, "fgt": 1, "direct": 2}
ROUTE_NAMES = {v: k for k, v in ROUTES.items()}
EXCLUDE_SELF = 1
M2L_VALU = 2
TWO_LEVEL = 4
M2L_BF16X3 = 8
WEIGHTS_STAGED = 16
STAGE_WEIGHTS = 32


class MspError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = _lib.msp_last_error().decode(errors="replace")
        status = _lib.msp_status_string(code).decode()
        super().__init__(f"{where}: {status} ({code}): {msg}")


class TreeInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_nodes", ctypes.c_int64), ("depth", ctypes.c_int32),
                ("leaf_max", ctypes.c_int32), ("max_depth", ctypes.c_int32),
                ("qmax", ctypes.c_int32 * 3), ("lo", ctypes.c_double * 3), ("side", ctypes.c_double),
                ("level_offset", ctypes.c_int64 * 23)]


class TreeArrays(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in
                ("keys", "perm", "node_level", "node_first", "node_count", "node_parent",
                 "node_first_child", "node_n_children", "node_digit", "node_ix", "node_iy", "node_iz")]


class FgtParams(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("level", ctypes.c_int32), ("sigma", ctypes.c_float),
                ("cutoff_sigmas", ctypes.c_float), ("route", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class FgtInfo(ctypes.Structure):
    _fields_ = [("route", ctypes.c_int32), ("level", ctypes.c_int32), ("grid", ctypes.c_int32 * 3),
                ("p", ctypes.c_int32), ("rho", ctypes.c_double), ("fgt_cost", ctypes.c_double),
                ("direct_cost", ctypes.c_double), ("fine_terms", ctypes.c_int32)]


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_lib.msp_status_string.restype = ctypes.c_char_p
_lib.msp_status_string.argtypes = [ctypes.c_int]
_lib.msp_last_error.restype = ctypes.c_char_p
_lib.msp_last_error.argtypes = []
_lib.msp_tree_create.argtypes = [ctypes.POINTER(_vp)]
_lib.msp_tree_destroy.argtypes = [_vp]
_lib.msp_tree_destroy.restype = None
_lib.msp_octree_build.argtypes = [_vp, _vp, _vp, _vp, _i64, _i32, _i32, _vp]
_sz = ctypes.c_size_t
_lib.msp_octree_build_weighted.argtypes = [_vp, _vp, _vp, _vp, _vp, _i64, _i32, _i32, _vp]
_lib.msp_octree_build_query.argtypes = [_i64, _i32, _i32, ctypes.POINTER(_sz), ctypes.POINTER(_sz)]
_lib.msp_octree_build_ws.argtypes = [_vp, _vp, _vp, _vp, _i64, _i32, _i32, _vp, _sz, _vp, _sz, _vp]
_lib.msp_fgt_forward_query.argtypes = [_vp, ctypes.POINTER(FgtParams), ctypes.POINTER(_sz), _vp]
_lib.msp_fgt_forward_ws.argtypes = [_vp, _vp, _vp, ctypes.POINTER(FgtParams), _vp, _vp, _sz, _vp]
_lib.msp_fgt_forward_noalloc.argtypes = [_vp, _vp, _vp, ctypes.POINTER(FgtParams), _vp, _vp]
_lib.msp_tree_get_info.argtypes = [_vp, ctypes.POINTER(TreeInfo)]
_lib.msp_tree_export.argtypes = [_vp, ctypes.POINTER(TreeArrays), _vp]
_lib.msp_fgt_plan.argtypes = [_vp, ctypes.POINTER(FgtParams), ctypes.POINTER(FgtInfo)]
_lib.msp_fgt_forward.argtypes = [_vp, _vp, _vp, ctypes.POINTER(FgtParams), _vp, _vp]
_lib.msp_fgt_backward.argtypes = [_vp, _vp, _vp, ctypes.POINTER(FgtParams), _vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.msp_direct_sum.argtypes = [_vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _i64, ctypes.c_float, _vp, _vp]
_lib.msp_descent_step.argtypes = [_vp, _vp, _vp, ctypes.POINTER(FgtParams), ctypes.c_uint64, ctypes.c_int32,
                                  _vp, _vp, _i64, _vp, _vp, _i64, ctypes.POINTER(_i64), _vp, _vp, _i64,
                                  ctypes.POINTER(_i64), _vp]
_lib.msp_partner_descent.argtypes = [_vp, _vp, _vp, ctypes.POINTER(FgtParams), ctypes.c_uint64, _vp, _vp, _vp,
                                     ctypes.POINTER(_i64), ctypes.POINTER(_i32), _vp]
_lib.msp_partner_probabilities.argtypes = [_vp, _vp, ctypes.POINTER(FgtParams), _vp, _vp, _i64, _vp,
                                           _vp, _vp, _vp]
_lib.msp_fgt_debug_buffer.argtypes = [_vp, _i32, _vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t), _vp]
_lib.msp_tree_set_work_counting.argtypes = [_vp, ctypes.c_int]
_lib.msp_tree_get_work_counts.argtypes = [_vp, ctypes.POINTER(_i64), ctypes.c_int]
_lib.msp_tree_set_timing.argtypes = [_vp, ctypes.c_int]
_lib.msp_tree_get_timing.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64), ctypes.c_int]
_lib.msp_phase_name.restype = ctypes.c_char_p
_lib.msp_phase_name.argtypes = [ctypes.c_int]
_lib.msp_batch_create.argtypes = [ctypes.POINTER(_vp)]
_lib.msp_batch_destroy.argtypes = [_vp]
_lib.msp_batch_destroy.restype = None
_lib.msp_batch_build.argtypes = [_vp, _vp, _vp, _vp, _vp, _i32, _vp, _i32, _vp]
_lib.msp_batch_autotune.argtypes = [_vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp, ctypes.POINTER(FgtParams),
                                    _vp, _i32, _i32, _vp, _vp, _vp, _vp]
_lib.msp_batch_forward.argtypes = [_vp, _vp, _vp, _vp, ctypes.POINTER(FgtParams), _vp, _i32, _vp]
_lib.msp_batch_backward.argtypes = [_vp, _vp, _vp, _vp, ctypes.POINTER(FgtParams), _vp, _vp, _vp, _vp, _vp,
                                    _vp, ctypes.c_int32, _vp]
_lib.msp_batch_instance_ms.argtypes = [_vp, _vp]
_lib.msp_batch_info.argtypes = [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i64)]
_lib.msp_batch_pair_count.argtypes = [_vp, ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_double), _vp]
PHASE_COUNT = 32
for _f in ("msp_octree_build_weighted", "msp_octree_build_query", "msp_octree_build_ws", "msp_fgt_forward_query", "msp_fgt_forward_ws",
           "msp_fgt_forward_noalloc",
           "msp_fgt_backward", "msp_tree_set_work_counting", "msp_tree_get_work_counts", "msp_tree_set_timing", "msp_tree_get_timing", "msp_tree_create", "msp_octree_build", "msp_tree_get_info", "msp_tree_export",
           "msp_fgt_plan", "msp_fgt_forward", "msp_direct_sum", "msp_partner_probabilities",
           "msp_descent_step", "msp_partner_descent",
           "msp_fgt_debug_buffer", "msp_batch_create", "msp_batch_build", "msp_batch_autotune",
           "msp_batch_forward", "msp_batch_backward", "msp_batch_instance_ms", "msp_batch_info",
           "msp_batch_pair_count"):
    getattr(_lib, _f).restype = ctypes.c_int


def declared_functions() -> list[str]:
    """Names of the functions include/mspfmm.h declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(msp_[a-z0-9_]+)\s*\(", text)))


def _check(rc: int, where: str):
    if rc != MSP_OK:
        raise MspError(rc, where)


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: torch.Tensor | None, dtype: torch.dtype, n: int | None, name: str):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return t.data_ptr() if t.numel() else None


def _params(sigma, p, level, route, cutoff_sigmas, exclude_self, m2l="mfma", two_level=False) -> FgtParams:
    flags = (EXCLUDE_SELF if exclude_self else 0) | (M2L_VALU if m2l == "valu" else 0)
    flags |= (M2L_BF16X3 if m2l == "bf16x3" else 0) | (TWO_LEVEL if two_level else 0)
    if m2l not in ("mfma", "valu", "bf16x3"):
        raise ValueError(f"m2l must be 'mfma', 'valu' or 'bf16x3', got {m2l!r}")
    return FgtParams(int(p), int(level), float(sigma), float(cutoff_sigmas),
                     ROUTES[route] if isinstance(route, str) else int(route), flags)


class Tree:
    """An octree built on the GPU (owns the library handle and its device memory)."""

    def __init__(self):
        h = _vp()
        _check(_lib.msp_tree_create(ctypes.byref(h)), "msp_tree_create")
        self._h = h
        self.n = 0

    def close(self):
        if getattr(self, "_h", None):
            _lib.msp_tree_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def build(self, x, y, z, leaf_max=64, max_depth=21, w=None):
        """Build the octree; with w, carry the weights into key order as well
        (msp_octree_build_weighted) for calls with weights_staged=True."""
        n = x.numel()
        px, py, pz = (_ptr(v, torch.float32, n, nm) for v, nm in ((x, "x"), (y, "y"), (z, "z")))
        if w is None:
            _check(_lib.msp_octree_build(self._h, px, py, pz, n, int(leaf_max), int(max_depth), _stream()),
                   "msp_octree_build")
        else:
            pw = _ptr(w, torch.float32, n, "w")
            _check(_lib.msp_octree_build_weighted(self._h, px, py, pz, pw, n, int(leaf_max), int(max_depth),
                                                  _stream()), "msp_octree_build_weighted")
        self.n = n
        self._keep = (x, y, z)
        return self

    def build_ws(self, x, y, z, tree_buf, ws, leaf_max=64, max_depth=21):
        """msp_octree_build_ws: the tree's arrays in tree_buf, the build scratch in ws
        (CUDA uint8 tensors of at least the sizes build_query gives; tree_buf is kept
        referenced by this object for as long as the tree uses it)."""
        n = x.numel()
        px, py, pz = (_ptr(v, torch.float32, n, nm) for v, nm in ((x, "x"), (y, "y"), (z, "z")))
        pt = _ptr(tree_buf, torch.uint8, None, "tree_buf")
        pw = _ptr(ws, torch.uint8, None, "ws")
        _check(_lib.msp_octree_build_ws(self._h, px, py, pz, n, int(leaf_max), int(max_depth), pt,
                                        tree_buf.numel(), pw, ws.numel(), _stream()), "msp_octree_build_ws")
        self.n = n
        self._keep = (x, y, z, tree_buf)
        return self

    def forward_query(self, sigma, p=8, level=-1, route="auto", cutoff_sigmas=4.5, exclude_self=False,
                      m2l="mfma", two_level=False) -> int:
        """Workspace bytes of forward_ws for these parameters (msp_fgt_forward_query)."""
        prm = _params(sigma, p, level, route, cutoff_sigmas, exclude_self, m2l, two_level)
        nbytes = _sz()
        _check(_lib.msp_fgt_forward_query(self._h, ctypes.byref(prm), ctypes.byref(nbytes), _stream()),
               "msp_fgt_forward_query")
        return nbytes.value

    def forward_ws(self, w, ws, is_target=None, sigma=100.0, p=8, level=-1, route="auto", cutoff_sigmas=4.5,
                   exclude_self=False, out=None, m2l="mfma", two_level=False, stage_weights=False):
        """forward() with every per-call buffer in ws, a CUDA uint8 tensor of at least
        forward_query() bytes (msp_fgt_forward_ws)."""
        n = self.n
        pw = _ptr(w, torch.float32, n, "w")
        pt = _ptr(is_target, torch.uint8, n, "is_target")
        pws = _ptr(ws, torch.uint8, None, "ws")
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=w.device)
        po = _ptr(out, torch.float32, n, "out")
        prm = _params(sigma, p, level, route, cutoff_sigmas, exclude_self, m2l, two_level)
        if stage_weights:
            prm.flags |= STAGE_WEIGHTS
        _check(_lib.msp_fgt_forward_ws(self._h, pw, pt, ctypes.byref(prm), po, pws, ws.numel(), _stream()),
               "msp_fgt_forward_ws")
        return out

    def forward_noalloc(self, w, is_target=None, sigma=100.0, p=8, level=-1, route="auto", cutoff_sigmas=4.5,
                        exclude_self=False, out=None, m2l="mfma", two_level=False):
        """forward() without any device allocation by the library: its buffers are the
        library's fixed per-device scratch (msp_fgt_forward_noalloc).  `out` must be
        given when the caller cannot allocate either."""
        n = self.n
        pw = _ptr(w, torch.float32, n, "w")
        pt = _ptr(is_target, torch.uint8, n, "is_target")
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=w.device)
        po = _ptr(out, torch.float32, n, "out")
        prm = _params(sigma, p, level, route, cutoff_sigmas, exclude_self, m2l, two_level)
        _check(_lib.msp_fgt_forward_noalloc(self._h, pw, pt, ctypes.byref(prm), po, _stream()),
               "msp_fgt_forward_noalloc")
        return out

    def info(self) -> dict:
        inf = TreeInfo()
        _check(_lib.msp_tree_get_info(self._h, ctypes.byref(inf)), "msp_tree_get_info")
        return {"n": inf.n, "n_nodes": inf.n_nodes, "depth": inf.depth, "leaf_max": inf.leaf_max,
                "max_depth": inf.max_depth, "qmax": list(inf.qmax), "lo": list(inf.lo), "side": inf.side,
                "level_offset": list(inf.level_offset)}

    def export(self) -> dict:
        inf = self.info()
        n, nn = inf["n"], inf["n_nodes"]
        dev = torch.device("cuda", torch.cuda.current_device())
        out = {"keys": torch.empty(n, dtype=torch.int64, device=dev),
               "perm": torch.empty(n, dtype=torch.int32, device=dev)}
        for k in ("node_level", "node_first", "node_count", "node_parent", "node_first_child",
                  "node_n_children", "node_digit", "node_ix", "node_iy", "node_iz"):
            out[k] = torch.empty(nn, dtype=torch.int32, device=dev)
        arr = TreeArrays(*[out[f[0]].data_ptr() if out[f[0]].numel() else None for f in TreeArrays._fields_])
        _check(_lib.msp_tree_export(self._h, ctypes.byref(arr), _stream()), "msp_tree_export")
        return out

    def plan(self, sigma, p=8, level=-1, route="auto", cutoff_sigmas=4.5, exclude_self=False,
             two_level=False) -> dict:
        prm = _params(sigma, p, level, route, cutoff_sigmas, exclude_self, two_level=two_level)
        inf = FgtInfo()
        _check(_lib.msp_fgt_plan(self._h, ctypes.byref(prm), ctypes.byref(inf)), "msp_fgt_plan")
        return {"route": ROUTE_NAMES[inf.route], "level": inf.level, "grid": list(inf.grid), "p": inf.p,
                "rho": inf.rho, "fgt_cost": inf.fgt_cost, "direct_cost": inf.direct_cost,
                "fine_terms": inf.fine_terms}

    def forward(self, w, is_target=None, sigma=100.0, p=8, level=-1, route="auto", cutoff_sigmas=4.5,
                exclude_self=False, out=None, m2l="mfma", two_level=False, stage_weights=False,
                weights_staged=False):
        """u[i] = sum_j w[j] exp(-|x_i - x_j|^2/sigma^2) for targets, 0 elsewhere.
        stage_weights: keep the weights gathered into key order for a following
        partner_probabilities(..., weights_staged=True) (MSP_STAGE_WEIGHTS).
        weights_staged: w equals the weights the tree already holds in key order
        (build(..., w=w), or an earlier call that kept them; MSP_WEIGHTS_STAGED)."""
        n = self.n
        pw = _ptr(w, torch.float32, n, "w")
        pt = _ptr(is_target, torch.uint8, n, "is_target")
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=w.device)
        po = _ptr(out, torch.float32, n, "out")
        prm = _params(sigma, p, level, route, cutoff_sigmas, exclude_self, m2l, two_level)
        if stage_weights:
            prm.flags |= STAGE_WEIGHTS
        if weights_staged:
            prm.flags |= WEIGHTS_STAGED
        _check(_lib.msp_fgt_forward(self._h, pw, pt, ctypes.byref(prm), po, _stream()), "msp_fgt_forward")
        return out

    def set_work_counting(self, enable: bool = True):
        """Count the partner query kernels' work (msp_tree_set_work_counting)."""
        _check(_lib.msp_tree_set_work_counting(self._h, 1 if enable else 0), "msp_tree_set_work_counting")

    WORK_NAMES = ("direct_queries", "direct_pairs", "wave_queries", "wave_pairs", "walk_queries", "walk_nodes",
                  "walk_expansions", "walk_pairs", "walk_rounds")

    def work_counts(self, reset: bool = True) -> dict:
        """The partner work counters (msp_tree_get_work_counts) by name."""
        c = (_i64 * 16)()
        _check(_lib.msp_tree_get_work_counts(self._h, c, 1 if reset else 0), "msp_tree_get_work_counts")
        return {name: int(c[k]) for k, name in enumerate(self.WORK_NAMES)}

    def set_timing(self, enable: bool = True, isolated: bool = False):
        """Record HIP events around every library phase on the caller's stream.
        isolated: the passes the library would overlap on a side stream run one
        after another on the caller's stream, so each phase's time is its own."""
        mode = (2 if isolated else 1) if enable else 0
        _check(_lib.msp_tree_set_timing(self._h, mode), "msp_tree_set_timing")

    def timing(self, reset: bool = True) -> dict:
        """{phase: (total ms, launches)} for phases that ran since the last reset."""
        ms = (ctypes.c_double * PHASE_COUNT)()
        cnt = (_i64 * PHASE_COUNT)()
        _check(_lib.msp_tree_get_timing(self._h, ms, cnt, 1 if reset else 0), "msp_tree_get_timing")
        out = {}
        for k in range(PHASE_COUNT):
            if cnt[k]:
                out[_lib.msp_phase_name(k).decode()] = (ms[k], int(cnt[k]))
        return out

    def backward(self, w, grad_u, is_target=None, sigma=100.0, p=8, level=-1, route="auto",
                 cutoff_sigmas=4.5, exclude_self=False, want=("w", "pos", "sigma"), m2l="mfma"):
        """Derivatives of sum_i grad_u[i] * u_i (targets only): dict with 'w' [n],
        'pos' ([n] x, y, z tensors), 'sigma' (float64 [1])."""
        n = self.n
        dev = w.device
        pw = _ptr(w, torch.float32, n, "w")
        pg = _ptr(grad_u, torch.float32, n, "grad_u")
        pt = _ptr(is_target, torch.uint8, n, "is_target")
        out = {}
        gw = torch.empty(n, dtype=torch.float32, device=dev) if "w" in want else None
        gpos = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(3)] if "pos" in want else None
        gs = torch.zeros(1, dtype=torch.float64, device=dev) if "sigma" in want else None
        prm = _params(sigma, p, level, route, cutoff_sigmas, exclude_self, m2l)
        ptr = lambda x: x.data_ptr() if (x is not None and x.numel()) else None
        _check(_lib.msp_fgt_backward(self._h, pw, pt, ctypes.byref(prm), pg, ptr(gw),
                                     *(ptr(g) for g in (gpos or (None, None, None))), ptr(gs), _stream()),
               "msp_fgt_backward")
        if gw is not None:
            out["w"] = gw
        if gpos is not None:
            out["pos"] = gpos
        if gs is not None:
            out["sigma"] = gs
        return out

    def debug_buffer(self, which: int) -> torch.Tensor:
        """Copy of an internal buffer: 0 moment grid, 1 Taylor grid (last expansion-route
        forward), 2 node moments, 3 node moment flags (last partner call), 4 box-pair
        attractions, 5 / 6 axon / dendrite box of each pair, 7 node of each box (last
        descent), 8 points in key order (x, y, z, staged weight), 9 inverse permutation."""
        nbytes = ctypes.c_size_t()
        _check(_lib.msp_fgt_debug_buffer(self._h, int(which), None, 0, ctypes.byref(nbytes), None),
               "msp_fgt_debug_buffer")
        if which == 3:
            out = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
        elif which == 4:
            out = torch.empty(nbytes.value // 8, dtype=torch.float64, device="cuda")
        elif which in (5, 6, 7, 9):
            out = torch.empty(nbytes.value // 4, dtype=torch.int32, device="cuda")
        else:
            out = torch.empty(nbytes.value // 4, dtype=torch.float32, device="cuda")
        _check(_lib.msp_fgt_debug_buffer(self._h, int(which), out.data_ptr(), nbytes.value,
                                         ctypes.byref(nbytes), _stream()), "msp_fgt_debug_buffer")
        return out

    def partner_probabilities(self, w, target_idx, node_id, sigma, p=8, uniforms=None,
                              exclude_self=False, level=-1, cutoff_sigmas=4.5, weights_staged=False,
                              out=None):
        """Child probabilities (msp_partner_probabilities): probs [nq, 8] and choice [nq].
        weights_staged: w is the weight array of the last forward, partner or descent
        call on this tree, unchanged since, and the weights that call gathered into
        key order are used again (MSP_WEIGHTS_STAGED).  out: (probs, choice) to fill
        (float32 [nq, 8] or [8 nq], int32 [nq]), else new tensors."""
        nq = target_idx.numel()
        pw = _ptr(w, torch.float32, self.n, "w")
        pti = _ptr(target_idx, torch.int32, nq, "target_idx")
        pni = _ptr(node_id, torch.int32, nq, "node_id")
        pu = _ptr(uniforms, torch.float32, nq, "uniforms")
        if out is None:
            probs = torch.empty(nq * 8, dtype=torch.float32, device=w.device)
            choice = torch.empty(nq, dtype=torch.int32, device=w.device)
        else:
            probs, choice = out
            _ptr(probs, torch.float32, nq * 8, "out probs")
            _ptr(choice, torch.int32, nq, "out choice")
        prm = _params(sigma, p, level, "auto", cutoff_sigmas, exclude_self)
        if weights_staged:
            prm.flags |= WEIGHTS_STAGED
        _check(_lib.msp_partner_probabilities(self._h, pw, ctypes.byref(prm), pti, pni, nq, pu,
                                              probs.data_ptr() if nq else None,
                                              choice.data_ptr() if nq else None, _stream()),
               "msp_partner_probabilities")
        return probs.view(nq, 8), choice

    def descent_step(self, w, a, S, T, step, seed, sigma, p=8, cutoff_sigmas=0.0):
        """One step of the partner descent (msp_descent_step) on host int64 arrays
        S, T of items (node id, or -(input index + 1) for a neuron).  Returns
        (S', T', requests as an int array [k, 2] of (axon, dendrite) input indices)."""
        import numpy as np
        S = np.ascontiguousarray(np.asarray(S, np.int64))
        T = np.ascontiguousarray(np.asarray(T, np.int64))
        m = S.size
        if T.size != m:
            raise ValueError("S and T must have the same length")
        pw = _ptr(w, torch.float32, self.n, "w")
        pa = _ptr(a, torch.float32, self.n, "a")
        cap = max(8 * m + 8, 64)
        while True:
            S2 = np.empty(cap, np.int64)
            T2 = np.empty(cap, np.int64)
            ra = np.empty(max(m, 1), np.int32)
            rd = np.empty(max(m, 1), np.int32)
            m2, nr = _i64(), _i64()
            prm = _params(sigma, p, -1, "auto", cutoff_sigmas, True)
            rc = _lib.msp_descent_step(self._h, pw, pa, ctypes.byref(prm), ctypes.c_uint64(int(seed)),
                                       int(step), S.ctypes.data_as(_vp), T.ctypes.data_as(_vp), m,
                                       S2.ctypes.data_as(_vp), T2.ctypes.data_as(_vp), cap, ctypes.byref(m2),
                                       ra.ctypes.data_as(_vp), rd.ctypes.data_as(_vp), ra.size, ctypes.byref(nr),
                                       _stream())
            if rc == MSP_ENOSPC and m2.value > cap:
                cap = m2.value
                continue
            _check(rc, "msp_descent_step")
            break
        req = np.stack([ra[:nr.value], rd[:nr.value]], 1).astype(np.int64)
        return S2[:m2.value].copy(), T2[:m2.value].copy(), req

    def partner_descent(self, w, a, sigma, seed, p=8, cutoff_sigmas=0.0):
        """The whole partner descent and the acceptance (msp_partner_descent).
        Returns a dict: 'axon', 'dendrite' (int32, input indices), 'accepted'
        (uint8) device tensors of the requests, and 'steps'."""
        pw = _ptr(w, torch.float32, self.n, "w")
        pa = _ptr(a, torch.float32, self.n, "a")
        dev = w.device
        n = max(self.n, 1)
        ra = torch.empty(n, dtype=torch.int32, device=dev)
        rd = torch.empty(n, dtype=torch.int32, device=dev)
        acc = torch.empty(n, dtype=torch.uint8, device=dev)
        nr, steps = _i64(), _i32()
        prm = _params(sigma, p, -1, "auto", cutoff_sigmas, True)
        _check(_lib.msp_partner_descent(self._h, pw, pa, ctypes.byref(prm), ctypes.c_uint64(int(seed)),
                                        ra.data_ptr(), rd.data_ptr(), acc.data_ptr(), ctypes.byref(nr),
                                        ctypes.byref(steps), _stream()), "msp_partner_descent")
        k = nr.value
        return {"axon": ra[:k], "dendrite": rd[:k], "accepted": acc[:k], "steps": steps.value}


def _host_array(values, ctype, n, name):
    import numpy as np
    a = np.ascontiguousarray(np.asarray(values), dtype={ctypes.c_int64: np.int64, ctypes.c_int32: np.int32,
                                                        ctypes.c_float: np.float32}[ctype])
    if a.ndim != 1 or a.size != n:
        raise ValueError(f"{name} must have {n} entries")
    return a, a.ctypes.data_as(ctypes.c_void_p)


class Batch:
    """Independent populations in one batch (msp_batch_*): population k owns the
    indices offsets[k] .. offsets[k+1]-1 of every per-point tensor."""

    def __init__(self):
        h = _vp()
        _check(_lib.msp_batch_create(ctypes.byref(h)), "msp_batch_create")
        self._h = h
        self.offsets = None

    def close(self):
        if getattr(self, "_h", None):
            _lib.msp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _set_offsets(self, offsets):
        import numpy as np
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        self.offsets = off
        self.npop = off.size - 1
        self.n = int(off[-1])
        return off

    def build(self, x, y, z, offsets, leaf_max=None, max_depth=21):
        off = self._set_offsets(offsets)
        ptrs = [_ptr(v, torch.float32, self.n, nm) for v, nm in ((x, "x"), (y, "y"), (z, "z"))]
        lm = _host_array(leaf_max, ctypes.c_int32, self.npop, "leaf_max") if leaf_max is not None else (None, None)
        _check(_lib.msp_batch_build(self._h, *ptrs, off.ctypes.data_as(_vp), self.npop, lm[1], max_depth,
                                    _stream()), "msp_batch_build")
        return self

    def autotune(self, x, y, z, offsets, w, sigmas, is_target=None, p=8, candidates=(32, 64, 128),
                 cutoff_sigmas=4.5, exclude_self=False, max_depth=21):
        """Pick (leaf size, route) per population by timing, and build with them.
        Returns (leaf sizes, route names)."""
        import numpy as np
        off = self._set_offsets(offsets)
        ptrs = [_ptr(v, torch.float32, self.n, nm) for v, nm in ((x, "x"), (y, "y"), (z, "z"))]
        pw = _ptr(w, torch.float32, self.n, "w")
        pt = _ptr(is_target, torch.uint8, self.n, "is_target")
        sg = _host_array(sigmas, ctypes.c_float, self.npop, "sigmas")
        cand = _host_array(candidates, ctypes.c_int32, len(candidates), "candidates")
        scratch = torch.empty(max(self.n, 1), dtype=torch.float32, device=w.device)
        leaf = np.zeros(self.npop, dtype=np.int32)
        route = np.zeros(self.npop, dtype=np.int32)
        prm = _params(1.0, p, -1, "auto", cutoff_sigmas, exclude_self)
        _check(_lib.msp_batch_autotune(self._h, *ptrs, off.ctypes.data_as(_vp), self.npop, pw, pt, sg[1],
                                       ctypes.byref(prm), cand[1], len(candidates), max_depth,
                                       scratch.data_ptr(), leaf.ctypes.data_as(_vp),
                                       route.ctypes.data_as(_vp), _stream()), "msp_batch_autotune")
        return leaf, [ROUTE_NAMES[int(r)] for r in route]

    def forward(self, w, sigmas, is_target=None, p=8, route="auto", cutoff_sigmas=4.5, exclude_self=False,
                out=None, m2l="mfma", use_graph=True):
        pw = _ptr(w, torch.float32, self.n, "w")
        pt = _ptr(is_target, torch.uint8, self.n, "is_target")
        sg = _host_array(sigmas, ctypes.c_float, self.npop, "sigmas")
        if out is None:
            out = torch.empty(self.n, dtype=torch.float32, device=w.device)
        po = _ptr(out, torch.float32, self.n, "out")
        prm = _params(1.0, p, -1, route, cutoff_sigmas, exclude_self, m2l)
        _check(_lib.msp_batch_forward(self._h, pw, pt, sg[1], ctypes.byref(prm), po, 1 if use_graph else 0,
                                      _stream()), "msp_batch_forward")
        return out

    def backward(self, w, grad_u, sigmas, is_target=None, p=8, route="auto", cutoff_sigmas=4.5,
                 exclude_self=False, want=("w", "pos", "sigma"), m2l="mfma", out=None, use_graph=False):
        """Per-population derivatives as Tree.backward; 'sigma' is float64 [npop].

        out: a dict returned by an earlier call, to be filled again (same addresses);
        use_graph replays a captured graph when the arguments repeat, so it pays only
        together with out."""
        n = self.n
        dev = w.device
        pw = _ptr(w, torch.float32, n, "w")
        pg = _ptr(grad_u, torch.float32, n, "grad_u")
        pt = _ptr(is_target, torch.uint8, n, "is_target")
        sg = _host_array(sigmas, ctypes.c_float, self.npop, "sigmas")
        if out is not None:
            gw = out.get("w")
            gpos = out.get("pos")
            gs = out.get("sigma_full")
            for x, nm in ((gw, "w"), *(((g, "pos") for g in gpos) if gpos else ())):
                if x is not None:
                    _ptr(x, torch.float32, n, nm)
            if gs is not None:
                _ptr(gs, torch.float64, max(self.npop, 1), "sigma")
        else:
            gw = torch.empty(n, dtype=torch.float32, device=dev) if "w" in want else None
            gpos = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(3)] if "pos" in want else None
            gs = torch.zeros(max(self.npop, 1), dtype=torch.float64, device=dev) if "sigma" in want else None
        prm = _params(1.0, p, -1, route, cutoff_sigmas, exclude_self, m2l)
        ptr = lambda x: x.data_ptr() if (x is not None and x.numel()) else None
        _check(_lib.msp_batch_backward(self._h, pw, pt, sg[1], ctypes.byref(prm), pg, ptr(gw),
                                       *(ptr(g) for g in (gpos or (None, None, None))), ptr(gs),
                                       1 if use_graph else 0, _stream()),
               "msp_batch_backward")
        res = {}
        if gw is not None:
            res["w"] = gw
        if gpos is not None:
            res["pos"] = gpos
        if gs is not None:
            res["sigma"] = gs[:self.npop]
            res["sigma_full"] = gs
        return res

    def instance_ms(self):
        """Per-population latency (ms) of the last forward, from device timestamps."""
        import numpy as np
        ms = np.zeros(max(self.npop, 1), dtype=np.float64)
        _check(_lib.msp_batch_instance_ms(self._h, ms.ctypes.data_as(_vp)), "msp_batch_instance_ms")
        return ms[:self.npop]

    def info(self) -> dict:
        npop, launches = _i32(), _i64()
        _check(_lib.msp_batch_info(self._h, ctypes.byref(npop), ctypes.byref(launches)), "msp_batch_info")
        return {"populations": npop.value, "launches_last_eager_forward": launches.value}

    def pair_count(self) -> tuple[int, float]:
        """(point pairs, span in ms) of the direct-route populations in the last forward:
        the pairs their P2P pass evaluates and the time from the first to the last work
        item of the shared persistent launch (msp_batch_pair_count)."""
        pairs, span = _i64(), ctypes.c_double()
        _check(_lib.msp_batch_pair_count(self._h, ctypes.byref(pairs), ctypes.byref(span), _stream()),
               "msp_batch_pair_count")
        return pairs.value, span.value


def build_query(n, leaf_max=64, max_depth=21) -> tuple[int, int]:
    """(tree_bytes, ws_bytes) for Tree.build_ws over n points (msp_octree_build_query)."""
    tb, wb = _sz(), _sz()
    _check(_lib.msp_octree_build_query(int(n), int(leaf_max), int(max_depth), ctypes.byref(tb), ctypes.byref(wb)),
           "msp_octree_build_query")
    return tb.value, wb.value


def build_tree(x, y, z, leaf_max=64, max_depth=21) -> Tree:
    return Tree().build(x, y, z, leaf_max, max_depth)


def direct_sum(tx, ty, tz, sx, sy, sz, w, sigma, out=None):
    """All-pairs GPU direct sum (no tree, no cutoff)."""
    nt, ns = tx.numel(), sx.numel()
    ptrs_t = [_ptr(v, torch.float32, nt, nm) for v, nm in ((tx, "tx"), (ty, "ty"), (tz, "tz"))]
    ptrs_s = [_ptr(v, torch.float32, ns, nm) for v, nm in ((sx, "sx"), (sy, "sy"), (sz, "sz"), (w, "w"))]
    if out is None:
        out = torch.empty(nt, dtype=torch.float32, device=tx.device)
    po = _ptr(out, torch.float32, nt, "out")
    _check(_lib.msp_direct_sum(*ptrs_t, nt, *ptrs_s[:3], ptrs_s[3], ns, float(sigma), po, _stream()),
           "msp_direct_sum")
    return out


class _AttractionFn(torch.autograd.Function):
    """u = msp_fgt_forward(...) with msp_fgt_backward as its adjoint."""

    @staticmethod
    def forward(ctx, x, y, z, w, sigma, is_target, opts):
        tree = opts.get("tree") or Tree()
        tree.build(x, y, z, leaf_max=opts.get("leaf_max", 64))
        s = float(sigma.item()) if isinstance(sigma, torch.Tensor) else float(sigma)
        u = tree.forward(w, is_target, sigma=s, p=opts.get("p", 8), route=opts.get("route", "auto"),
                         cutoff_sigmas=opts.get("cutoff_sigmas", 4.5),
                         exclude_self=opts.get("exclude_self", False), m2l=opts.get("m2l", "mfma"))
        ctx.tree, ctx.sigma, ctx.opts = tree, s, opts
        ctx.save_for_backward(w, is_target if is_target is not None else torch.empty(0))
        ctx.sigma_is_tensor = isinstance(sigma, torch.Tensor)
        ctx.sigma_dtype = sigma.dtype if ctx.sigma_is_tensor else None
        return u

    @staticmethod
    def backward(ctx, grad_u):
        w, tg = ctx.saved_tensors
        tg = tg if tg.numel() else None
        o = ctx.opts
        need_pos = any(ctx.needs_input_grad[:3])
        want = ["w"] if ctx.needs_input_grad[3] else []
        if need_pos:
            want.append("pos")
        if ctx.needs_input_grad[4]:
            want.append("sigma")
        if not want:
            return None, None, None, None, None, None, None
        g = ctx.tree.backward(w, grad_u.contiguous().float(), tg, sigma=ctx.sigma, p=o.get("p", 8),
                              route=o.get("route", "auto"), cutoff_sigmas=o.get("cutoff_sigmas", 4.5),
                              exclude_self=o.get("exclude_self", False), want=tuple(want),
                              m2l=o.get("m2l", "mfma"))
        gx = gy = gz = None
        if need_pos:
            gx, gy, gz = g["pos"]
        gs = None
        if "sigma" in g:
            gs = g["sigma"].to(ctx.sigma_dtype).reshape(())
        return gx, gy, gz, g.get("w"), gs, None, None


def attraction(x, y, z, w, sigma, is_target=None, p=8, route="auto", cutoff_sigmas=4.5,
               exclude_self=False, leaf_max=64, tree=None, m2l="mfma"):
    """Differentiable attraction sums u (float32 [n], 0 for non-targets).

    x, y, z, w: CUDA float32 [n]; sigma: float or 0-d CUDA tensor.  Gradients flow
    to x, y, z, w and sigma through msp_fgt_backward (no autograd tape inside)."""
    opts = dict(p=p, route=route, cutoff_sigmas=cutoff_sigmas, exclude_self=exclude_self,
                leaf_max=leaf_max, tree=tree, m2l=m2l)
    return _AttractionFn.apply(x, y, z, w, sigma, is_target, opts)
