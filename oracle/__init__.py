"""The oracle: plain, slow, obviously correct CPU implementations of what the
hot path computes.  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the bench's CPU-baseline leg may import or
call anything here.  The product library (the HIP path and its Python binding)
shares no code with this package and never calls it.

Contents
  direct.c / gauss_sum, gauss_grad   FP64 direct Gaussian sums and their
                                     derivatives (Eq. (2) with the kernel of Eq. (8))
  octree.py                          Morton keys, stable sort, adaptive node table
                                     (section "A Distributed Octree")
  fgt.py                             FP64 Hermite / Taylor expansions and the
                                     translation operators (Eqs. (6)-(7)), truncation bounds
  partner.py                         child probabilities and proportional choice
                                     (Algorithm 2)
  descent.py                         the partner descent over pairs of items
                                     (Algorithm 1 with Algorithm 2's choice), the
                                     counter-based generator it draws from, and the
                                     acceptance of requests at the dendrites
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile direct.c with gcc (FP64, OpenMP, no FMA contraction)."""
    src = os.path.join(_HERE, "direct.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC",
                               src, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_SO)
        d = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        lib.oracle_gauss_sum.argtypes = [i64, d, d, d, ctypes.POINTER(i64), i64, d, d, d, d,
                                         ctypes.c_double, d, ctypes.c_int]
        lib.oracle_gauss_sum.restype = ctypes.c_int
        lib.oracle_gauss_grad.argtypes = [i64, d, d, d, d, i64, d, d, d, d, ctypes.c_double,
                                          d, d, d, d, ctypes.c_int]
        lib.oracle_gauss_grad.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def gauss_sum(tgt, src, w, sigma, self_idx=None, threads: int = 0) -> np.ndarray:
    """u[i] = sum_j w[j] exp(-|tgt[i] - src[j]|^2 / sigma^2) in FP64.

    tgt: (nt, 3), src: (ns, 3) arrays (any float dtype; widened exactly).
    self_idx: optional int array (nt,) naming one source each target skips (-1: none)."""
    lib = _load()
    tgt = _f64(tgt).reshape(-1, 3)
    src = _f64(src).reshape(-1, 3)
    tx, ty, tz = (_f64(tgt[:, k]) for k in range(3))
    sx, sy, sz = (_f64(src[:, k]) for k in range(3))
    ww = _f64(w).reshape(-1)
    assert ww.shape[0] == src.shape[0]
    out = np.zeros(tgt.shape[0], np.float64)
    sp = None
    if self_idx is not None:
        si = np.ascontiguousarray(np.asarray(self_idx, np.int64))
        sp = si.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    rc = lib.oracle_gauss_sum(tgt.shape[0], _dp(tx), _dp(ty), _dp(tz), sp, src.shape[0], _dp(sx),
                              _dp(sy), _dp(sz), _dp(ww), float(sigma), _dp(out), int(threads))
    if rc != 0:
        raise ValueError("oracle_gauss_sum: bad arguments")
    return out


def gauss_grad(tgt, g, src, w, sigma, threads: int = 0, want=("w", "s", "t", "sigma")):
    """Direct-sum derivatives of L = sum_i g_i u(t_i); returns a dict with the
    requested entries: 'w' (ns,), 's' (ns,3), 't' (nt,3), 'sigma' (scalar)."""
    lib = _load()
    tgt = _f64(tgt).reshape(-1, 3)
    src = _f64(src).reshape(-1, 3)
    tx, ty, tz = (_f64(tgt[:, k]) for k in range(3))
    sx, sy, sz = (_f64(src[:, k]) for k in range(3))
    gg = _f64(g).reshape(-1)
    ww = _f64(w).reshape(-1)
    nt, ns = tgt.shape[0], src.shape[0]
    gw = np.zeros(ns) if "w" in want else None
    gs = np.zeros(3 * ns) if "s" in want else None
    gt = np.zeros(3 * nt) if "t" in want else None
    gsig = np.zeros(nt) if "sigma" in want else None
    rc = lib.oracle_gauss_grad(nt, _dp(tx), _dp(ty), _dp(tz), _dp(gg), ns, _dp(sx), _dp(sy),
                               _dp(sz), _dp(ww), float(sigma), _dp(gw), _dp(gs), _dp(gt),
                               _dp(gsig), int(threads))
    if rc != 0:
        raise ValueError("oracle_gauss_grad: bad arguments")
    out = {}
    if gw is not None:
        out["w"] = gw
    if gs is not None:
        out["s"] = gs.reshape(ns, 3)
    if gt is not None:
        out["t"] = gt.reshape(nt, 3)
    if gsig is not None:
        out["sigma"] = float(np.sum(gsig))
    return out


def attraction(wl, target_idx=None, threads: int = 0, exclude_self: bool = False) -> np.ndarray:
    """u for a synth.Workload at the given target indices (default: all neurons
    with a > 0); sources are all neurons with w > 0 in index order."""
    pos = wl.pos64()
    if target_idx is None:
        target_idx = np.nonzero(wl.a > 0)[0]
    target_idx = np.asarray(target_idx, np.int64)
    src_idx = np.nonzero(wl.w > 0)[0]
    self_idx = None
    if exclude_self:
        where = np.full(wl.n, -1, np.int64)
        where[src_idx] = np.arange(src_idx.size)
        self_idx = where[target_idx]
    return gauss_sum(pos[target_idx], pos[src_idx], wl.w[src_idx], wl.sigma, self_idx, threads)
