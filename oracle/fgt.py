"""Oracle expansions of the Gaussian sum (fast Gauss transform), FP64, numpy.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Notation follows the paper's section on the mathematics of the method
(Eqs. (3)-(7)): multi-indices alpha = (n1, n2, n3), |alpha|, alpha!, t^alpha;
delta = sigma^2 so that sqrt(delta) = sigma.  A multi-index runs over the
tensor range 0 <= n_k < p (p terms per axis, p^3 coefficients).

Hermite functions (the h(alpha, x) the paper takes from Greengard and Strain):
    h_n(x) = (-1)^n d^n/dx^n exp(-x^2) = H_n(x) exp(-x^2),
    h_0 = exp(-x^2), h_1 = 2x exp(-x^2), h_{n+1} = 2x h_n - 2n h_{n-1},
    h_alpha(x) = h_{n1}(x_1) h_{n2}(x_2) h_{n3}(x_3).
With it exp(-(x - a)^2) = sum_n a^n / n! h_n(x) (generating function) and
h_n' = -h_{n+1}.

Operators (c_S a source-box centre, c_T a target-box centre, y = (t - c)/sigma):
  P2M  (Eq. (7))  A_a = 1/a! sum_j w_j ((s_j - c_S)/sigma)^a
  M2P  (Eq. (7))  u(t) = sum_a A_a h_a((t - c_S)/sigma)
  P2L  (Eq. (6), sign read so that the series is exact, see below)
                  B_b = 1/b! sum_j w_j h_b((s_j - c_T)/sigma)
  L2P  (Eq. (6))  u(t) = sum_b B_b ((t - c_T)/sigma)^b
  M2L  (derived)  C_b = (-1)^|b| / b! sum_a A_a h_{a+b}((c_T - c_S)/sigma)
  M2M  (derived)  A'_a = sum_{g<=a} A_g d^(a-g) / (a-g)!,  d = (c_child - c_parent)/sigma
  L2L  (derived)  C'_b = sum_{g>=b} C_g binom(g, b) d^(g-b),  d = (c_child - c_parent)/sigma

Eq. (6) as printed carries (-1)^|b| in front of h_b((s_j - t_C)/sqrt(delta));
with h as above that factor belongs with the argument (t_C - s_j).  The
reading used here, B_b = 1/b! sum_j w_j h_b((s_j - t_C)/sigma), is the one under
which the Taylor series reproduces the direct sum; tests pin it with a
two-point case.  M2L, M2M and L2L are not printed in the paper (it evaluates
both expansions straight from the points); they follow from the generating
function and from the binomial theorem.
"""
from __future__ import annotations

import math

import numpy as np

CRAMER_K = 1.086435


def hermite_functions(x: np.ndarray, nmax: int) -> np.ndarray:
    """h_n(x) for n = 0..nmax-1; result shape x.shape + (nmax,)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty(x.shape + (max(nmax, 1),), np.float64)
    out[..., 0] = np.exp(-x * x)
    if nmax > 1:
        out[..., 1] = 2.0 * x * out[..., 0]
    for n in range(1, nmax - 1):
        out[..., n + 1] = 2.0 * x * out[..., n] - 2.0 * n * out[..., n - 1]
    return out[..., :nmax]


def _fact(p: int) -> np.ndarray:
    return np.array([math.factorial(k) for k in range(p)], np.float64)


def _powers(v: np.ndarray, p: int) -> np.ndarray:
    """v^k for k = 0..p-1, shape v.shape + (p,)."""
    v = np.asarray(v, np.float64)
    out = np.ones(v.shape + (p,), np.float64)
    for k in range(1, p):
        out[..., k] = out[..., k - 1] * v
    return out


def p2m(src: np.ndarray, w: np.ndarray, centre: np.ndarray, sigma: float, p: int) -> np.ndarray:
    """Hermite moments A[ax, ay, az] of the weighted points src[j] about centre."""
    z = (np.asarray(src, np.float64) - centre) / sigma
    X, Y, Zp = _powers(z[:, 0], p), _powers(z[:, 1], p), _powers(z[:, 2], p)
    f = _fact(p)
    A = np.einsum("j,ja,jb,jc->abc", np.asarray(w, np.float64), X, Y, Zp)
    return A / (f[:, None, None] * f[None, :, None] * f[None, None, :])


def m2p(A: np.ndarray, centre: np.ndarray, tgt: np.ndarray, sigma: float) -> np.ndarray:
    """Evaluate a Hermite expansion at points tgt (Eq. (7))."""
    p = A.shape[0]
    y = (np.asarray(tgt, np.float64) - centre) / sigma
    Hx, Hy, Hz = (hermite_functions(y[:, k], p) for k in range(3))
    return np.einsum("abc,ta,tb,tc->t", A, Hx, Hy, Hz)


def p2l(src: np.ndarray, w: np.ndarray, centre: np.ndarray, sigma: float, p: int) -> np.ndarray:
    """Taylor coefficients B[bx, by, bz] about a target centre (Eq. (6), sign as read above)."""
    z = (np.asarray(src, np.float64) - centre) / sigma
    Hx, Hy, Hz = (hermite_functions(z[:, k], p) for k in range(3))
    f = _fact(p)
    B = np.einsum("j,ja,jb,jc->abc", np.asarray(w, np.float64), Hx, Hy, Hz)
    return B / (f[:, None, None] * f[None, :, None] * f[None, None, :])


def l2p(B: np.ndarray, centre: np.ndarray, tgt: np.ndarray, sigma: float) -> np.ndarray:
    """Evaluate a Taylor expansion at points tgt (Eq. (6))."""
    p = B.shape[0]
    y = (np.asarray(tgt, np.float64) - centre) / sigma
    X, Y, Zp = _powers(y[:, 0], p), _powers(y[:, 1], p), _powers(y[:, 2], p)
    return np.einsum("abc,ta,tb,tc->t", B, X, Y, Zp)


def m2l(A: np.ndarray, c_src: np.ndarray, c_tgt: np.ndarray, sigma: float) -> np.ndarray:
    """Hermite expansion about c_src -> Taylor expansion about c_tgt.

    C_b = (-1)^|b| / b! * sum_a A_a h_{a+b}(d), d = (c_tgt - c_src)/sigma, written
    as the full double sum over a and b (p^3 x p^3 matrix)."""
    p = A.shape[0]
    d = (np.asarray(c_tgt, np.float64) - np.asarray(c_src, np.float64)) / sigma
    h = [hermite_functions(np.array(d[k]), 2 * p - 1) for k in range(3)]
    f = _fact(p)
    idx = np.arange(p)
    # full operator M[(bx,by,bz),(ax,ay,az)]
    hx = h[0][idx[:, None] + idx[None, :]]   # [b, a]
    hy = h[1][idx[:, None] + idx[None, :]]
    hz = h[2][idx[:, None] + idx[None, :]]
    M = np.einsum("Aa,Bb,Cc->ABCabc", hx, hy, hz).reshape(p ** 3, p ** 3)
    b = np.stack(np.meshgrid(idx, idx, idx, indexing="ij"), axis=-1).reshape(-1, 3)
    sign = (-1.0) ** b.sum(axis=1)
    bfact = f[b[:, 0]] * f[b[:, 1]] * f[b[:, 2]]
    C = (sign / bfact) * (M @ A.reshape(-1))
    return C.reshape(p, p, p)


def m2m(A: np.ndarray, c_child: np.ndarray, c_parent: np.ndarray, sigma: float) -> np.ndarray:
    """Shift Hermite moments from a child centre to its parent's centre."""
    p = A.shape[0]
    d = (np.asarray(c_child, np.float64) - np.asarray(c_parent, np.float64)) / sigma
    f = _fact(p)
    out = np.zeros_like(A, dtype=np.float64)
    for ax in range(p):
        for ay in range(p):
            for az in range(p):
                acc = 0.0
                for gx in range(ax + 1):
                    for gy in range(ay + 1):
                        for gz in range(az + 1):
                            acc += (A[gx, gy, gz]
                                    * d[0] ** (ax - gx) / f[ax - gx]
                                    * d[1] ** (ay - gy) / f[ay - gy]
                                    * d[2] ** (az - gz) / f[az - gz])
                out[ax, ay, az] = acc
    return out


def l2l(C: np.ndarray, c_parent: np.ndarray, c_child: np.ndarray, sigma: float) -> np.ndarray:
    """Re-centre a Taylor polynomial from the parent's centre to a child's."""
    p = C.shape[0]
    d = (np.asarray(c_child, np.float64) - np.asarray(c_parent, np.float64)) / sigma
    out = np.zeros_like(C, dtype=np.float64)
    for bx in range(p):
        for by in range(p):
            for bz in range(p):
                acc = 0.0
                for gx in range(bx, p):
                    for gy in range(by, p):
                        for gz in range(bz, p):
                            acc += (C[gx, gy, gz]
                                    * math.comb(gx, bx) * d[0] ** (gx - bx)
                                    * math.comb(gy, by) * d[1] ** (gy - by)
                                    * math.comb(gz, bz) * d[2] ** (gz - bz))
                out[bx, by, bz] = acc
    return out


# ---------------------------------------------------------------------------------------
# Truncation bounds (Cramer's inequality |h_n(x)| <= K 2^(n/2) sqrt(n!) exp(-x^2/2))
# ---------------------------------------------------------------------------------------

def _series(x: float, start: int, terms: int = 200) -> float:
    """sum_{N >= start} x^N / sqrt(N!)"""
    acc = 0.0
    for N in range(start, start + terms):
        acc += math.exp(N * math.log(x) - 0.5 * math.lgamma(N + 1)) if x > 0 else (1.0 if N == 0 else 0.0)
    return acc


def hermite_bound(p: int, rho_s: float, dist_sigma: float = 0.0) -> float:
    """Bound per unit |weight| on |M2P_p(t) - direct(t)| for sources within rho_s*sigma
    (per axis) of the centre and a target at distance dist_sigma*sigma from it.

    Per axis the terms are a^n/n! h_n(X) with |a| <= rho_s; the tensor range
    misses some term iff some axis has n >= p, so the error is at most
    3 * T * F^2 with T, F the tail and the full per-axis sums."""
    x = math.sqrt(2.0) * rho_s
    T = CRAMER_K * _series(x, p)
    F = CRAMER_K * _series(x, 0)
    return 3.0 * T * F * F * math.exp(-0.5 * dist_sigma ** 2)


def hermite_taylor_bound(p: int, rho_s: float, rho_t: float, centre_dist_sigma: float = 0.0) -> float:
    """Bound per unit |weight| on |L2P(M2L(P2M)) - direct| for one source box
    (half-side rho_s*sigma) and one target box (half-side rho_t*sigma) whose
    centres are centre_dist_sigma*sigma apart.

    Per axis the double series a^n/n! (-y)^m/m! h_{n+m}(X0) with |a| <= rho_s,
    |y| <= rho_t sums, by Cramer's inequality and the binomial theorem, to at
    most K e^{-X0^2/2} sum_N (sqrt2 (rho_s+rho_t))^N / sqrt(N!); the dropped
    terms all have n + m >= p."""
    x = math.sqrt(2.0) * (rho_s + rho_t)
    T = CRAMER_K * _series(x, p)
    F = CRAMER_K * _series(x, 0)
    return 3.0 * T * F * F * math.exp(-0.5 * centre_dist_sigma ** 2)


# ---------------------------------------------------------------------------------------
# Reference single-level transform on a uniform grid of cells (small inputs only)
# ---------------------------------------------------------------------------------------

def cell_centre(lo: np.ndarray, side: float, level: int, ijk: np.ndarray) -> np.ndarray:
    h = side / (1 << level)
    return np.asarray(lo, np.float64) + (np.asarray(ijk, np.float64) + 0.5) * h


def grid_transform(pos: np.ndarray, w: np.ndarray, is_target: np.ndarray, sigma: float, p: int,
                   level: int):
    """All-pairs Hermite -> Taylor transform over the occupied cells of one level.

    Each point goes to its cell at `level` of the octree's root cube (the cell
    of a point is the level-`level` prefix of its Morton key); each occupied
    cell gets P2M moments about its geometric centre; every cell holding
    targets receives M2L from every occupied cell (no cutoff, the cell itself
    included); targets evaluate their cell's Taylor series.  Returns
    (u, cells, A, C) with cells the sorted unique integer cell coordinates."""
    from . import octree
    pos = np.asarray(pos, np.float64)
    lo, side = octree.root_cube(pos[:, 0], pos[:, 1], pos[:, 2])
    scale = float(2 ** octree.DEPTH) / side
    shift = np.uint64(octree.DEPTH - level)
    ijk = np.stack([(octree.quantise(pos[:, k], lo[k], scale) >> shift).astype(np.int64)
                    for k in range(3)], axis=1)
    cells, inv = np.unique(ijk, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    nc = cells.shape[0]
    centres = np.array([cell_centre(lo, side, level, c) for c in cells])
    A = np.zeros((nc, p, p, p))
    for c in range(nc):
        m = inv == c
        A[c] = p2m(pos[m], w[m], centres[c], sigma, p)
    C = np.zeros((nc, p, p, p))
    u = np.zeros(pos.shape[0])
    for t in range(nc):
        m = (inv == t) & (np.asarray(is_target) > 0)
        if not m.any():
            continue
        for s in range(nc):
            C[t] += m2l(A[s], centres[s], centres[t], sigma)
        u[m] = l2p(C[t], centres[t], pos[m], sigma)
    return u, cells, A, C
