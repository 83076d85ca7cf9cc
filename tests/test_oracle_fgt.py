"""Pins for the oracle's expansions (Eqs. (6)-(7)) and translation operators."""
import math

import numpy as np
import pytest
from numpy.polynomial import hermite as nph

import oracle
from oracle import fgt


def test_hermite_functions_against_library_polynomials():
    """h_n(x) = H_n(x) exp(-x^2) with H_n the physicists' Hermite polynomial
    (numpy.polynomial.hermite evaluates those from their coefficient series)."""
    x = np.linspace(-4, 4, 41)
    h = fgt.hermite_functions(x, 16)
    for n in range(16):
        c = np.zeros(n + 1)
        c[n] = 1.0
        np.testing.assert_allclose(h[:, n], nph.hermval(x, c) * np.exp(-x * x), rtol=1e-10, atol=1e-10)


def test_hermite_generating_function_and_derivative():
    x = np.linspace(-3, 3, 13)
    h = fgt.hermite_functions(x, 60)
    for a in (-0.7, 0.2, 1.1):
        s = sum(a ** n / math.factorial(n) * h[:, n] for n in range(60))
        np.testing.assert_allclose(s, np.exp(-(x - a) ** 2), rtol=1e-12, atol=1e-14)
    eps = 1e-6
    hp = fgt.hermite_functions(x + eps, 10)
    hm = fgt.hermite_functions(x - eps, 10)
    np.testing.assert_allclose((hp - hm)[:, :9] / (2 * eps), -h[:, 1:10], rtol=1e-6, atol=1e-7)


def test_cramer_inequality_holds_numerically():
    x = np.linspace(-12, 12, 4801)
    h = fgt.hermite_functions(x, 40)
    for n in range(40):
        bound = fgt.CRAMER_K * 2 ** (n / 2) * math.sqrt(math.factorial(n)) * np.exp(-x * x / 2)
        assert np.all(np.abs(h[:, n]) <= bound * (1 + 1e-9))


def _rand_cluster(rng, n, centre, half):
    return centre + (rng.random((n, 3)) * 2 - 1) * half


def test_hermite_expansion_converges_to_direct():
    """Eq. (7): sum_a A_a h_a((t - s_C)/sigma) reproduces the direct sum."""
    rng = np.random.default_rng(1)
    sigma = 10.0
    cs = np.array([1.0, 2.0, 3.0])
    S = _rand_cluster(rng, 40, cs, 4.0)
    w = rng.random(40) + 0.5
    T = rng.random((25, 3)) * 40 - 10
    A = fgt.p2m(S, w, cs, sigma, 24)
    np.testing.assert_allclose(fgt.m2p(A, cs, T, sigma), oracle.gauss_sum(T, S, w, sigma), rtol=1e-11, atol=1e-13)


def test_taylor_sign_two_point():
    """Two points, sigma = 1: source s = 0.3 (weight 1), target t = 2.1, source
    centre 0.1, target centre 2.0 (all on the x axis).  The direct value is
    exp(-(2.1-0.3)^2) = exp(-3.24).  The Taylor series with the sign read as
    B_b = 1/b! h_b((s - t_C)/sigma) reproduces it; with the extra (-1)^|b|
    printed in Eq. (6) the same series gives a different number."""
    s = np.array([[0.3, 0.0, 0.0]])
    t = np.array([[2.1, 0.0, 0.0]])
    tc = np.array([2.0, 0.0, 0.0])
    B = fgt.p2l(s, np.ones(1), tc, 1.0, 30)
    direct = math.exp(-3.24)
    assert fgt.l2p(B, tc, t, 1.0)[0] == pytest.approx(direct, rel=1e-12)
    sign = (-1.0) ** (np.arange(30)[:, None, None] + np.arange(30)[None, :, None] + np.arange(30)[None, None, :])
    printed = fgt.l2p(B * sign, tc, t, 1.0)[0]
    assert abs(printed - direct) > 0.03


def test_m2l_matches_m2p_and_reduces_to_p2l():
    rng = np.random.default_rng(2)
    sigma = 5.0
    cs, ct = np.array([0.0, 0.0, 0.0]), np.array([6.0, -3.0, 2.0])
    S = _rand_cluster(rng, 30, cs, 1.0)
    w = rng.random(30)
    T = _rand_cluster(rng, 20, ct, 1.0)
    p = 16
    A = fgt.p2m(S, w, cs, sigma, p)
    C = fgt.m2l(A, cs, ct, sigma)
    ref = oracle.gauss_sum(T, S, w, sigma)
    np.testing.assert_allclose(fgt.l2p(C, ct, T, sigma), ref, rtol=1e-10)
    # a single source sitting at the source centre: A = w delta_{a,0}, and M2L must equal P2L
    A1 = fgt.p2m(cs[None, :], np.array([2.5]), cs, sigma, 8)
    np.testing.assert_allclose(fgt.m2l(A1, cs, ct, sigma), fgt.p2l(cs[None, :], np.array([2.5]), ct, sigma, 8),
                               rtol=1e-12, atol=1e-15)


def test_m2l_separable_product():
    """For one pair, the 3-D operator is the tensor product of three 1-D ones:
    a product-form A (a_x x a_y x a_z) maps to the product of the 1-D images."""
    rng = np.random.default_rng(3)
    p = 6
    ax, ay, az = rng.random(p), rng.random(p), rng.random(p)
    A = np.einsum("a,b,c->abc", ax, ay, az)
    cs, ct, sigma = np.zeros(3), np.array([0.7, -1.3, 2.2]), 1.0
    C = fgt.m2l(A, cs, ct, sigma)

    def one_d(a, d):
        h = fgt.hermite_functions(np.array(d), 2 * p - 1)
        return np.array([(-1) ** b / math.factorial(b) * sum(a[k] * h[k + b] for k in range(p)) for b in range(p)])

    np.testing.assert_allclose(C, np.einsum("a,b,c->abc", one_d(ax, 0.7), one_d(ay, -1.3), one_d(az, 2.2)),
                               rtol=1e-12, atol=1e-14)


def test_m2m_exact_and_l2l_exact():
    rng = np.random.default_rng(4)
    sigma, p = 3.0, 6
    cp = np.array([1.0, 1.0, 1.0])
    cc = cp + np.array([0.5, -0.5, 0.5])
    S = _rand_cluster(rng, 25, cc, 0.5)
    w = rng.random(25)
    np.testing.assert_allclose(fgt.m2m(fgt.p2m(S, w, cc, sigma, p), cc, cp, sigma),
                               fgt.p2m(S, w, cp, sigma, p), rtol=1e-12, atol=1e-15)
    C = rng.normal(size=(p, p, p))
    T = _rand_cluster(rng, 10, cc, 0.5)
    np.testing.assert_allclose(fgt.l2p(fgt.l2l(C, cp, cc, sigma), cc, T, sigma), fgt.l2p(C, cp, T, sigma),
                               rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("p,rho", [(4, 0.1), (6, 0.2), (8, 0.3), (8, 0.45)])
def test_truncation_within_cramer_bounds(p, rho):
    """Brute force on one source box and one target box (random points,
    half-side rho*sigma): the truncated expansions stay within the bounds
    derived from Cramer's inequality."""
    rng = np.random.default_rng(p * 100 + int(rho * 100))
    sigma = 1.0
    for dist in (0.0, 1.0, 2.5):
        cs = np.zeros(3)
        ct = np.array([dist, 0.3 * dist, -0.2 * dist])
        S = _rand_cluster(rng, 50, cs, rho)
        w = rng.random(50)
        T = _rand_cluster(rng, 30, ct, rho)
        ref = oracle.gauss_sum(T, S, w, sigma)
        A = fgt.p2m(S, w, cs, sigma, p)
        err_h = np.max(np.abs(fgt.m2p(A, cs, T, sigma) - ref))
        dmin = max(0.0, np.linalg.norm(ct - cs) - 2 * math.sqrt(3) * rho)
        assert err_h <= fgt.hermite_bound(p, rho, dmin) * w.sum()
        C = fgt.m2l(A, cs, ct, sigma)
        err_ht = np.max(np.abs(fgt.l2p(C, ct, T, sigma) - ref))
        assert err_ht <= fgt.hermite_taylor_bound(p, rho, rho, np.linalg.norm(ct - cs)) * w.sum()


def test_grid_transform_accuracy():
    """Single-level all-pairs transform at p = 8 on cells of half-side <= 0.42
    sigma stays within 1e-4 per target of the direct sum."""
    rng = np.random.default_rng(6)
    n = 600
    pos = rng.random((n, 3)) * 400.0
    w = rng.integers(0, 6, n).astype(float)
    tgt = rng.integers(0, 2, n)
    side = 400.0  # root side is max extent (just under 400)
    level = 2     # cells of side ~100: half-side 50 = 0.42 sigma at sigma 120
    sigma = 120.0
    u, cells, A, C = fgt.grid_transform(pos, w, tgt, sigma, 8, level)
    m = tgt > 0
    ref = oracle.gauss_sum(pos[m], pos, w, sigma)
    assert np.max(np.abs(u[m] - ref) / ref) < 1e-4
