"""Pins for the oracle's FP64 direct sum (Eq. (2) with the kernel of Eq. (8)).

Each check comes from somewhere other than the oracle's own formula: Poisson
summation on a lattice, the Gaussian-cluster integral, symmetry of the kernel,
invariances, and limits.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def test_lattice_poisson_summation():
    """A cubic lattice of unit weights at spacing a around the target gives
    prod_k theta(a/sigma) with theta(r) = sum_n exp(-r^2 n^2).  Poisson summation
    gives the dual form sqrt(pi)/r * sum_m exp(-pi^2 m^2 / r^2), computed here
    independently of the oracle; a wrong kernel scale (sigma vs sigma^2), a
    dropped coordinate or a wrong sign in the distance all break it."""
    a, sigma = 30.0, 40.0
    r = a / sigma
    m = np.arange(-12, 13)
    g = np.stack(np.meshgrid(m, m, m, indexing="ij"), axis=-1).reshape(-1, 3) * a
    t = np.array([[0.0, 0.0, 0.0]])
    u = oracle.gauss_sum(t, g, np.ones(len(g)), sigma)[0]
    dual = math.sqrt(math.pi) / r * sum(math.exp(-math.pi ** 2 * k * k / (r * r)) for k in range(-20, 21))
    assert u == pytest.approx(dual ** 3, rel=1e-12)
    # shifted target: theta with characteristic x: sum_n exp(-(n r - x)^2), dual
    # sqrt(pi)/r sum_m exp(-pi^2 m^2/r^2) cos(2 pi m x / r)
    x = (7.0 / sigma, -11.0 / sigma, 3.0 / sigma)
    t2 = np.array([[7.0, -11.0, 3.0]])
    u2 = oracle.gauss_sum(t2, g, np.ones(len(g)), sigma)[0]
    prod = 1.0
    for xk in x:
        prod *= math.sqrt(math.pi) / r * sum(
            math.exp(-math.pi ** 2 * k * k / (r * r)) * math.cos(2 * math.pi * k * xk / r)
            for k in range(-20, 21))
    assert u2 == pytest.approx(prod, rel=1e-12)


def test_gaussian_cluster_integral():
    """N sources ~ N(mu, s^2 I) with weight w: E[u(t)] =
    N w (sigma^2/(sigma^2+2 s^2))^{3/2} exp(-|t-mu|^2/(sigma^2+2 s^2)).
    Monte Carlo with 4e5 samples; tolerance ~ 5 standard errors."""
    rng = np.random.default_rng(7)
    N, s, sigma, wv = 400_000, 50.0, 200.0, 2.5
    mu = np.array([1000.0, 2000.0, 500.0])
    src = mu + rng.normal(0, s, size=(N, 3))
    t = np.array([[1000.0, 2000.0, 500.0], [1100.0, 1950.0, 560.0]])
    u = oracle.gauss_sum(t, src, np.full(N, wv), sigma)
    v = sigma ** 2 + 2 * s ** 2
    expect = N * wv * (sigma ** 2 / v) ** 1.5 * np.exp(-np.sum((t - mu) ** 2, axis=1) / v)
    # per-sample spread of the kernel is below its mean here, so SE < mean/sqrt(N)
    np.testing.assert_allclose(u, expect, rtol=5 / math.sqrt(N))


def test_two_point_and_role_symmetry():
    rng = np.random.default_rng(3)
    T = rng.random((200, 3)) * 300
    S = rng.random((150, 3)) * 300
    a = rng.integers(0, 6, 200).astype(float)
    w = rng.integers(0, 6, 150).astype(float)
    sigma = 75.0
    u = oracle.gauss_sum(T, S, w, sigma)
    v = oracle.gauss_sum(S, T, a, sigma)
    assert np.dot(a, u) == pytest.approx(np.dot(w, v), rel=1e-12)


def test_linearity_translation_scaling():
    rng = np.random.default_rng(4)
    T = rng.random((64, 3)) * 500
    S = rng.random((300, 3)) * 500
    w1 = rng.random(300)
    w2 = rng.random(300)
    sig = 120.0
    u1 = oracle.gauss_sum(T, S, w1, sig)
    u2 = oracle.gauss_sum(T, S, w2, sig)
    u12 = oracle.gauss_sum(T, S, 2 * w1 - 3 * w2, sig)
    np.testing.assert_allclose(u12, 2 * u1 - 3 * u2, rtol=1e-10, atol=1e-12)
    shift = np.array([123.25, -77.5, 1000.0])
    np.testing.assert_allclose(oracle.gauss_sum(T + shift, S + shift, w1, sig), u1, rtol=1e-12)
    np.testing.assert_allclose(oracle.gauss_sum(T * 2.0, S * 2.0, w1, sig * 2.0), u1, rtol=1e-12)


def test_large_sigma_limit():
    rng = np.random.default_rng(5)
    S = rng.random((500, 3)) * 100
    T = rng.random((5, 3)) * 100
    w = rng.random(500)
    sigma = 1e5
    u = oracle.gauss_sum(T, S, w, sigma)
    dmax2 = 3 * 100.0 ** 2
    assert np.all(np.abs(u - w.sum()) <= w.sum() * dmax2 / sigma ** 2)


def test_exclude_self_and_union_set():
    """A neuron in both sets: skipping itself removes exactly w_i * K(0) = w_i."""
    wl = synth.uniform_box(300, sigma=80.0, seed=11)
    tgt = np.nonzero(wl.a > 0)[0]
    u_in = oracle.attraction(wl, tgt)
    u_ex = oracle.attraction(wl, tgt, exclude_self=True)
    np.testing.assert_allclose(u_in - u_ex, wl.w[tgt], rtol=1e-9, atol=1e-12)


def test_empty_inputs():
    assert oracle.gauss_sum(np.zeros((0, 3)), np.zeros((5, 3)), np.ones(5), 1.0).shape == (0,)
    assert oracle.gauss_sum(np.zeros((3, 3)), np.zeros((0, 3)), np.ones(0), 1.0).tolist() == [0, 0, 0]
    with pytest.raises(ValueError):
        oracle.gauss_sum(np.zeros((1, 3)), np.zeros((1, 3)), np.ones(1), 0.0)


def test_gradients_against_finite_differences():
    """Direct-sum derivatives vs central differences of the oracle's own sum
    (the difference quotient is computed from the sum, not from the derivative
    formulas)."""
    rng = np.random.default_rng(9)
    T = rng.random((20, 3)) * 200
    S = rng.random((30, 3)) * 200
    w = rng.random(30) + 0.5
    g = rng.random(20) + 0.5
    sigma = 60.0
    d = oracle.gauss_grad(T, g, S, w, sigma)

    def L(T_, S_, w_, s_):
        return float(np.dot(g, oracle.gauss_sum(T_, S_, w_, s_)))

    h = 1e-3
    for i, k in [(0, 0), (5, 1), (19, 2)]:
        Tp, Tm = T.copy(), T.copy()
        Tp[i, k] += h
        Tm[i, k] -= h
        assert d["t"][i, k] == pytest.approx((L(Tp, S, w, sigma) - L(Tm, S, w, sigma)) / (2 * h), rel=1e-6, abs=1e-9)
    for j, k in [(0, 0), (7, 1), (29, 2)]:
        Sp, Sm = S.copy(), S.copy()
        Sp[j, k] += h
        Sm[j, k] -= h
        assert d["s"][j, k] == pytest.approx((L(T, Sp, w, sigma) - L(T, Sm, w, sigma)) / (2 * h), rel=1e-6, abs=1e-9)
    for j in [0, 13]:
        wp = w.copy()
        wp[j] += 1.0
        assert d["w"][j] == pytest.approx(L(T, S, wp, sigma) - L(T, S, w, sigma), rel=1e-10)
    hs = 1e-4
    assert d["sigma"] == pytest.approx((L(T, S, w, sigma + hs) - L(T, S, w, sigma - hs)) / (2 * hs), rel=1e-6)
