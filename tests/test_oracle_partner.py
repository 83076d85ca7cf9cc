"""Pins for the oracle's child probabilities and proportional choice (Algorithm 2)."""
import math

import numpy as np

import oracle
import synth
from oracle import octree, partner


def test_probabilities_brute_force_and_normalisation():
    wl = synth.uniform_box(400, extent=(300.0, 300.0, 300.0), sigma=60.0, seed=21)
    t = octree.build(wl.x, wl.y, wl.z, leaf_max=16)
    pos = wl.pos64()
    inner = np.nonzero(t.is_leaf == 0)[0]
    rng = np.random.default_rng(0)
    tq = rng.integers(0, wl.n, 12)
    nq = rng.choice(inner, 12)
    P, S, _ = partner.probabilities(t, pos, wl.w, wl.sigma, tq, nq)
    lo, side = octree.root_cube(wl.x, wl.y, wl.z)
    for q in range(12):
        X = nq[q]
        l = int(t.level[X]) + 1
        h = side / (1 << l)
        # brute force: a point is in octant d of X iff its level-(l) lattice cell is
        # (2*ix + dx, 2*iy + dy, 2*iz + dz)
        qz = np.stack([octree.quantise(pos[:, k], lo[k], 2.0 ** 21 / side) for k in range(3)], 1)
        cell = (qz >> np.uint64(21 - l)).astype(np.int64)
        base = np.array([t.ix[X], t.iy[X], t.iz[X]]) * 2
        Sbf = np.zeros(8)
        for d in range(8):
            off = np.array([(d >> 2) & 1, (d >> 1) & 1, d & 1])
            m = np.all(cell == base + off, axis=1) & (wl.w > 0)
            if m.any():
                Sbf[d] = oracle.gauss_sum(pos[tq[q]][None], pos[m], wl.w[m], wl.sigma)[0]
        np.testing.assert_allclose(S[q], Sbf, rtol=1e-12, atol=0)
        assert math.isclose(P[q].sum(), 1.0, rel_tol=1e-12)
        assert np.all(P[q][Sbf == 0] == 0)


def test_single_source_closed_form_and_choice():
    # two sources in opposite octants of the root; one target at the centre
    x = np.array([0.0, 100.0, 50.0], np.float32)
    y = np.array([0.0, 100.0, 50.0], np.float32)
    z = np.array([0.0, 100.0, 50.0], np.float32)
    w = np.array([1.0, 3.0, 0.0])
    t = octree.build(x, y, z, leaf_max=1)
    sig = 80.0
    P, S, ch = partner.probabilities(t, np.stack([x, y, z], 1), w, sig, [2], [0],
                                     uniforms=np.array([0.1], np.float32))
    d2 = 3 * 50.0 ** 2
    k = math.exp(-d2 / sig ** 2)
    # the source at the origin sits in octant 0, the one at (100,100,100) in octant 7
    assert math.isclose(S[0, 0], 1.0 * k, rel_tol=1e-12)
    assert math.isclose(S[0, 7], 3.0 * k, rel_tol=1e-12)
    assert math.isclose(P[0, 0], 0.25, rel_tol=1e-12) and math.isclose(P[0, 7], 0.75, rel_tol=1e-12)
    # r = 0.1: running sums (0.25 k, ..., k): the first to exceed 0.1 is octant 0
    assert t.digit[ch[0]] == 0
    _, _, ch2 = partner.probabilities(t, np.stack([x, y, z], 1), w, sig, [2], [0],
                                      uniforms=np.array([0.5], np.float32))
    assert t.digit[ch2[0]] == 7
    # zero total: no choice
    _, _, ch3 = partner.probabilities(t, np.stack([x, y, z], 1), np.zeros(3), sig, [2], [0],
                                      uniforms=np.array([0.5], np.float32))
    assert ch3[0] == -1
