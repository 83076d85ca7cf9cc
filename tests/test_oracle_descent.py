"""Pins for the oracle of the partner descent (Algorithm 1 with Algorithm 2's
proportional choice, and the acceptance at the dendrites)."""
import math

import numpy as np

import synth
from oracle import descent, octree


def test_splitmix64_published_outputs():
    # first outputs of the SplitMix64 reference implementation for states 0 and 1234567
    s, out = 0, []
    for _ in range(3):
        s, v = descent.splitmix64_next(s)
        out.append(v)
    assert out == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    s, out = 1234567, []
    for _ in range(3):
        s, v = descent.splitmix64_next(s)
        out.append(v)
    assert out == [6457827717110365317, 3203168211198807973, 9817491932198370423]


def test_uniform_range_and_spread():
    u = np.array([descent.uniform(7, 3, k) for k in range(-20000, 20000)])
    assert np.all(u >= 0.0) and np.all(u < 1.0)
    assert np.unique(u).size == u.size
    # Kolmogorov-Smirnov distance of 40,000 draws from U[0,1)
    s = np.sort(u)
    d = np.max(np.abs(s - (np.arange(1, s.size + 1) - 0.5) / s.size))
    assert d < 1.63 / math.sqrt(s.size)      # 1 % level
    # different steps and seeds give unrelated draws
    assert descent.uniform(7, 3, 5) != descent.uniform(7, 4, 5) != descent.uniform(8, 3, 5)


def test_choice_frequencies_are_proportional():
    rng = np.random.default_rng(3)
    for _ in range(20):
        v = rng.random(rng.integers(1, 9)) * (rng.random(1) < 0.8)
        v[rng.random(v.size) < 0.3] = 0.0
        total = v.sum()
        if total == 0:
            assert descent.choose(v, 0.3) == -1
            continue
        n = 20000
        ks = np.array([descent.choose(v, (m + 0.5) / n) for m in range(n)])
        assert np.all(v[ks] > 0)
        freq = np.bincount(ks, minlength=v.size) / n
        np.testing.assert_allclose(freq, v / total, atol=2.0 / n)


def _tiny(n, seed, leaf_max=4, sigma=80.0):
    wl = synth.uniform_box(n, extent=(300.0, 300.0, 300.0), sigma=sigma, seed=seed)
    t = octree.build(wl.x, wl.y, wl.z, leaf_max=leaf_max)
    return wl, t, descent.Descent(t, wl.pos64(), wl.a, wl.w, wl.sigma)


def test_attraction_brute_force():
    wl, t, d = _tiny(60, 11)
    pos = wl.pos64()
    rng = np.random.default_rng(1)
    items = list(range(t.n_nodes)) + [-(i + 1) for i in range(wl.n)]
    for _ in range(40):
        S, C = (items[k] for k in rng.integers(0, len(items), 2))
        ref = 0.0
        for i in d.neurons(S):
            for j in d.neurons(C):
                if i != j:
                    r2 = float(np.sum((pos[i] - pos[j]) ** 2))
                    ref += float(wl.a[i]) * float(wl.w[j]) * math.exp(-r2 / float(wl.sigma) ** 2)
        assert math.isclose(d.att(S, C), ref, rel_tol=1e-12, abs_tol=1e-300)


def test_children_partition_points():
    wl, t, d = _tiny(200, 12)
    for v in range(t.n_nodes):
        ch = d.children(v)
        got = np.sort(np.concatenate([d.neurons(c) for c in ch]))
        assert np.array_equal(got, np.sort(d.neurons(v)))
        if t.n_children[v] > 0:
            assert [int(t.digit[c]) for c in ch] == sorted(int(t.digit[c]) for c in ch)


def test_two_neurons_form_one_request():
    x = np.array([0.0, 50.0], np.float32)
    y = np.zeros(2, np.float32)
    z = np.zeros(2, np.float32)
    t = octree.build(x, y, z, leaf_max=4)
    pos = np.stack([x, y, z], 1).astype(np.float64)
    d = descent.Descent(t, pos, np.array([1.0, 0.0]), np.array([0.0, 2.0]), 100.0)
    assert d.run(seed=5) == [(0, 1)]
    # no dendrites anywhere: no request
    d0 = descent.Descent(t, pos, np.array([1.0, 0.0]), np.array([0.0, 0.0]), 100.0)
    assert d0.run(seed=5) == []


def test_single_axon_lands_proportionally():
    # one axon neuron: the probabilities telescope over the levels, so the dendrite
    # reached is drawn with probability w_j K(t, s_j) / sum_k w_k K(t, s_k)
    wl = synth.uniform_box(40, extent=(200.0, 200.0, 200.0), sigma=90.0, seed=13)
    a = np.zeros(wl.n)
    a[7] = 2.0
    w = np.where(np.arange(wl.n) == 7, 0.0, 1.0 + (np.arange(wl.n) % 3))
    t = octree.build(wl.x, wl.y, wl.z, leaf_max=4)
    pos = wl.pos64()
    d = descent.Descent(t, pos, a, w, wl.sigma)
    k = w * np.exp(-np.sum((pos - pos[7]) ** 2, 1) / wl.sigma ** 2)
    p = k / k.sum()
    n = 3000
    hits = np.zeros(wl.n)
    for seed in range(n):
        req = d.run(seed)
        assert len(req) == 1 and req[0][0] == 7
        hits[req[0][1]] += 1
    assert hits[7] == 0
    m = p > 0
    chi2 = float(np.sum((hits[m] - n * p[m]) ** 2 / (n * p[m])))
    assert chi2 < 85.0        # 38 degrees of freedom; p-value about 2e-5


def test_every_axon_neuron_requests_at_most_once():
    wl, t, d = _tiny(150, 14, leaf_max=8)
    req = d.run(seed=9)
    axons = [i for i, _ in req]
    assert len(axons) == len(set(axons))
    for i, j in req:
        assert wl.a[i] > 0 and wl.w[j] > 0 and i != j
    assert d.run(seed=9) == req
    assert d.run(seed=10) != req


def test_acceptance_rules():
    rng = np.random.default_rng(4)
    w = rng.integers(0, 4, 30).astype(np.float64)
    req = [(int(i), int(j)) for i, j in zip(rng.permutation(200)[:120], rng.integers(0, 30, 120))]
    acc = descent.accept(req, w, seed=21)
    for j in range(30):
        ks = [k for k, r in enumerate(req) if r[1] == j]
        took = [k for k in ks if acc[k]]
        assert len(took) == min(len(ks), int(w[j]))
        if took and len(took) < len(ks):
            worst = max(descent.priority(21, req[k][0]) for k in took)
            best_rejected = min(descent.priority(21, req[k][0]) for k in ks if not acc[k])
            assert worst < best_rejected
