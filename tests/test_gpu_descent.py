"""Partner descent on the GPU (Algorithm 1 with Algorithm 2's proportional choice,
and the acceptance at the dendrites) against the FP64 oracle: step by step on
the same frontier, whole descents, the landing distribution of a single axon,
and the invariants of a larger run."""
import numpy as np
import pytest

import synth
from oracle import descent, octree

pytestmark = pytest.mark.gpu

TIE = 1e-4   # a choice closer than this (relative to the total) to a boundary may flip


def _setup(wl, leaf_max):
    import torch
    import paper_2301_10570_amd as msp
    T = lambda v: torch.from_numpy(np.ascontiguousarray(v)).cuda()
    tree = msp.build_tree(T(wl.x), T(wl.y), T(wl.z), leaf_max=leaf_max)
    ot = octree.build(wl.x, wl.y, wl.z, leaf_max=leaf_max)
    od = descent.Descent(ot, wl.pos64(), wl.a, wl.w, wl.sigma)
    return tree, od, T(wl.w), T(wl.a)


def _pairs(S, T):
    return sorted(zip((int(x) for x in S), (int(y) for y in T)))


@pytest.mark.parametrize("leaf_max", [8, 32])
def test_steps_match_oracle(leaf_max):
    wl = synth.uniform_box(1500, extent=(400.0, 400.0, 400.0), sigma=90.0, seed=31)
    print(f"descent steps, 1500 neurons, leaf_max {leaf_max}", flush=True)
    tree, od, w, a = _setup(wl, leaf_max)
    S, T = np.array([0]), np.array([0])
    seed, total_req, flips = 77, 0, 0
    for step in range(60):
        if S.size == 0:
            break
        S2, T2, req = tree.descent_step(w, a, S, T, step, seed, wl.sigma, cutoff_sigmas=0.0)
        onxt, oreq, dec = od.step(list(zip(S.tolist(), T.tolist())), step, seed)
        assert sorted(map(tuple, req.tolist())) == sorted(oreq)
        g, o = set(_pairs(S2, T2)), set(onxt)
        if g != o:
            diff = len(g ^ o) // 2
            near = sum(1 for _, _, m in dec if m < TIE)
            assert diff <= near, (step, diff, near)
            flips += diff
        total_req += len(oreq)
        S, T = S2, T2
    assert S.size == 0
    assert total_req > 50
    print(f"  requests {total_req}, near-tie flips {flips}")


def _oracle_run(od, seed):
    frontier, req, mmin = [(0, 0)], [], np.inf
    for step in range(200):
        if not frontier:
            break
        frontier, r, dec = od.step(frontier, step, seed)
        req += r
        if dec:
            mmin = min(mmin, min(m for _, _, m in dec))
    return sorted(req), mmin


def test_whole_descent_and_acceptance_match_oracle():
    wl = synth.uniform_box(900, extent=(300.0, 300.0, 300.0), sigma=70.0, seed=32)
    print("whole descent, 900 neurons", flush=True)
    tree, od, w, a = _setup(wl, 16)
    # a seed whose oracle choices all stay clear of the boundaries (decided by the oracle)
    for seed in range(20):
        oreq, mmin = _oracle_run(od, seed)
        if mmin >= TIE:
            break
    assert mmin >= TIE
    got = tree.partner_descent(w, a, wl.sigma, seed, cutoff_sigmas=0.0)
    ga = got["axon"].cpu().numpy()
    gd = got["dendrite"].cpu().numpy()
    gacc = got["accepted"].cpu().numpy().astype(bool)
    assert sorted(zip(ga.tolist(), gd.tolist())) == oreq
    oacc = descent.accept(list(zip(ga.tolist(), gd.tolist())), wl.w, seed)
    np.testing.assert_array_equal(gacc, oacc)
    print(f"  seed {seed}: {len(oreq)} requests, {int(gacc.sum())} accepted, {got['steps']} steps")


def test_single_axon_landing_distribution():
    wl = synth.uniform_box(40, extent=(200.0, 200.0, 200.0), sigma=90.0, seed=13)
    print("single-axon landing distribution, 600 seeds", flush=True)
    av = np.zeros(wl.n, np.float32)
    av[7] = 2.0
    wv = np.where(np.arange(wl.n) == 7, 0.0, 1.0 + (np.arange(wl.n) % 3)).astype(np.float32)
    wl.a, wl.w = av, wv
    tree, od, w, a = _setup(wl, 4)
    pos = wl.pos64()
    k = wv * np.exp(-np.sum((pos - pos[7]) ** 2, 1) / wl.sigma ** 2)
    p = k / k.sum()
    n = 600
    hits = np.zeros(wl.n)
    for seed in range(n):
        got = tree.partner_descent(w, a, wl.sigma, seed, cutoff_sigmas=0.0)
        ax = got["axon"].cpu().numpy()
        dd = got["dendrite"].cpu().numpy()
        assert ax.tolist() == [7]
        hits[dd[0]] += 1
    m = p > 0
    chi2 = float(np.sum((hits[m] - n * p[m]) ** 2 / (n * p[m])))
    assert hits[7] == 0 and chi2 < 85.0     # 38 degrees of freedom


def test_larger_run_invariants():
    wl = synth.blobs(16, 2048, extent=2000.0, std=60.0, sigma=120.0, seed=33)
    print(f"descent invariants, {wl.n} neurons", flush=True)
    tree, od, w, a = _setup(wl, 64)
    r1 = tree.partner_descent(w, a, wl.sigma, 5)
    r2 = tree.partner_descent(w, a, wl.sigma, 5)
    ax = r1["axon"].cpu().numpy()
    dd = r1["dendrite"].cpu().numpy()
    acc = r1["accepted"].cpu().numpy().astype(bool)
    for key in ("axon", "dendrite", "accepted"):
        np.testing.assert_array_equal(r1[key].cpu().numpy(), r2[key].cpu().numpy())
    assert ax.size > 0.5 * np.count_nonzero(wl.a > 0)
    assert np.unique(ax).size == ax.size
    assert np.all(wl.a[ax] > 0) and np.all(wl.w[dd] > 0) and np.all(ax != dd)
    oacc = descent.accept(list(zip(ax.tolist(), dd.tolist())), wl.w, 5)
    np.testing.assert_array_equal(acc, oacc)
    cnt = np.bincount(dd[acc], minlength=wl.n)
    assert np.all(cnt <= np.floor(wl.w))
    print(f"  {ax.size} requests, {int(acc.sum())} accepted, {r1['steps']} steps")


def test_degenerate_descents():
    import torch
    import paper_2301_10570_amd as msp
    print("descent edge cases: no axons, no dendrites, one neuron, coincident points", flush=True)
    T = lambda v: torch.from_numpy(np.ascontiguousarray(v)).cuda()
    wl = synth.uniform_box(300, extent=(200.0, 200.0, 200.0), sigma=60.0, seed=34)
    tree = msp.build_tree(T(wl.x), T(wl.y), T(wl.z), leaf_max=16)
    zero = np.zeros(wl.n, np.float32)
    for a, w in ((zero, wl.w), (wl.a, zero)):
        r = tree.partner_descent(T(w), T(a), wl.sigma, 3)
        assert r["axon"].numel() == 0
    # one neuron: no partner but itself, which is excluded
    one = msp.build_tree(T(wl.x[:1]), T(wl.y[:1]), T(wl.z[:1]), leaf_max=16)
    r = one.partner_descent(T(np.ones(1, np.float32)), T(np.ones(1, np.float32)), wl.sigma, 3)
    assert r["axon"].numel() == 0
    # coincident points: one depth-21 leaf holding all of them; every choice is by weight
    n = 200
    x = np.full(n, 5.0, np.float32)
    av = np.ones(n, np.float32)
    wv = (np.arange(n) % 3).astype(np.float32)
    ct = msp.build_tree(T(x), T(x), T(x), leaf_max=16)
    ot = octree.build(x, x, x, leaf_max=16)
    od = descent.Descent(ot, np.stack([x, x, x], 1).astype(np.float64), av, wv, 50.0)
    got = ct.partner_descent(T(wv), T(av), 50.0, 8, cutoff_sigmas=0.0)
    g = sorted(zip(got["axon"].cpu().numpy().tolist(), got["dendrite"].cpu().numpy().tolist()))
    oreq, mmin = _oracle_run(od, 8)
    if mmin >= TIE:
        assert g == oreq
    assert len(g) == n and all(wv[j] > 0 and i != j for i, j in g)
    acc = got["accepted"].cpu().numpy().astype(bool)
    dd = got["dendrite"].cpu().numpy()
    assert np.all(np.bincount(dd[acc], minlength=n) <= np.floor(wv))


def _clustered():
    """8 tight blobs of 1,024 neurons (std 12 um, sigma 60 um): the central boxes of
    the box level hold a few hundred neurons, so box pairs go through expansions."""
    return synth.blobs(8, 1024, extent=600.0, std=12.0, sigma=60.0, seed=35)


def _oracle_boxes(ot, level, wl):
    """Boxes from the oracle tree: nodes at or below `level` whose parent lies above
    it, and leaves above it, in key order; with their axon and dendrite counts."""
    lv, par = ot.level.astype(np.int64), ot.parent.astype(np.int64)
    parent_above = (par < 0) | (lv[np.maximum(par, 0)] < level)
    isbox = ((lv >= level) & parent_above) | ((ot.is_leaf == 1) & (lv < level))
    nodes = np.nonzero(isbox)[0]
    nodes = nodes[np.argsort(ot.first[nodes], kind="stable")]
    na = np.array([np.count_nonzero(wl.a[ot.perm[ot.first[v]:ot.first[v] + ot.count[v]]] > 0) for v in nodes])
    nd = np.array([np.count_nonzero(wl.w[ot.perm[ot.first[v]:ot.first[v] + ot.count[v]]] > 0) for v in nodes])
    cen = np.array([octree.node_box(ot, int(v))[0] for v in nodes])
    half = np.array([octree.node_box(ot, int(v))[1] for v in nodes])
    return nodes, na, nd, cen, half


@pytest.mark.parametrize("cutoff", [0.0, 1.5])
def test_box_pairs_match_oracle(cutoff):
    """The box table and the pair lists of a descent are exactly those the oracle's
    tree gives (every axon box against every dendrite box within the cutoff), and
    every sampled pair attraction matches the oracle's direct Att(s, c): expansions
    (both boxes at or below the box level, more than 70 axons / dendrites, centres
    within 2.5 sigma) to 1e-4, direct pairs to 2e-5 (float32 terms relative to
    the boxes' closest approach, float64 sums)."""
    wl = _clustered()
    print(f"box pairs, {wl.n} clustered neurons, cutoff {cutoff} sigma", flush=True)
    tree, od, w, a = _setup(wl, 32)
    tree.descent_step(w, a, np.array([0]), np.array([0]), 0, 5, wl.sigma, cutoff_sigmas=cutoff)
    L = tree.plan(wl.sigma, p=8, route="fgt")["level"] + 1
    nodes, na, nd, cen, half = _oracle_boxes(od.tree, L, wl)
    bn = tree.debug_buffer(7).cpu().numpy()
    np.testing.assert_array_equal(bn, nodes)
    F = tree.debug_buffer(4).cpu().numpy()
    ps = tree.debug_buffer(5).cpu().numpy()
    pc = tree.debug_buffer(6).cpu().numpy()
    # expected pairs, grouped by axon box, dendrite boxes in key order
    exp_s, exp_c = [], []
    for s in np.nonzero(na > 0)[0]:
        gap = np.maximum(np.abs(cen - cen[s]) - half[:, None] - half[s], 0.0)
        ok = nd > 0
        if cutoff > 0:
            ok &= np.sum(gap * gap, 1) <= (cutoff * wl.sigma) ** 2
        c = np.nonzero(ok)[0]
        exp_s += [s] * c.size
        exp_c += c.tolist()
    np.testing.assert_array_equal(ps, np.array(exp_s))
    np.testing.assert_array_equal(pc, np.array(exp_c))
    lv = od.tree.level[nodes]
    dist = np.linalg.norm(cen[ps] - cen[pc], axis=1) / wl.sigma
    expo = (lv[ps] >= L) & (lv[pc] >= L) & (na[ps] > 70) & (nd[pc] > 70) & (dist <= 2.5)
    ie, idr = np.nonzero(expo)[0], np.nonzero(~expo)[0]
    assert ie.size >= 20, ie.size
    pick_e = ie[synth.sample_indices(ie.size, min(ie.size, 120), seed=501)]
    pick_d = idr[synth.sample_indices(idr.size, min(idr.size, 120), seed=502)]
    worst_e = worst_d = 0.0
    for k in np.concatenate([pick_e, pick_d]):
        ref = od.att(int(nodes[ps[k]]), int(nodes[pc[k]]))
        e = abs(F[k] - ref) / ref if ref > 0 else abs(F[k])
        if expo[k]:
            worst_e = max(worst_e, e)
            assert e <= 1e-4, (k, F[k], ref)
        else:
            worst_d = max(worst_d, e)
            assert e <= 2e-5, (k, F[k], ref)
    print(f"  {ps.size} pairs, {ie.size} by expansion; max rel err: expansion {worst_e:.2e}, direct {worst_d:.2e}")


def test_clustered_steps_match_oracle():
    """Step by step on the clustered workload (no cutoff): the steps above the box
    level choose from box-pair sums, expansions included."""
    wl = _clustered()
    print(f"clustered descent steps, {wl.n} neurons", flush=True)
    tree, od, w, a = _setup(wl, 32)
    S, T = np.array([0]), np.array([0])
    seed, flips, total = 91, 0, 0
    for step in range(4):
        S2, T2, req = tree.descent_step(w, a, S, T, step, seed, wl.sigma, cutoff_sigmas=0.0)
        onxt, oreq, dec = od.step(list(zip(S.tolist(), T.tolist())), step, seed)
        assert sorted(map(tuple, req.tolist())) == sorted(oreq)
        g, o = set(_pairs(S2, T2)), set(onxt)
        diff = len(g ^ o) // 2
        near = sum(1 for _, _, m in dec if m < TIE)
        assert diff <= near, (step, diff, near)
        flips += diff
        total += len(dec)
        # continue from the oracle's frontier so that both sides see the same pairs
        S = np.array([s for s, _ in onxt], np.int64)
        T = np.array([t for _, t in onxt], np.int64)
    print(f"  {total} choices, {flips} near-tie flips")
