"""Child probabilities and proportional choice (Algorithm 2) vs the oracle's
restricted FP64 direct sums on the same (bit-exact) octree."""
import numpy as np
import pytest

import synth
from oracle import octree, partner
from tests.helpers import paper_parameters, to_dev

pytestmark = pytest.mark.gpu


def _queries(tree, n, k, seed, ancestors_only=False):
    """k (target, node) pairs: targets drawn from all points, nodes either an
    ancestor of the target's leaf at a random level or any inner node."""
    rng = np.random.default_rng(seed)
    tq = rng.integers(0, n, k)
    inner = np.nonzero(tree.is_leaf == 0)[0]
    # leaf of every sorted position
    leaf_of = np.empty(n, np.int64)
    for v in np.nonzero(tree.is_leaf)[0]:
        leaf_of[tree.first[v]:tree.first[v] + tree.count[v]] = v
    inv = np.empty(n, np.int64)
    inv[tree.perm] = np.arange(n)
    nq = np.empty(k, np.int64)
    for j in range(k):
        if ancestors_only or j % 2 == 0:
            path = []
            v = tree.parent[leaf_of[inv[tq[j]]]]
            while v >= 0:
                path.append(v)
                v = tree.parent[v]
            nq[j] = path[rng.integers(0, len(path))] if path else 0
        else:
            nq[j] = rng.choice(inner)
    return tq, nq


def _run(wl, tq, nq, uniforms=None, cutoff=0.0, exclude_self=False, p=8):
    import torch
    import paper_2301_10570_amd as msp
    d = to_dev(wl)
    tree = msp.build_tree(d["x"], d["y"], d["z"], leaf_max=wl.leaf_max)
    T = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(d["x"].device)
    P, ch = tree.partner_probabilities(d["w"], T(tq, np.int32), T(nq, np.int32), wl.sigma, p=p,
                                       uniforms=None if uniforms is None else T(uniforms, np.float32),
                                       exclude_self=exclude_self, cutoff_sigmas=cutoff)
    return P.cpu().numpy().astype(np.float64), ch.cpu().numpy()


def _check(wl, tq, nq, seed, cutoff=0.0, exclude_self=False, p=8):
    tr = octree.build(wl.x, wl.y, wl.z, leaf_max=wl.leaf_max)
    u = synth.uniforms(len(tq), seed)
    P, ch = _run(wl, tq, nq, u, cutoff, exclude_self, p)
    Pr, Sr, chr_ = partner.probabilities(tr, wl.pos64(), wl.w, wl.sigma, tq, nq, uniforms=u,
                                         exclude_self=exclude_self)
    # queries whose FP64 sums underflow entirely (node beyond ~26 sigma) have no
    # defined probabilities in the oracle; compare the rest
    live = Sr.sum(axis=1) > 0
    err = np.abs(P - Pr)[live]
    # 1e-4 relative per child, with an absolute floor of 1e-7 of the query's total
    # (the accuracy contract of the moments: M2P where its error is below 1e-7 of
    # the running total)
    bound = 1e-4 * Pr[live] + 1e-7
    print(f"  max |dP| {err.max():.2e}, max |dP| / bound {np.max(err / bound):.3f}")
    assert np.all(err <= bound), (err.max(), np.argmax(err))
    # choices agree unless r*total sits within 1e-4*total of a running-sum boundary
    run = np.cumsum(Sr, axis=1)
    tot = run[:, -1:]
    near = np.any(np.abs(run - u[:, None] * tot) <= 1e-4 * tot, axis=1)
    ok = (ch == chr_) | near | ~live
    assert np.all(ok), np.nonzero(~ok)
    return err.max()


def test_partner_uniform4k():
    wl = synth.uniform4k()
    tr = octree.build(wl.x, wl.y, wl.z, leaf_max=wl.leaf_max)
    tq, nq = _queries(tr, wl.n, 300, seed=5)
    print("partner, 4,096-point cube, 300 queries", flush=True)
    e = _check(wl, tq, nq, seed=6)
    print(f"  max |dP| {e:.2e}")


def test_partner_blobs_exclude_self():
    wl = synth.blobs262k(0.125)
    tr = octree.build(wl.x, wl.y, wl.z, leaf_max=wl.leaf_max)
    tq, nq = _queries(tr, wl.n, 200, seed=7)
    print("partner blobs (1/8), exclude self", flush=True)
    _check(wl, tq, nq, seed=8, exclude_self=True)


def test_partner_slab_ancestors():
    """Full 4M slab: moments are used for the large children."""
    wl = synth.slab4m()
    tr = octree.build(wl.x, wl.y, wl.z, leaf_max=wl.leaf_max)
    tq, nq = _queries(tr, wl.n, 48, seed=9, ancestors_only=True)
    print("partner slab 4M, 48 ancestor queries", flush=True)
    e = _check(wl, tq, nq, seed=10)
    print(f"  max |dP| {e:.2e}")


@pytest.mark.parametrize("p", [4, 10])
def test_partner_other_p(p):
    wl = synth.slab4m(0.0625)
    tr = octree.build(wl.x, wl.y, wl.z, leaf_max=wl.leaf_max)
    tq, nq = _queries(tr, wl.n, 64, seed=11 + p, ancestors_only=True)
    print(f"partner slab 1/16, p={p}", flush=True)
    _check(wl, tq, nq, seed=12, p=p)


def test_partner_edge_cases():
    import torch
    import paper_2301_10570_amd as msp
    wl = synth.uniform_box(500, seed=3)
    d = to_dev(wl)
    tree = msp.build_tree(d["x"], d["y"], d["z"], leaf_max=16)
    ex = tree.export()
    leaf = int(np.nonzero(ex["node_n_children"].cpu().numpy() == 0)[0][0])
    dev = d["x"].device
    tq = torch.tensor([0, 1, 2, 10**6], dtype=torch.int32, device=dev)
    nq = torch.tensor([leaf, 0, -3, 0], dtype=torch.int32, device=dev)
    uni = torch.full((4,), 0.5, device=dev)
    P, ch = tree.partner_probabilities(d["w"], tq, nq, wl.sigma, uniforms=uni)
    P, ch = P.cpu().numpy(), ch.cpu().numpy()
    # leaf, bad node id, bad target id: zeros and no choice
    for q in (0, 2, 3):
        assert np.all(P[q] == 0) and ch[q] == -1
    assert abs(P[1].sum() - 1) < 1e-5 and ch[1] >= 1
    # zero weights everywhere: total 0, no choice
    P, ch = tree.partner_probabilities(torch.zeros_like(d["w"]), tq, nq, wl.sigma, uniforms=uni)
    assert np.all(P.cpu().numpy() == 0) and np.all(ch.cpu().numpy() == -1)
    # no queries
    e = torch.zeros(0, dtype=torch.int32, device=dev)
    P, ch = tree.partner_probabilities(d["w"], e, e, wl.sigma)
    assert P.shape == (0, 8)


@pytest.mark.parametrize("leaf_max", [None, 512])
def test_node_moments_m2m_parity(leaf_max):
    """Node moments (P2M at the lowest moment-carrying nodes, M2M upward) equal the
    oracle's P2M over all points of the node about its centre (M2M is exact
    under the tensor truncation), and the slab's large nodes carry them; with
    leaves of up to 512 points, leaves carry moments too (from their own points)."""
    import torch
    import paper_2301_10570_amd as msp
    from oracle import fgt as ofgt
    wl = synth.slab4m(0.0625)
    if leaf_max is not None:
        wl.leaf_max = leaf_max
    tr = octree.build(wl.x, wl.y, wl.z, leaf_max=wl.leaf_max)
    d = to_dev(wl)
    tree = msp.build_tree(d["x"], d["y"], d["z"], leaf_max=wl.leaf_max)
    e = torch.zeros(0, dtype=torch.int32, device=d["x"].device)
    print(f"node moments parity (slab 1/16, p=8, leaf_max {wl.leaf_max})", flush=True)
    p = 8
    tree.partner_probabilities(d["w"], e, e, wl.sigma, p=p)
    has = tree.debug_buffer(3).cpu().numpy()
    A = tree.debug_buffer(2).cpu().numpy()
    nodes = np.nonzero(has)[0]
    assert nodes.size > 50
    lh = tree.plan(wl.sigma, p=p)["level"]
    # exactly the nodes at or below the moment level with more than c1 = 70 sources
    # (points of nonzero weight; Algorithm 2's threshold) carry moments
    S = np.concatenate([[0], np.cumsum(wl.w[tr.perm] != 0)])
    nsrc = S[tr.first + tr.count] - S[tr.first]
    c1 = paper_parameters()["c1"]
    np.testing.assert_array_equal(has != 0, (tr.level >= lh) & (nsrc > c1))
    slot0 = tr.level_offset[lh]
    A = A.reshape(-1, p, p, p)   # [slot][az][ay][ax]
    pos = wl.pos64()
    rng = np.random.default_rng(1)
    pick = rng.choice(nodes, 40, replace=False)
    if leaf_max is not None:
        leaves = nodes[tr.is_leaf[nodes] != 0]
        assert leaves.size > 0
        pick = np.concatenate([pick, rng.choice(leaves, min(10, leaves.size), replace=False)])
    for v in pick:
        c, _ = octree.node_box(tr, v)
        ids = tr.perm[tr.first[v]:tr.first[v] + tr.count[v]]
        ref = ofgt.p2m(pos[ids], wl.w[ids], c, wl.sigma, p)   # [ax, ay, az]
        got = A[v - slot0].transpose(2, 1, 0)
        assert np.abs(got - ref).max() <= 2e-5 * np.abs(ref).max(), v


def test_staged_weights_reused_after_forward():
    """MSP_WEIGHTS_STAGED: after a forward on the same tree (whose P2M gathers w into
    key order, or whose direct route stages it) the partner probabilities reuse the
    gathered weights and equal those of a call that gathers them itself; without
    such a forward, or after a backward, the flag is refused."""
    import torch
    import paper_2301_10570_amd as msp
    wl = synth.slab4m(0.0625)
    print(f"partner with staged weights, slab {wl.n} points", flush=True)
    tr = octree.build(wl.x, wl.y, wl.z, leaf_max=wl.leaf_max)
    tq, nq = _queries(tr, wl.n, 400, seed=41)
    d = to_dev(wl)
    T = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(d["x"].device)
    tqd, nqd = T(tq, np.int32), T(nq, np.int32)
    u = T(synth.uniforms(len(tq), 42), np.float32)
    tgt = T((wl.a > 0).astype(np.uint8), np.uint8)
    tree = msp.build_tree(d["x"], d["y"], d["z"], leaf_max=wl.leaf_max)
    with pytest.raises(RuntimeError):
        tree.partner_probabilities(d["w"], tqd, nqd, wl.sigma, uniforms=u, weights_staged=True)
    P0, c0 = tree.partner_probabilities(d["w"], tqd, nqd, wl.sigma, uniforms=u)
    # a forward on the expansion route keeps its gathered weights only when asked to
    tree.forward(d["w"], tgt, sigma=wl.sigma, route="fgt")
    with pytest.raises(RuntimeError):
        tree.partner_probabilities(d["w"], tqd, nqd, wl.sigma, uniforms=u, weights_staged=True)
    for route in ("fgt", "direct"):
        tree.forward(d["w"] * 0.5, tgt, sigma=wl.sigma, route="direct")   # other weights in between
        tree.forward(d["w"], tgt, sigma=wl.sigma, route=route, stage_weights=True)
        P1, c1 = tree.partner_probabilities(d["w"], tqd, nqd, wl.sigma, uniforms=u, weights_staged=True)
        np.testing.assert_array_equal(P1.cpu().numpy(), P0.cpu().numpy())
        np.testing.assert_array_equal(c1.cpu().numpy(), c0.cpu().numpy())
    # a second partner call may reuse the weights of the first
    P2, _ = tree.partner_probabilities(d["w"], tqd, nqd, wl.sigma, uniforms=u, weights_staged=True)
    np.testing.assert_array_equal(P2.cpu().numpy(), P0.cpu().numpy())
    tree.backward(d["w"], torch.ones_like(d["w"]), tgt, sigma=wl.sigma)
    with pytest.raises(RuntimeError):
        tree.partner_probabilities(d["w"], tqd, nqd, wl.sigma, uniforms=u, weights_staged=True)
    tree.close()


def test_work_counters_match_the_query_classes():
    """The work counters: queries and point pairs of the eight-lane and wavefront
    passes equal what the oracle's tree gives for the queries' nodes (nodes with
    children: up to 512 points, 513 to 16384 points); the walk takes the rest and
    reports nodes, expansions and pairs; counting does not change the results."""
    import torch
    import paper_2301_10570_amd as msp
    wl = synth.blobs262k(0.5)
    tr = octree.build(wl.x, wl.y, wl.z, leaf_max=wl.leaf_max)
    tq, nq = _queries(tr, wl.n, 2000, seed=21)
    print("partner work counters, blobs 1/2, 2,000 queries", flush=True)
    d = to_dev(wl)
    tree = msp.build_tree(d["x"], d["y"], d["z"], leaf_max=wl.leaf_max)
    T = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).cuda()
    P0, _ = tree.partner_probabilities(d["w"], T(tq, np.int32), T(nq, np.int32), wl.sigma, cutoff_sigmas=4.5)
    tree.set_work_counting(True)
    P1, _ = tree.partner_probabilities(d["w"], T(tq, np.int32), T(nq, np.int32), wl.sigma, cutoff_sigmas=4.5)
    c = tree.work_counts()
    tree.set_work_counting(False)
    assert torch.equal(P0, P1)
    cnt = tr.count[nq].astype(np.int64)
    inner = tr.n_children[nq] > 0
    small, mid, big = inner & (cnt <= 512), inner & (cnt > 512) & (cnt <= 16384), inner & (cnt > 16384)
    print(f"  counts {c}", flush=True)
    assert c["direct_queries"] == int(small.sum()) and c["direct_pairs"] == int(cnt[small].sum())
    assert c["wave_queries"] == int(mid.sum()) and c["wave_pairs"] == int(cnt[mid].sum())
    assert c["walk_queries"] == int(big.sum())
    if big.any():
        assert c["walk_nodes"] >= c["walk_queries"] and c["walk_rounds"] >= c["walk_queries"]
        assert c["walk_expansions"] + c["walk_pairs"] > 0


def test_forward_and_partner_on_two_streams():
    """After a weighted build, the forward and the partner probabilities (both with
    the staged weights) share no device memory of the handle: issued on two streams
    at once they give the same bits as one after the other on one stream, over
    several steps of build, forward and partner call."""
    import torch
    import paper_2301_10570_amd as msp
    wl = synth.slab4m(0.125)
    print(f"forward and partner on two streams, slab {wl.n} points", flush=True)
    tr = octree.build(wl.x, wl.y, wl.z, leaf_max=wl.leaf_max)
    tq, nq = _queries(tr, wl.n, 3000, seed=61)
    d = to_dev(wl)
    T = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(d["x"].device)
    tqd, nqd = T(tq, np.int32), T(nq, np.int32)
    uni = T(synth.uniforms(len(tq), 62), np.float32)
    tgt = T((wl.a > 0).astype(np.uint8), np.uint8)
    u = torch.empty(wl.n, dtype=torch.float32, device=d["x"].device)
    tree = msp.Tree()

    def step(side):
        tree.build(d["x"], d["y"], d["z"], leaf_max=wl.leaf_max, w=d["w"])
        main = torch.cuda.current_stream()
        if side is None:
            tree.forward(d["w"], tgt, sigma=wl.sigma, route="fgt", out=u, weights_staged=True)
            P, c = tree.partner_probabilities(d["w"], tqd, nqd, wl.sigma, uniforms=uni, weights_staged=True)
        else:
            side.wait_stream(main)
            with torch.cuda.stream(side):
                P, c = tree.partner_probabilities(d["w"], tqd, nqd, wl.sigma, uniforms=uni,
                                                  weights_staged=True)
            tree.forward(d["w"], tgt, sigma=wl.sigma, route="fgt", out=u, weights_staged=True)
            main.wait_stream(side)
        return u.clone(), P.clone(), c.clone()

    u0, P0, c0 = step(None)
    torch.cuda.synchronize()
    # the weighted build counted the sources per position for the node moments; a
    # tree built without weights, whose partner call stages them and counts itself,
    # gives the same bits
    plain = msp.build_tree(d["x"], d["y"], d["z"], leaf_max=wl.leaf_max)
    Pp, cp = plain.partner_probabilities(d["w"], tqd, nqd, wl.sigma, uniforms=uni)
    assert torch.equal(Pp, P0) and torch.equal(cp, c0)
    plain.close()
    side = torch.cuda.Stream()
    for it in range(3):
        u1, P1, c1 = step(side)
        torch.cuda.synchronize()
        assert torch.equal(u1, u0), it
        assert torch.equal(P1, P0), it
        assert torch.equal(c1, c0), it
    # isolated timing: the same bits with every pass on the caller's stream
    tree.set_timing(True, isolated=True)
    tree.timing(reset=True)
    u2, P2, c2 = step(None)
    ph = tree.timing(reset=True)
    tree.set_timing(False)
    assert torch.equal(u2, u0) and torch.equal(P2, P0) and torch.equal(c2, c0)
    for name in ("node_moments", "partner", "partner_direct", "partner_wave", "p2m", "l2p"):
        assert name in ph and ph[name][1] >= 1, name
    assert msp._lib.msp_tree_set_timing(tree._h, 3) == msp.MSP_EINVAL
    tree.close()


def test_source_counts_follow_the_staged_weights():
    """The node moments reuse the per-position source counts of a weighted build only
    while the staged weights are those of the build: after a forward that stages
    other weights, or a partner call that stages its own, the counts are taken
    again, and every result equals that of a fresh tree given the same weights."""
    import torch
    import paper_2301_10570_amd as msp
    wl = synth.slab4m(0.0625)
    print(f"source counts and staged weights, slab {wl.n} points", flush=True)
    tr = octree.build(wl.x, wl.y, wl.z, leaf_max=wl.leaf_max)
    tq, nq = _queries(tr, wl.n, 600, seed=71)
    d = to_dev(wl)
    T = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(d["x"].device)
    tqd, nqd = T(tq, np.int32), T(nq, np.int32)
    uni = T(synth.uniforms(len(tq), 72), np.float32)
    tgt = T((wl.a > 0).astype(np.uint8), np.uint8)
    # other weights: about half the sources switched off, so that the nodes' source
    # counts (and with them which nodes carry moments) change
    keep = np.random.default_rng(73).random(wl.n) < 0.5
    w2 = T(np.where(keep, wl.w, 0).astype(np.float32), np.float32)

    def fresh(w):
        t = msp.build_tree(d["x"], d["y"], d["z"], leaf_max=wl.leaf_max)
        P, c = t.partner_probabilities(w, tqd, nqd, wl.sigma, uniforms=uni)
        t.close()
        return P, c

    P1r, c1r = fresh(d["w"])
    P2r, c2r = fresh(w2)
    assert not torch.equal(P1r, P2r)
    tree = msp.Tree()
    tree.build(d["x"], d["y"], d["z"], leaf_max=wl.leaf_max, w=d["w"])
    P, c = tree.partner_probabilities(d["w"], tqd, nqd, wl.sigma, uniforms=uni, weights_staged=True)
    assert torch.equal(P, P1r) and torch.equal(c, c1r)
    # a forward that stages w2 into the records
    u = torch.empty(wl.n, dtype=torch.float32, device=d["x"].device)
    tree.forward(w2, tgt, sigma=wl.sigma, route="fgt", out=u, stage_weights=True)
    P, c = tree.partner_probabilities(w2, tqd, nqd, wl.sigma, uniforms=uni, weights_staged=True)
    assert torch.equal(P, P2r) and torch.equal(c, c2r)
    # a partner call that stages its own weights, then one that reuses them
    P, c = tree.partner_probabilities(d["w"], tqd, nqd, wl.sigma, uniforms=uni)
    assert torch.equal(P, P1r) and torch.equal(c, c1r)
    P, c = tree.partner_probabilities(d["w"], tqd, nqd, wl.sigma, uniforms=uni, weights_staged=True)
    assert torch.equal(P, P1r) and torch.equal(c, c1r)
    # a weighted build with w2, then its counts
    tree.build(d["x"], d["y"], d["z"], leaf_max=wl.leaf_max, w=w2)
    P, c = tree.partner_probabilities(w2, tqd, nqd, wl.sigma, uniforms=uni, weights_staged=True)
    assert torch.equal(P, P2r) and torch.equal(c, c2r)
    tree.close()
