"""Batches of independent populations (the many-population workload at half size): the batched
forward matches the single-tree calls on every population (bit for bit on the
direct route, to float32 rounding on the expansion route), the batched backward
matches them (bit for bit on the direct route, to float32 rounding on the expansion
route), both agree with the FP64 oracle, and replays of the captured graph
equal the eager result."""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _concat(pops, empty_at=None):
    import torch
    xs, ys, zs, ws, ts, offs = [], [], [], [], [], [0]
    sig = []
    for k, wl in enumerate(pops):
        if empty_at is not None and k == empty_at:
            offs.append(offs[-1])
            sig.append(100.0)
        xs.append(wl.x); ys.append(wl.y); zs.append(wl.z); ws.append(wl.w)
        ts.append((wl.a > 0).astype(np.uint8))
        offs.append(offs[-1] + wl.n)
        sig.append(wl.sigma)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(np.concatenate(a))).cuda()
    return (T(xs), T(ys), T(zs), T(ws), T(ts), np.array(offs, dtype=np.int64),
            np.array(sig, dtype=np.float32))


def _single(wl, p=8, leaf_max=64, route="auto"):
    import torch
    import paper_2301_10570_amd as msp
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    tree = msp.build_tree(T(wl.x), T(wl.y), T(wl.z), leaf_max=leaf_max)
    tgt = T((wl.a > 0).astype(np.uint8))
    u = tree.forward(T(wl.w), tgt, sigma=float(np.float32(wl.sigma)), p=p, route=route)
    return tree, u.cpu().numpy()


@pytest.fixture(scope="module")
def pops():
    return synth.populations(count=20, scale=0.5)


def test_batch_forward_equals_single_trees_and_oracle(pops):
    import paper_2301_10570_amd as msp
    print("batch forward vs single trees, 20 populations + 1 empty", flush=True)
    x, y, z, w, tg, off, sig = _concat(pops, empty_at=7)
    b = msp.Batch().build(x, y, z, off)
    u = b.forward(w, sig, is_target=tg, use_graph=False).cpu().numpy()
    routes = []
    k = 0
    for i in range(len(off) - 1):
        lo, hi = off[i], off[i + 1]
        if hi == lo:
            continue
        wl = pops[k]
        k += 1
        tree, us = _single(wl)
        route = tree.plan(float(np.float32(wl.sigma)), p=8)["route"]
        routes.append(route)
        if route == "direct":
            np.testing.assert_array_equal(u[lo:hi], us)   # same P2P kernel body
        else:
            # the batched moments are summed in another order (one wavefront per cell)
            np.testing.assert_allclose(u[lo:hi], us, rtol=2e-5, atol=1e-6 * np.abs(us).max())
        tgt = np.nonzero(wl.a > 0)[0]
        sel = tgt[synth.sample_indices(tgt.size, 24, seed=900 + i)]
        ref = oracle.attraction(wl, sel)
        assert rel_err(u[lo:hi][sel], ref).max() <= TOL
    print(f"  routes: {routes}")
    assert "fgt" in routes and "direct" in routes   # both paths of the batch are exercised
    ms = b.instance_ms()
    assert ms[7] == 0.0 and (np.delete(ms, 7) > 0).all()
    b.close()


def test_batch_graph_replays_match_eager(pops):
    import torch
    import paper_2301_10570_amd as msp
    print("batch graph replay x3 with eager work between", flush=True)
    x, y, z, w, tg, off, sig = _concat(pops[:12])
    b = msp.Batch().build(x, y, z, off)
    out = torch.empty(x.numel(), dtype=torch.float32, device="cuda")
    ref = b.forward(w, sig, is_target=tg, out=out).cpu().numpy().copy()   # eager + capture
    assert b.info()["launches_last_eager_forward"] > 0
    for rep in range(3):
        a = torch.randn(512, 512, device="cuda")
        (a @ a).sum().item()           # unrelated eager work and a synchronisation
        out.zero_()
        torch.cuda.synchronize()
        got = b.forward(w, sig, is_target=tg, out=out).cpu().numpy()   # graph replay
        np.testing.assert_array_equal(got, ref)
    b.close()


def test_batch_backward_equals_single_trees(pops):
    import torch
    import paper_2301_10570_amd as msp
    print("batch backward vs single trees", flush=True)
    sub = pops[:8]
    x, y, z, w, tg, off, sig = _concat(sub)
    b = msp.Batch().build(x, y, z, off)
    g = torch.from_numpy(synth.uniforms(x.numel(), 901) + np.float32(0.5)).cuda()
    got = b.backward(w, g, sig, is_target=tg)
    u_all = b.forward(w, sig, is_target=tg, use_graph=False).cpu().numpy()
    routes = []
    for k, wl in enumerate(sub):
        lo, hi = off[k], off[k + 1]
        tree, _ = _single(wl)
        T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        ref = tree.backward(T(wl.w), g[lo:hi].contiguous(), T((wl.a > 0).astype(np.uint8)),
                            sigma=float(np.float32(wl.sigma)), p=8)
        route = tree.plan(float(np.float32(wl.sigma)), p=8)["route"]
        routes.append(route)
        pairs = [(got["w"][lo:hi], ref["w"])] + [(got["pos"][a][lo:hi], ref["pos"][a]) for a in range(3)]
        if route == "direct":
            # the same P2P-with-derivatives and combination bodies: identical bits
            for gv, rv in pairs:
                np.testing.assert_array_equal(gv.cpu().numpy(), rv.cpu().numpy())
            assert got["sigma"][k].item() == ref["sigma"].item()
        else:
            # the batched moments and translations are summed in another order
            for gv, rv in pairs:
                r = rv.cpu().numpy()
                np.testing.assert_allclose(gv.cpu().numpy(), r, rtol=1e-4, atol=1e-5 * np.abs(r).max())
            assert abs(got["sigma"][k].item() - ref["sigma"].item()) <= 1e-4 * abs(ref["sigma"].item())
        # against the oracle: weight and position derivatives at 64 seeded points of
        # the population, and its sigma derivative over all pairs
        smp = synth.sample_indices(wl.n, 64, seed=910 + k)
        gk = g[lo:hi].cpu().numpy().astype(np.float64)
        pos = wl.pos64()
        tgt = np.nonzero(wl.a > 0)[0]
        d_src = oracle.gauss_grad(pos[tgt], gk[tgt], pos[smp], wl.w[smp], wl.sigma, want=("w", "s"))
        st = smp[wl.a[smp] > 0]
        d_tgt = oracle.gauss_grad(pos[st], gk[st], pos, wl.w, wl.sigma, want=("t",))
        sig_ref = oracle.gauss_grad(pos[tgt], gk[tgt], pos, wl.w, wl.sigma, want=("sigma",))["sigma"]
        gpos_ref = d_src["s"].copy()
        gpos_ref[np.searchsorted(smp, st)] += d_tgt["t"]
        gw_b = got["w"][lo:hi].cpu().numpy()[smp]
        assert np.max(np.abs(gw_b - d_src["w"]) / d_src["w"]) <= TOL, k
        gp_b = np.stack([got["pos"][a][lo:hi].cpu().numpy()[smp] for a in range(3)], 1)
        u_b = u_all[lo:hi][smp]
        scale = 2.0 / wl.sigma * (gk[smp] * (wl.a[smp] > 0) * u_b + wl.w[smp] * d_src["w"])
        perr = np.max(np.abs(gp_b - gpos_ref), axis=1)
        assert np.all(perr <= 5e-4 * scale + 1e-12), k
        assert abs(got["sigma"][k].item() - sig_ref) <= TOL * abs(sig_ref), k
    print(f"  routes: {routes}")
    assert "fgt" in routes and "direct" in routes   # both paths of the batched backward are exercised
    # the second call with the same arguments replays the captured graph
    keep = {"w": got["w"].cpu().numpy().copy(), "sigma": got["sigma"].cpu().numpy().copy(),
            "pos": [a.cpu().numpy().copy() for a in got["pos"]]}
    again = b.backward(w, g, sig, is_target=tg, use_graph=True)      # eager, then captured
    for rep in range(3):
        g.sum().item()                                                  # eager work and a synchronisation
        for k_ in ("w", "sigma_full"):
            again[k_].zero_()
        for a in again["pos"]:
            a.zero_()
        again = b.backward(w, g, sig, is_target=tg, out=again, use_graph=True)   # graph replay
        np.testing.assert_array_equal(again["w"].cpu().numpy(), keep["w"])
        np.testing.assert_array_equal(again["sigma"].cpu().numpy(), keep["sigma"])
        for a in range(3):
            np.testing.assert_array_equal(again["pos"][a].cpu().numpy(), keep["pos"][a])
    b.close()


def test_batch_autotune(pops):
    import paper_2301_10570_amd as msp
    print("batch autotune over leaf sizes 16/32/64 and both routes", flush=True)
    sub = pops[:8]
    x, y, z, w, tg, off, sig = _concat(sub)
    b = msp.Batch()
    leaf, routes = b.autotune(x, y, z, off, w, sig, is_target=tg, candidates=(16, 32, 64))
    print(f"  leaf {leaf.tolist()} routes {routes}")
    assert set(leaf.tolist()) <= {16, 32, 64} and set(routes) <= {"fgt", "direct"}
    u = b.forward(w, sig, is_target=tg).cpu().numpy()
    for k, wl in enumerate(sub):
        lo = off[k]
        tgt = np.nonzero(wl.a > 0)[0]
        sel = tgt[synth.sample_indices(tgt.size, 16, seed=950 + k)]
        assert rel_err(u[lo:lo + wl.n][sel], oracle.attraction(wl, sel)).max() <= TOL
    b.close()


def _single_backward(wl, g, want):
    import torch
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    tree, _ = _single(wl)
    ref = tree.backward(T(wl.w), g.contiguous(), T((wl.a > 0).astype(np.uint8)),
                        sigma=float(np.float32(wl.sigma)), p=8, want=want)
    route = tree.plan(float(np.float32(wl.sigma)), p=8)["route"]
    tree.close()
    return ref, route


def test_batch_backward_subsets_and_empty_population(pops):
    import torch
    import paper_2301_10570_amd as msp
    print("batch backward: one empty population, gradient subsets", flush=True)
    sub = pops[8:14]
    x, y, z, w, tg, off, sig = _concat(sub, empty_at=2)
    b = msp.Batch().build(x, y, z, off)
    g = torch.from_numpy(synth.uniforms(x.numel(), 902) + np.float32(0.5)).cuda()
    for want in (("w",), ("sigma",), ("pos", "sigma")):
        got = b.backward(w, g, sig, is_target=tg, want=want)
        if "sigma" in want:
            assert got["sigma"][2].item() == 0.0          # the empty population
        k = 0
        for i in range(len(off) - 1):
            lo, hi = off[i], off[i + 1]
            if hi == lo:
                continue
            ref, route = _single_backward(sub[k], g[lo:hi], want)
            k += 1
            for key in want:
                if key == "sigma":
                    gs, rs = got["sigma"][i].item(), ref["sigma"].item()
                    if route == "direct":
                        assert gs == rs
                    else:
                        assert abs(gs - rs) <= 1e-4 * abs(rs) + 1e-30
                    continue
                gv = [got[key]] if key == "w" else got[key]
                rv = [ref[key]] if key == "w" else ref[key]
                for a_, b_ in zip(gv, rv):
                    a_, b_ = a_[lo:hi].cpu().numpy(), b_.cpu().numpy()
                    if route == "direct":
                        np.testing.assert_array_equal(a_, b_)
                    else:
                        np.testing.assert_allclose(a_, b_, rtol=1e-4, atol=1e-5 * np.abs(b_).max())
    b.close()


def test_batch_forward_and_backward_graphs_alternate(pops):
    import torch
    import paper_2301_10570_amd as msp
    print("batch forward and backward graphs, alternating, against eager results", flush=True)
    sub = pops[:5]
    x, y, z, w, tg, off, sig = _concat(sub)
    b = msp.Batch().build(x, y, z, off)
    g = torch.from_numpy(synth.uniforms(x.numel(), 903) + np.float32(0.5)).cuda()
    u_ref = b.forward(w, sig, is_target=tg, use_graph=False).cpu().numpy()
    gr = b.backward(w, g, sig, is_target=tg)
    g_ref = {"w": gr["w"].cpu().numpy(), "sigma": gr["sigma"].cpu().numpy(),
             "pos": [a.cpu().numpy() for a in gr["pos"]]}
    u = torch.empty(x.numel(), dtype=torch.float32, device="cuda")
    out = None
    for rep in range(3):
        u.zero_()
        b.forward(w, sig, is_target=tg, out=u, use_graph=True)     # eager + capture, then replays
        np.testing.assert_array_equal(u.cpu().numpy(), u_ref)
        if out is not None:
            for k_ in ("w", "sigma_full"):
                out[k_].zero_()
            for a in out["pos"]:
                a.zero_()
        out = b.backward(w, g, sig, is_target=tg, out=out, use_graph=True)
        np.testing.assert_array_equal(out["w"].cpu().numpy(), g_ref["w"])
        np.testing.assert_array_equal(out["sigma"].cpu().numpy(), g_ref["sigma"])
        for a in range(3):
            np.testing.assert_array_equal(out["pos"][a].cpu().numpy(), g_ref["pos"][a])
        torch.cuda.synchronize()
    b.close()


def test_batch_split_bf16_translation(pops):
    """Split-bfloat16 translation in the batched route (p = 8): forward and
    backward within the split's rounding of the fp32 batch, the forward within
    1e-4 of the oracle; p != 8 is refused."""
    import torch
    import paper_2301_10570_amd as msp
    print("batch forward/backward with split bf16 M2L", flush=True)
    sub = pops[:8]
    x, y, z, w, tg, off, sig = _concat(sub)
    b = msp.Batch().build(x, y, z, off)
    u32 = b.forward(w, sig, is_target=tg, use_graph=False).cpu().numpy()
    u16 = b.forward(w, sig, is_target=tg, use_graph=False, m2l="bf16x3").cpu().numpy()
    tgt = tg.cpu().numpy() > 0
    d = np.abs(u16[tgt].astype(np.float64) - u32[tgt]) / np.abs(u32[tgt])
    print(f"  forward: max rel diff from fp32 {d.max():.2e}")
    assert d.max() <= 5e-5
    errs = []
    for k in range(len(sub)):
        wl = sub[k]
        t_k = np.nonzero(wl.a > 0)[0]
        sel = t_k[synth.sample_indices(t_k.size, 16, seed=930 + k)]
        ref = oracle.attraction(wl, sel)
        errs.append(rel_err(u16[off[k]:off[k + 1]][sel], ref))
    e = np.concatenate(errs)
    print(f"  forward vs oracle: max rel err {e.max():.2e}")
    assert e.max() <= TOL
    g = torch.from_numpy(synth.uniforms(x.numel(), 931) + np.float32(0.5)).cuda()
    r32 = b.backward(w, g, sig, is_target=tg)
    r16 = b.backward(w, g, sig, is_target=tg, m2l="bf16x3")
    gw32, gw16 = r32["w"].cpu().numpy(), r16["w"].cpu().numpy()
    assert np.max(np.abs(gw16 - gw32) / np.abs(gw32)) <= 5e-5
    s32, s16 = r32["sigma"].cpu().numpy(), r16["sigma"].cpu().numpy()
    assert np.max(np.abs(s16 - s32) / np.abs(s32)) <= 5e-5
    with pytest.raises(msp.MspError) as ei:
        b.forward(w, sig, is_target=tg, p=6, m2l="bf16x3")
    assert ei.value.code == msp.MSP_ENOTSUP
    b.close()


def test_batch_pair_count(pops):
    """The direct-route pair count: with no cutoff every leaf lists every leaf, so a
    population of n points contributes n^2 pairs; with the cutoff it lies between n
    (each leaf lists itself) and n^2, and below the count without a cutoff."""
    import paper_2301_10570_amd as msp
    print("batch pair count: no cutoff (closed form), cutoff (bounds), state checks", flush=True)
    sub = pops[:6]
    x, y, z, w, tg, off, sig = _concat(sub, empty_at=2)
    b = msp.Batch().build(x, y, z, off)
    with pytest.raises(msp.MspError) as e:
        b.pair_count()
    assert e.value.code == -6
    sizes = np.diff(off)
    b.forward(w, sig, is_target=tg, route="direct", cutoff_sigmas=0.0, use_graph=False)
    pairs_all, span = b.pair_count()
    assert pairs_all == int((sizes.astype(np.int64) ** 2).sum())
    assert span > 0.0
    b.forward(w, sig, is_target=tg, route="direct", use_graph=True)
    pairs_cut, _ = b.pair_count()
    assert int(sizes.sum()) <= pairs_cut < pairs_all
    b.forward(w, sig, is_target=tg, route="direct", use_graph=True)   # graph replay: same lists
    assert b.pair_count()[0] == pairs_cut
    b.forward(w, sig, is_target=tg, route="fgt", use_graph=False)     # no direct-route population
    assert b.pair_count() == (0, 0.0)
    b.build(x, y, z, off)
    with pytest.raises(msp.MspError):
        b.pair_count()
    b.close()
