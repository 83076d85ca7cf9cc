"""GPU forward sums vs the FP64 oracle: max per-target relative error <= 1e-4
(the accuracy bar of the study), pass-level parity of the expansion grids, and
edge cases."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import fgt as ofgt
from oracle import octree
from tests.helpers import rel_err, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _forward(wl, **kw):
    import paper_2301_10570_amd as msp
    d = to_dev(wl)
    tree = msp.build_tree(d["x"], d["y"], d["z"], leaf_max=wl.leaf_max)
    kw.setdefault("sigma", wl.sigma)
    kw.setdefault("p", wl.p)
    u = tree.forward(d["w"], d["tgt"], **kw).cpu().numpy()
    return tree, u


@pytest.mark.parametrize("route,cutoff", [("fgt", 4.5), ("direct", 4.5), ("direct", 0.0), ("auto", 4.5)])
def test_uniform4k_all_targets(route, cutoff):
    wl = synth.uniform4k()
    print(f"4,096-point cube route={route} cutoff={cutoff}", flush=True)
    tree, u = _forward(wl, route=route, cutoff_sigmas=cutoff)
    tgt = np.nonzero(wl.a > 0)[0]
    ref = oracle.attraction(wl, tgt)
    err = rel_err(u[tgt], ref)
    print(f"  plan={tree.plan(wl.sigma, route=route, cutoff_sigmas=cutoff)} max rel err {err.max():.3e}")
    assert err.max() <= TOL
    non = np.nonzero(wl.a == 0)[0]
    assert np.all(u[non] == 0)


@pytest.mark.parametrize("route", ["fgt", "direct"])
def test_blobs262k(route):
    wl = synth.blobs262k()
    print(f"262,144-point blobs route={route}", flush=True)
    tree, u = _forward(wl, route=route)
    tgt = np.nonzero(wl.a > 0)[0]
    sel = tgt[synth.sample_indices(tgt.size, 4096, seed=202)]
    ref = oracle.attraction(wl, sel)
    err = rel_err(u[sel], ref)
    print(f"  plan={tree.plan(wl.sigma, route=route)} max rel err {err.max():.3e} p99 {np.quantile(err, 0.99):.3e}")
    assert err.max() <= TOL


@pytest.mark.parametrize("p,n,extent", [(6, 1500, (400.0, 300.0, 200.0)), (8, 6000, (400.0, 300.0, 100.0))])
def test_pass_level_parity_grids(p, n, extent):
    """P2M moments and M2L output per cell vs the oracle's FP64 single-level
    transform on the same cells (level forced).  p = 8 runs the matrix-core P2M
    (several 256-point chunks per cell and a ragged last chunk); p = 6 the vector
    P2M."""
    import paper_2301_10570_amd as msp
    wl = synth.uniform_box(n, extent=extent, sigma=120.0, seed=31)
    level = 2
    print(f"pass-level parity p={p} level={level} n={n}", flush=True)
    tree, u = _forward(wl, p=p, level=level, route="fgt")
    plan = tree.plan(wl.sigma, p=p, level=level, route="fgt")
    G = plan["grid"]
    A = tree.debug_buffer(0).cpu().numpy().reshape(G[2], p, G[1], p, G[0], p)
    C = tree.debug_buffer(1).cpu().numpy().reshape(G[2], p, G[1], p, G[0], p)
    pos = wl.pos64()
    u_ref, cells, A_ref, C_ref = ofgt.grid_transform(pos, wl.w.astype(np.float64), np.ones(wl.n), wl.sigma, p, level)
    for c, (ix, iy, iz) in enumerate(cells):
        a_gpu = A[iz, :, iy, :, ix, :].transpose(2, 1, 0)   # -> [ax, ay, az]
        c_gpu = C[iz, :, iy, :, ix, :].transpose(2, 1, 0)
        scale_a = np.abs(A_ref[c]).max()
        assert np.abs(a_gpu - A_ref[c]).max() <= 1e-5 * scale_a
        scale_c = np.abs(C_ref[c]).max()
        assert np.abs(c_gpu - C_ref[c]).max() <= 1e-4 * scale_c
    # empty cells of the grid carry zero moments
    occ = np.zeros((G[2], G[1], G[0]), bool)
    occ[cells[:, 2], cells[:, 1], cells[:, 0]] = True
    assert np.all(A.transpose(0, 2, 4, 1, 3, 5)[~occ] == 0)
    tgt = np.nonzero(wl.a > 0)[0]
    np.testing.assert_allclose(u[tgt], u_ref[tgt], rtol=2e-5)


def test_direct_baseline():
    import torch
    import paper_2301_10570_amd as msp
    wl = synth.uniform4k()
    print("all-pairs direct baseline", flush=True)
    tgt = np.nonzero(wl.a > 0)[0]
    src = np.nonzero(wl.w > 0)[0]
    dev = torch.device("cuda", 0)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    u = msp.direct_sum(T(wl.x[tgt]), T(wl.y[tgt]), T(wl.z[tgt]), T(wl.x[src]), T(wl.y[src]), T(wl.z[src]),
                       T(wl.w[src]), wl.sigma).cpu().numpy()
    ref = oracle.attraction(wl, tgt)
    assert rel_err(u, ref).max() <= 1e-5
    # ragged tile tails
    for nt, ns in ((1, 1), (257, 1023), (300, 1025), (5, 2049)):
        rng = np.random.default_rng(nt + ns)
        t = rng.random((nt, 3)).astype(np.float32) * 300
        s = rng.random((ns, 3)).astype(np.float32) * 300
        w = rng.random(ns).astype(np.float32) + 0.1
        got = msp.direct_sum(T(t[:, 0]), T(t[:, 1]), T(t[:, 2]), T(s[:, 0]), T(s[:, 1]), T(s[:, 2]), T(w),
                             80.0).cpu().numpy()
        assert rel_err(got, oracle.gauss_sum(t, s, w, 80.0)).max() <= 1e-5


def test_exclude_self():
    wl = synth.uniform_box(3000, extent=(800.0, 800.0, 800.0), sigma=90.0, seed=41)
    print("exclude self, direct and expansion routes", flush=True)
    tgt = np.nonzero(wl.a > 0)[0]
    ref = oracle.attraction(wl, tgt, exclude_self=True)
    _, u = _forward(wl, route="direct", exclude_self=True, cutoff_sigmas=0.0)
    assert rel_err(u[tgt], ref).max() <= TOL
    _, u = _forward(wl, route="fgt", exclude_self=True)
    # subtraction after the fact: absolute error bounded by the transform's error on u
    full = oracle.attraction(wl, tgt)
    assert np.max(np.abs(u[tgt] - ref) / full) <= TOL


def test_deterministic_and_linear():
    import torch
    import paper_2301_10570_amd as msp
    wl = synth.slab4m(0.125)
    print("determinism + linearity (slab, 1/8 size)", flush=True)
    d = to_dev(wl)
    tree = msp.build_tree(d["x"], d["y"], d["z"])
    for route in ("fgt", "direct"):
        u1 = tree.forward(d["w"], d["tgt"], sigma=wl.sigma, route=route).cpu().numpy()
        u2 = tree.forward(d["w"], d["tgt"], sigma=wl.sigma, route=route).cpu().numpy()
        assert np.array_equal(u1, u2)
    u_a = tree.forward(d["w"], d["tgt"], sigma=wl.sigma, route="fgt").double()
    u_b = tree.forward(2.0 * d["w"], d["tgt"], sigma=wl.sigma, route="fgt").double()
    assert torch.allclose(u_b, 2 * u_a, rtol=1e-6, atol=0)
    # outputs, weights and flags at unaligned offsets (the expansion route's flag and
    # self-term pass then takes one point per thread instead of four): the same bits
    for exclude in (False, True):
        ref = tree.forward(d["w"], d["tgt"], sigma=wl.sigma, route="fgt", exclude_self=exclude)
        ub = torch.empty(wl.n + 1, dtype=torch.float32, device=d["x"].device)
        wb = torch.empty(wl.n + 1, dtype=torch.float32, device=d["x"].device)
        tb = torch.empty(wl.n + 1, dtype=torch.uint8, device=d["x"].device)
        wb[1:] = d["w"]
        tb[1:] = d["tgt"]
        tree.forward(wb[1:], tb[1:], sigma=wl.sigma, route="fgt", exclude_self=exclude, out=ub[1:])
        assert torch.equal(ub[1:], ref), exclude


def test_edge_cases():
    import torch
    import paper_2301_10570_amd as msp
    dev = torch.device("cuda", 0)
    one = torch.tensor([5.0], device=dev)
    print("edge: single point", flush=True)
    tree = msp.build_tree(one, one, one)
    for route in ("fgt", "direct"):
        u = tree.forward(torch.tensor([3.0], device=dev), None, sigma=10.0, route=route).cpu().numpy()
        assert abs(u[0] - 3.0) <= 3.0 * TOL
    print("edge: zero weights, no targets", flush=True)
    wl = synth.uniform_box(2000, seed=8)
    d = to_dev(wl)
    tree = msp.build_tree(d["x"], d["y"], d["z"])
    for route in ("fgt", "direct"):
        u = tree.forward(torch.zeros_like(d["w"]), None, sigma=100.0, route=route)
        assert torch.count_nonzero(u).item() == 0
        u = tree.forward(d["w"], torch.zeros_like(d["tgt"]), sigma=100.0, route=route)
        assert torch.count_nonzero(u).item() == 0
    print("edge: empty input", flush=True)
    e = torch.zeros(0, device=dev)
    tree = msp.build_tree(e, e, e)
    assert tree.forward(e, None, sigma=1.0).numel() == 0
    print("edge: bad params", flush=True)
    tree = msp.build_tree(d["x"], d["y"], d["z"])
    for bad in (dict(p=0), dict(p=17), dict(sigma=0.0), dict(sigma=float("inf")), dict(level=22)):
        kw = dict(sigma=100.0)
        kw.update(bad)
        with pytest.raises(msp.MspError):
            tree.forward(d["w"], d["tgt"], **kw)


@pytest.mark.parametrize("p,level", [(8, 4), (5, 5), (3, 3)])
def test_m2l_matrix_cores_match_vector_path(p, level):
    """The MFMA translation passes give the vector-ALU passes' Taylor grid up to
    float32 rounding (checks the matrix-core lane layout), on ragged grids."""
    import paper_2301_10570_amd as msp
    wl = synth.slab4m(0.03)
    print(f"M2L mfma vs valu p={p} level={level}", flush=True)
    d = to_dev(wl)
    tree = msp.build_tree(d["x"], d["y"], d["z"])
    u_m = tree.forward(d["w"], d["tgt"], sigma=wl.sigma, p=p, level=level, route="fgt").cpu().numpy()
    C_m = tree.debug_buffer(1).cpu().numpy()
    u_v = tree.forward(d["w"], d["tgt"], sigma=wl.sigma, p=p, level=level, route="fgt", m2l="valu").cpu().numpy()
    C_v = tree.debug_buffer(1).cpu().numpy()
    scale = np.abs(C_v).max()
    assert np.abs(C_m - C_v).max() <= 1e-5 * scale
    tgt = wl.a > 0
    np.testing.assert_allclose(u_m[tgt], u_v[tgt], rtol=1e-5)


@pytest.mark.parametrize("p,level", [(8, 4), (5, 5), (10, 3)])
def test_m2l_bf16x3_matches_fp32(p, level):
    """Split-bfloat16 translation passes: Taylor grid within the split's rounding
    (about 2^-16 per product) of the float32 vector-ALU grid, on ragged grids."""
    import paper_2301_10570_amd as msp
    wl = synth.slab4m(0.03)
    print(f"M2L bf16x3 vs valu p={p} level={level}", flush=True)
    d = to_dev(wl)
    tree = msp.build_tree(d["x"], d["y"], d["z"])
    u_b = tree.forward(d["w"], d["tgt"], sigma=wl.sigma, p=p, level=level, route="fgt", m2l="bf16x3").cpu().numpy()
    C_b = tree.debug_buffer(1).cpu().numpy()
    u_v = tree.forward(d["w"], d["tgt"], sigma=wl.sigma, p=p, level=level, route="fgt", m2l="valu").cpu().numpy()
    C_v = tree.debug_buffer(1).cpu().numpy()
    scale = np.abs(C_v).max()
    dC = np.abs(C_b - C_v).max() / scale
    tgt = wl.a > 0
    du = np.abs(u_b[tgt] - u_v[tgt]) / np.abs(u_v[tgt])
    print(f"  grid max |dC|/max|C| {dC:.2e}, u max rel diff {du.max():.2e}")
    assert dC <= 2e-4
    assert du.max() <= 5e-5


def test_weighted_build_and_staged_forward():
    """Weights carried into key order by the build (msp_octree_build_weighted): a
    forward with MSP_WEIGHTS_STAGED gives the bits of a plain forward on every P2M
    path (matrix-core p = 8, vector p = 6, two-level), on the direct route, and
    with the self term; without staged weights the flag is refused."""
    import torch
    import paper_2301_10570_amd as msp
    wl = synth.slab4m(0.125)
    print("weighted build + staged forward (slab 1/8)", flush=True)
    d = to_dev(wl)
    plain = msp.build_tree(d["x"], d["y"], d["z"])
    staged = msp.Tree().build(d["x"], d["y"], d["z"], w=d["w"])
    for kw in (dict(p=8, route="fgt"), dict(p=6, route="fgt"), dict(p=8, route="fgt", two_level=True),
               dict(p=8, route="direct"), dict(p=8, route="fgt", exclude_self=True)):
        ref = plain.forward(d["w"], d["tgt"], sigma=wl.sigma, **kw).cpu().numpy()
        got = staged.forward(d["w"], d["tgt"], sigma=wl.sigma, weights_staged=True, **kw).cpu().numpy()
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), kw
    # partner probabilities from the staged weights match the plain call
    tq = torch.arange(0, 64, dtype=torch.int32, device=d["x"].device) * 997
    nq = torch.zeros(64, dtype=torch.int32, device=d["x"].device)
    P0, _ = plain.partner_probabilities(d["w"], tq, nq, wl.sigma)
    P1, _ = staged.partner_probabilities(d["w"], tq, nq, wl.sigma, weights_staged=True)
    assert torch.equal(P0, P1)
    # a backward stages other weights; a plain build stages none
    staged.backward(d["w"], torch.ones_like(d["w"]), d["tgt"], sigma=wl.sigma, want=("w",))
    for t in (staged, plain.build(d["x"], d["y"], d["z"])):
        with pytest.raises(msp.MspError) as e:
            t.forward(d["w"], d["tgt"], sigma=wl.sigma, weights_staged=True)
        assert e.value.code == msp.MSP_ESTATE
