"""The 4,194,304-neuron slab (10 x 10 x 2 mm, sigma 750 um) against the FP64
oracle, at 65,536 seeded targets plus every target within one p = 8 expansion
cell of a corner of the slab and 8,192 targets near its x and y faces:

* max per-target relative error <= 1e-4 for p = 4, 6, 8, 10, with the
  Hermite-to-Taylor translation in fp32 on the matrix cores and as split
  bfloat16 products;
* sampled cells of the p = 8 moment grid (the matrix-core P2M at full size)
  against the oracle's P2M over the cell's points;
* the two-level variant (sub-cell moments shifted up by M2M, Taylor series
  shifted down by L2L), at full size against the oracle's sums, and pass by pass
  against the oracle's P2M, M2M, M2L, L2L and L2P on a small grid."""
import numpy as np
import pytest

import synth
from oracle import fgt as ofgt
from oracle import octree
from tests.helpers import rel_err, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def slab_tree(slab_reference):
    import paper_2301_10570_amd as msp
    wl = slab_reference[0]
    d = to_dev(wl)
    return msp.build_tree(d["x"], d["y"], d["z"], leaf_max=wl.leaf_max), d


def _report(err, where):
    parts = []
    for g, idx in where.items():
        e = err[idx]
        parts.append(f"{g}[{idx.size}] max {e.max():.2e} p99 {np.quantile(e, 0.99):.2e}")
    return "; ".join(parts)


@pytest.mark.parametrize("m2l", ["mfma", "bf16x3"])
@pytest.mark.parametrize("p", [4, 6, 8, 10])
def test_slab4m_accuracy(slab_reference, slab_tree, p, m2l):
    wl, sel, ref, where = slab_reference
    tree, d = slab_tree
    print(f"slab 4M p={p} m2l={m2l}", flush=True)
    u = tree.forward(d["w"], d["tgt"], sigma=wl.sigma, p=p, route="fgt", m2l=m2l).cpu().numpy()
    err = rel_err(u[sel], ref)
    print(f"  plan={tree.plan(wl.sigma, p=p, route='fgt')}\n  {_report(err, where)}", flush=True)
    assert err.max() <= TOL
    assert tree.plan(wl.sigma, p=8)["route"] == "fgt"   # the transform is what the default picks here


def test_slab4m_moment_grid_cells(slab_reference, slab_tree):
    """Matrix-core P2M (p = 8) at full size: 24 seeded occupied cells of the
    moment grid against the oracle's FP64 moments of the cell's points."""
    wl, _, _, _ = slab_reference
    tree, d = slab_tree
    p = 8
    print("slab 4M moment grid, 24 cells vs oracle P2M", flush=True)
    tree.forward(d["w"], d["tgt"], sigma=wl.sigma, p=p, route="fgt")
    plan = tree.plan(wl.sigma, p=p, route="fgt")
    level, G = plan["level"], plan["grid"]
    A = tree.debug_buffer(0).cpu().numpy().reshape(G[2], p, G[1], p, G[0], p)
    pos = wl.pos64()
    lo, side = octree.root_cube(pos[:, 0], pos[:, 1], pos[:, 2])
    scale = float(2 ** octree.DEPTH) / side
    shift = np.uint64(octree.DEPTH - level)
    ijk = np.stack([(octree.quantise(pos[:, k], lo[k], scale) >> shift).astype(np.int64) for k in range(3)], 1)
    flat = (ijk[:, 2] * G[1] + ijk[:, 1]) * G[0] + ijk[:, 0]
    occupied = np.unique(flat)
    pick = occupied[synth.sample_indices(occupied.size, 24, seed=305)]
    worst = 0.0
    for c in pick:
        m = flat == c
        cx, cy, cz = c % G[0], (c // G[0]) % G[1], c // (G[0] * G[1])
        a_ref = ofgt.p2m(pos[m], wl.w[m].astype(np.float64), ofgt.cell_centre(lo, side, level, (cx, cy, cz)),
                         wl.sigma, p)
        a_gpu = A[cz, :, cy, :, cx, :].transpose(2, 1, 0)
        e = np.abs(a_gpu - a_ref).max() / np.abs(a_ref).max()
        worst = max(worst, e)
        assert e <= 1e-5, (c, int(m.sum()), e)
    print(f"  worst |dA|/max|A| {worst:.2e}")


def test_slab4m_two_level(slab_reference, slab_tree):
    wl, sel, ref, where = slab_reference
    tree, d = slab_tree
    print("slab 4M two-level (M2M / L2L) p=8", flush=True)
    plan2 = tree.plan(wl.sigma, p=8, two_level=True)
    assert plan2["fine_terms"] > 0
    u2 = tree.forward(d["w"], d["tgt"], sigma=wl.sigma, p=8, two_level=True).cpu().numpy()
    err = rel_err(u2[sel], ref)
    print(f"  plan={plan2}\n  {_report(err, where)}")
    assert err.max() <= TOL


def test_two_level_passes_vs_oracle():
    """Two-level route on a 2 x 1 x 1 grid (level forced): the moment grid after
    M2M equals the oracle's P2M at the 64 sub-cells of each cell (fine_terms terms),
    shifted to the cell centre by the oracle's M2M; the Taylor grid equals the
    oracle's M2L of those moments; every target's sum equals the oracle's L2L of
    that Taylor series to its sub-cell, truncated to fine_terms terms, evaluated by
    the oracle's L2P."""
    import paper_2301_10570_amd as msp
    # the root cube's side is the x extent (just under 400 um): y and z stay below
    # 190 um, inside the first level-1 cell
    wl = synth.uniform_box(20000, extent=(400.0, 190.0, 190.0), sigma=300.0, seed=33)
    p, level = 8, 1
    d = to_dev(wl)
    tree = msp.build_tree(d["x"], d["y"], d["z"], leaf_max=wl.leaf_max)
    plan = tree.plan(wl.sigma, p=p, level=level, route="fgt", two_level=True)
    pf = plan["fine_terms"]
    print(f"two-level passes vs oracle: plan {plan}", flush=True)
    assert pf > 0 and plan["grid"] == [2, 1, 1]
    u = tree.forward(d["w"], d["tgt"], sigma=wl.sigma, p=p, level=level, route="fgt", two_level=True)
    u = u.cpu().numpy()
    G = plan["grid"]
    A = tree.debug_buffer(0).cpu().numpy().reshape(G[2], p, G[1], p, G[0], p)
    C = tree.debug_buffer(1).cpu().numpy().reshape(G[2], p, G[1], p, G[0], p)
    pos = wl.pos64()
    w = wl.w.astype(np.float64)
    lo, side = octree.root_cube(pos[:, 0], pos[:, 1], pos[:, 2])
    scale = float(2 ** octree.DEPTH) / side
    q = np.stack([octree.quantise(pos[:, k], lo[k], scale) for k in range(3)], 1)
    cell = (q >> np.uint64(octree.DEPTH - level)).astype(np.int64)
    sub = (q >> np.uint64(octree.DEPTH - level - 2)).astype(np.int64)
    cells = [(0, 0, 0), (1, 0, 0)]
    centres = [ofgt.cell_centre(lo, side, level, c) for c in cells]
    A_ref = []
    for ci, c in enumerate(cells):
        acc = np.zeros((p, p, p))
        in_cell = np.all(cell == c, axis=1)
        for s in np.unique(sub[in_cell], axis=0):
            m = in_cell & np.all(sub == s, axis=1)
            a = np.zeros((p, p, p))
            a[:pf, :pf, :pf] = ofgt.p2m(pos[m], w[m], ofgt.cell_centre(lo, side, level + 2, s), wl.sigma, pf)
            acc += ofgt.m2m(a, ofgt.cell_centre(lo, side, level + 2, s), centres[ci], wl.sigma)
        A_ref.append(acc)
        a_gpu = A[c[2], :, c[1], :, c[0], :].transpose(2, 1, 0)
        assert np.abs(a_gpu - acc).max() <= 1e-5 * np.abs(acc).max(), ci
    C_ref = []
    for ti, t in enumerate(cells):
        c_ref = sum(ofgt.m2l(A_ref[si], centres[si], centres[ti], wl.sigma) for si in range(len(cells)))
        C_ref.append(c_ref)
        c_gpu = C[t[2], :, t[1], :, t[0], :].transpose(2, 1, 0)
        assert np.abs(c_gpu - c_ref).max() <= 1e-4 * np.abs(c_ref).max(), ti
    tgt = wl.a > 0
    u_ref = np.zeros(wl.n)
    for ti, t in enumerate(cells):
        in_cell = np.all(cell == t, axis=1)
        for s in np.unique(sub[in_cell], axis=0):
            m = in_cell & np.all(sub == s, axis=1) & tgt
            if not m.any():
                continue
            cs = ofgt.cell_centre(lo, side, level + 2, s)
            cl = ofgt.l2l(C_ref[ti], centres[ti], cs, wl.sigma)[:pf, :pf, :pf]
            u_ref[m] = ofgt.l2p(cl, cs, pos[m], wl.sigma)
    e = rel_err(u[tgt], u_ref[tgt])
    print(f"  fine_terms {pf}: max rel diff from the oracle's two-level chain {e.max():.2e}")
    assert e.max() <= 2e-5
