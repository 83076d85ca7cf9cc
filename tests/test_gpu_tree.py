"""GPU octree vs the oracle octree: bit-exact keys, permutation and node table."""
import numpy as np
import pytest

import synth
from oracle import octree
from tests.helpers import to_dev

pytestmark = pytest.mark.gpu


def _gpu_tree(x, y, z, leaf_max=64, max_depth=21):
    import torch
    import paper_2301_10570_amd as msp
    dev = torch.device("cuda", 0)
    tx, ty, tz = (torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).to(dev) for v in (x, y, z))
    tree = msp.build_tree(tx, ty, tz, leaf_max=leaf_max, max_depth=max_depth)
    out = {k: v.cpu().numpy() for k, v in tree.export().items()}
    return tree, out


def _compare(x, y, z, leaf_max=64, max_depth=21):
    ref = octree.build(x, y, z, leaf_max=leaf_max, max_depth=max_depth)
    tree, got = _gpu_tree(x, y, z, leaf_max, max_depth)
    info = tree.info()
    assert info["n_nodes"] == ref.n_nodes
    assert info["side"] == ref.side
    assert np.array_equal(np.asarray(info["lo"]), ref.lo)
    assert np.array_equal(got["keys"].view(np.uint64), ref.keys)
    assert np.array_equal(got["perm"].astype(np.int64), ref.perm)
    assert np.array_equal(got["node_level"], ref.level)
    assert np.array_equal(got["node_first"], ref.first)
    assert np.array_equal(got["node_count"], ref.count)
    assert np.array_equal(got["node_parent"], ref.parent)
    assert np.array_equal(got["node_first_child"], ref.first_child)
    assert np.array_equal(got["node_n_children"], ref.n_children)
    assert np.array_equal(got["node_digit"], ref.digit)
    assert np.array_equal(got["node_ix"], ref.ix)
    assert np.array_equal(got["node_iy"], ref.iy)
    assert np.array_equal(got["node_iz"], ref.iz)
    lo = np.asarray(info["level_offset"][:len(ref.level_offset)])
    assert np.array_equal(lo, ref.level_offset)
    _check_records(tree, x, y, z, ref.perm)
    tree.close()


def _check_records(tree, x, y, z, perm, w=None):
    """The points in key order (and the weights, for a weighted build) are the
    inputs through the permutation, bit for bit, and the inverse permutation
    inverts it."""
    n = perm.size
    rec = tree.debug_buffer(8).cpu().numpy().reshape(n, 4)
    for k, v in enumerate((x, y, z) if w is None else (x, y, z, w)):
        assert np.array_equal(rec[:, k], np.asarray(v, np.float32)[perm]), k
    ip = tree.debug_buffer(9).cpu().numpy()
    assert np.array_equal(ip[perm], np.arange(n, dtype=np.int32))


@pytest.mark.parametrize("make,scale", [("uniform4k", 1.0), ("blobs262k", 1.0), ("slab4m", 0.0625)])
def test_tree_bitexact_workloads(make, scale):
    wl = getattr(synth, make)(scale)
    print(f"tree bit-exact: {make} x {scale} n={wl.n}", flush=True)
    _compare(wl.x, wl.y, wl.z)


@pytest.mark.parametrize("leaf_max,max_depth", [(1, 21), (7, 21), (64, 3), (100, 21), (64, 0), (1500, 21)])
def test_tree_bitexact_params(leaf_max, max_depth):
    wl = synth.blobs(6, 700, extent=1500.0, std=40.0, seed=12)
    print(f"tree params leaf_max={leaf_max} max_depth={max_depth}", flush=True)
    _compare(wl.x, wl.y, wl.z, leaf_max, max_depth)


def test_tree_full_slab():
    """4,194,304 points: the full slab workload."""
    wl = synth.slab4m()
    print("tree bit-exact: full slab", flush=True)
    _compare(wl.x, wl.y, wl.z)


def test_weighted_build_records():
    """A weighted build carries the weights into key order with the positions."""
    import torch
    import paper_2301_10570_amd as msp
    wl = synth.slab4m(0.0625)
    print("weighted build records, slab 1/16", flush=True)
    ref = octree.build(wl.x, wl.y, wl.z, leaf_max=wl.leaf_max)
    d = to_dev(wl)
    tree = msp.Tree()
    tree.build(d["x"], d["y"], d["z"], leaf_max=wl.leaf_max, w=d["w"])
    _check_records(tree, wl.x, wl.y, wl.z, ref.perm, wl.w)
    tree.close()


def test_tree_edge_cases():
    z1 = np.zeros(1, np.float32)
    print("tree edge: n=1", flush=True)
    _compare(z1, z1, z1)
    print("tree edge: duplicates", flush=True)
    x = np.zeros(300, np.float32)
    x[:5] = [1, 2, 3, 4, 5]
    _compare(x, np.zeros(300, np.float32), np.zeros(300, np.float32), leaf_max=10)
    print("tree edge: identical points", flush=True)
    _compare(np.full(200, 3.5, np.float32), np.full(200, -1.0, np.float32), np.full(200, 7.0, np.float32), 16)
    print("tree edge: planar", flush=True)
    rng = np.random.default_rng(3)
    _compare(rng.random(5000).astype(np.float32), rng.random(5000).astype(np.float32),
             np.zeros(5000, np.float32), 8)
    print("tree edge: n = leaf_max and n = leaf_max + 1", flush=True)
    wl = synth.uniform_box(65, seed=5)
    _compare(wl.x[:64], wl.y[:64], wl.z[:64], 64)
    _compare(wl.x, wl.y, wl.z, 64)
    print("tree edge: runs of ~100 points in one level-8 cell, across wavefront boundaries", flush=True)
    rng = np.random.default_rng(21)
    ctr = rng.random((40, 3)) * 1000.0
    pts = (np.repeat(ctr, 100, axis=0) + rng.random((4000, 3)) * 0.5).astype(np.float32)
    pts = pts[rng.permutation(4000)]
    _compare(pts[:, 0].copy(), pts[:, 1].copy(), pts[:, 2].copy(), 16)
    print("tree edge: ragged sizes around the 4096-point tile", flush=True)
    for n in (4095, 4096, 4097, 12289):
        wl = synth.uniform_box(n, seed=n)
        _compare(wl.x, wl.y, wl.z, 5)


def test_tree_unaligned_views():
    """Coordinates passed as views at an offset of one float (no 16-byte loads in
    the bounding box pass) give the same tree as aligned arrays."""
    import torch
    import paper_2301_10570_amd as msp
    wl = synth.uniform_box(10001, seed=31)
    print("tree: unaligned coordinate views", flush=True)
    ref = octree.build(wl.x[1:], wl.y[1:], wl.z[1:], leaf_max=16)
    dev = torch.device("cuda", 0)
    tx, ty, tz = (torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).to(dev) for v in (wl.x, wl.y, wl.z))
    tree = msp.build_tree(tx[1:], ty[1:], tz[1:], leaf_max=16)
    got = {k: v.cpu().numpy() for k, v in tree.export().items()}
    assert tree.info()["side"] == ref.side
    assert np.array_equal(got["keys"].view(np.uint64), ref.keys)
    assert np.array_equal(got["perm"].astype(np.int64), ref.perm)
    tree.close()


def test_tree_empty():
    import torch
    import paper_2301_10570_amd as msp
    e = torch.zeros(0, dtype=torch.float32, device="cuda")
    tree = msp.build_tree(e, e, e)
    info = tree.info()
    assert info["n"] == 0 and info["n_nodes"] == 1
    ex = tree.export()
    assert ex["node_count"].cpu().tolist() == [0] and ex["node_n_children"].cpu().tolist() == [0]


def test_tree_rejects_nonfinite_and_bad_args():
    import torch
    import paper_2301_10570_amd as msp
    x = torch.zeros(10, dtype=torch.float32, device="cuda")
    y = x.clone()
    y[3] = float("nan")
    with pytest.raises(msp.MspError) as e:
        msp.build_tree(x, y, x)
    assert e.value.code == msp.MSP_EINVAL
    with pytest.raises(msp.MspError):
        msp.build_tree(x, x, x, leaf_max=0)
    with pytest.raises(msp.MspError):
        msp.build_tree(x, x, x, max_depth=22)
