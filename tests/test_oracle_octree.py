"""Pins for the oracle octree (section "A Distributed Octree", split while a
cell holds more than leaf_max neurons)."""
import numpy as np
import pytest

import synth
from oracle import octree


def test_interleave_bit_positions():
    one = np.array([1], np.uint64)
    zero = np.array([0], np.uint64)
    assert int(octree.interleave(one, zero, zero)[0]) == 4
    assert int(octree.interleave(zero, one, zero)[0]) == 2
    assert int(octree.interleave(zero, zero, one)[0]) == 1
    top = np.array([1 << 20], np.uint64)
    assert int(octree.interleave(top, zero, zero)[0]) == 1 << 62
    full = np.array([(1 << 21) - 1], np.uint64)
    assert int(octree.interleave(full, full, full)[0]) == (1 << 63) - 1
    q = np.array([0b101, 0b011], np.uint64)
    r = np.array([0b110, 0b000], np.uint64)
    s = np.array([0b011, 0b111], np.uint64)
    k = octree.interleave(q, r, s)
    # digits (x,y,z) for bits 2,1,0 of q,r,s: (1,1,0),(0,1,1),(1,0,1) -> 6,3,5
    assert int(k[0]) == (6 << 6) | (3 << 3) | 5
    ix, iy, iz = octree.deinterleave(k, 21)
    assert ix.tolist() == [5, 3] and iy.tolist() == [6, 0] and iz.tolist() == [3, 7]


def test_lattice_closed_form():
    """A 64^3 lattice with leaf_max 64: every level-4 cell holds exactly 4^3
    lattice points, so there are 16^3 leaves at level 4 and 1+8+64+512 inner
    nodes."""
    g = np.arange(64, dtype=np.float32)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    t = octree.build(X.ravel(), Y.ravel(), Z.ravel(), leaf_max=64)
    assert t.n_nodes == 585 + 4096
    assert np.all(t.is_leaf[t.level == 4] == 1) and np.sum(t.level == 4) == 4096
    assert np.sum(t.is_leaf == 0) == 585
    assert np.all(t.count[t.level == 4] == 64)


def _check_tree(t, x, y, z, leaf_max, max_depth=21):
    n = x.shape[0]
    pos = np.stack([x, y, z], 1).astype(np.float64)
    # sorted keys, permutation is a permutation, stability for equal keys
    assert np.all(np.diff(t.keys.astype(np.float64)) >= 0) or np.all(t.keys[1:] >= t.keys[:-1])
    assert np.array_equal(np.sort(t.perm), np.arange(n))
    eq = t.keys[1:] == t.keys[:-1]
    assert np.all(t.perm[1:][eq] > t.perm[:-1][eq])
    leaves = np.nonzero(t.is_leaf)[0]
    # leaves partition [0, n) in order
    order = np.argsort(t.first[leaves], kind="stable")
    lf = leaves[order]
    if n:
        assert t.first[lf[0]] == 0
        assert np.all(t.first[lf[1:]] == t.first[lf[:-1]] + t.count[lf[:-1]])
        assert t.first[lf[-1]] + t.count[lf[-1]] == n
    for v in range(t.n_nodes):
        if t.is_leaf[v]:
            assert t.count[v] <= leaf_max or t.level[v] == max_depth
            # every point lies inside its leaf's cell (geometric check)
            c, h = octree.node_box(t, v)
            pts = pos[t.perm[t.first[v]:t.first[v] + t.count[v]]]
            assert np.all(pts >= c - h - 1e-9 * t.side) and np.all(pts <= c + h + 1e-9 * t.side)
        else:
            assert t.count[v] > leaf_max
            fc, nc = t.first_child[v], t.n_children[v]
            assert 1 <= nc <= 8
            assert t.count[fc:fc + nc].sum() == t.count[v]
            assert np.all(t.parent[fc:fc + nc] == v)
            assert np.all(t.level[fc:fc + nc] == t.level[v] + 1)
            assert t.first[fc] == t.first[v]
            assert np.all(np.diff(t.digit[fc:fc + nc]) > 0)
    # breadth-first: levels non-decreasing, firsts increasing within a level
    assert np.all(np.diff(t.level) >= 0)
    for l in range(len(t.level_offset) - 1):
        f = t.first[t.level_offset[l]:t.level_offset[l + 1]]
        assert np.all(np.diff(f) > 0)


def test_tree_properties_uniform():
    wl = synth.uniform_box(3000, seed=2)
    t = octree.build(wl.x, wl.y, wl.z, leaf_max=16)
    _check_tree(t, wl.x, wl.y, wl.z, 16)


def test_tree_properties_blobs():
    wl = synth.blobs(5, 400, extent=2000.0, std=30.0, seed=3)
    t = octree.build(wl.x, wl.y, wl.z, leaf_max=20)
    _check_tree(t, wl.x, wl.y, wl.z, 20)


def test_brute_force_membership():
    """Rebuild leaf membership by brute force: a point belongs to the cell of
    level l and lattice (i, j, k) iff floor-quantised coordinates match; each
    leaf must hold exactly the points whose level-l lattice cell is its own."""
    wl = synth.uniform_box(500, seed=4)
    t = octree.build(wl.x, wl.y, wl.z, leaf_max=8)
    lo, side = octree.root_cube(wl.x, wl.y, wl.z)
    scale = 2.0 ** 21 / side
    q = np.stack([octree.quantise(v, lo[k], scale) for k, v in enumerate((wl.x, wl.y, wl.z))], 1)
    for v in np.nonzero(t.is_leaf)[0]:
        l = int(t.level[v])
        cell = q >> np.uint64(21 - l)
        mine = np.nonzero((cell[:, 0] == t.ix[v]) & (cell[:, 1] == t.iy[v]) & (cell[:, 2] == t.iz[v]))[0]
        got = np.sort(t.perm[t.first[v]:t.first[v] + t.count[v]])
        assert np.array_equal(mine, got)


def test_duplicates_beyond_leaf_max_reach_max_depth():
    x = np.zeros(100, np.float32)
    y = np.zeros(100, np.float32)
    z = np.zeros(100, np.float32)
    x[0] = 1.0
    t = octree.build(x, y, z, leaf_max=10)
    deepest = int(t.level.max())
    assert deepest == 21
    big = np.nonzero((t.is_leaf == 1) & (t.count > 10))[0]
    assert len(big) == 1 and t.level[big[0]] == 21 and t.count[big[0]] == 99
    t2 = octree.build(x, y, z, leaf_max=10, max_depth=5)
    assert int(t2.level.max()) == 5


def test_small_and_degenerate():
    t = octree.build(np.zeros(1, np.float32), np.zeros(1, np.float32), np.zeros(1, np.float32))
    assert t.n_nodes == 1 and t.is_leaf[0] == 1 and t.side == 1.0
    wl = synth.uniform_box(64, seed=1)
    t = octree.build(wl.x, wl.y, wl.z, leaf_max=64)
    assert t.n_nodes == 1
    t = octree.build(wl.x, wl.y, wl.z, leaf_max=63)
    assert t.n_nodes > 1 and t.is_leaf[0] == 0
