"""Oracle octree: Morton keys, stable sort and the adaptive node table.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper inserts neurons into an octree that splits a cell into eight until
it holds few enough neurons; inner nodes aggregate the vacant elements of their
children (section "A Distributed Octree").  Here a cell splits while it holds
more than leaf_max neurons and its level is below max_depth (21, the depth a
63-bit Morton key resolves).  This module writes that definition out directly,
top-down and level by level, in numpy:

root cube   lo_k = min_i x_ik, side = max_k (max_i x_ik - lo_k), side := 1 if 0
quantise    q_k = min(floor((x_k - lo_k) * (2^21 / side)), 2^21 - 1), in float64
            (one subtraction, then one multiplication, both rounded)
key         bit b of q_x, q_y, q_z lands at bits 3b+2, 3b+1, 3b
order       stable sort by key (equal keys keep input order)
nodes       breadth-first: by level, then by key prefix (Morton order)
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

DEPTH = 21
QMAX = (1 << DEPTH) - 1


def root_cube(x: np.ndarray, y: np.ndarray, z: np.ndarray):
    """Lower corner and side of the root cube, in float64 (origin and 1 when empty)."""
    if np.asarray(x).size == 0:
        return np.zeros(3), 1.0
    lo = np.array([np.float64(np.min(x)), np.float64(np.min(y)), np.float64(np.min(z))])
    hi = np.array([np.float64(np.max(x)), np.float64(np.max(y)), np.float64(np.max(z))])
    side = float(np.max(hi - lo))
    if side == 0.0:
        side = 1.0
    return lo, side


def quantise(v: np.ndarray, lo: float, scale: float) -> np.ndarray:
    q = np.floor((v.astype(np.float64) - lo) * scale)
    return np.minimum(q, QMAX).astype(np.uint64)


def interleave(qx: np.ndarray, qy: np.ndarray, qz: np.ndarray) -> np.ndarray:
    """Bit b of qx goes to 3b+2, of qy to 3b+1, of qz to 3b."""
    key = np.zeros(qx.shape, dtype=np.uint64)
    one = np.uint64(1)
    for b in range(DEPTH):
        bb = np.uint64(b)
        key |= ((qx >> bb) & one) << np.uint64(3 * b + 2)
        key |= ((qy >> bb) & one) << np.uint64(3 * b + 1)
        key |= ((qz >> bb) & one) << np.uint64(3 * b)
    return key


def deinterleave(prefix: np.ndarray, level: int):
    """Lattice coordinates (ix, iy, iz) of cells given their level-`level` prefixes."""
    p = prefix.astype(np.uint64)
    ix = np.zeros(p.shape, np.int64)
    iy = np.zeros(p.shape, np.int64)
    iz = np.zeros(p.shape, np.int64)
    for b in range(level):
        t = (p >> np.uint64(3 * b)) & np.uint64(7)
        ix |= ((t >> np.uint64(2)) & np.uint64(1)).astype(np.int64) << b
        iy |= ((t >> np.uint64(1)) & np.uint64(1)).astype(np.int64) << b
        iz |= (t & np.uint64(1)).astype(np.int64) << b
    return ix, iy, iz


def morton_keys(x, y, z):
    lo, side = root_cube(x, y, z)
    scale = float(2 ** DEPTH) / side
    key = interleave(quantise(x, lo[0], scale), quantise(y, lo[1], scale),
                     quantise(z, lo[2], scale))
    return key, lo, side


@dataclass
class Octree:
    keys: np.ndarray       # uint64, sorted
    perm: np.ndarray       # int64, perm[k] = input index of the k-th sorted point
    lo: np.ndarray         # float64[3]
    side: float
    level: np.ndarray      # per node, int32
    first: np.ndarray      # first sorted point
    count: np.ndarray      # number of points
    parent: np.ndarray     # -1 for the root
    first_child: np.ndarray  # -1 for a leaf
    n_children: np.ndarray
    is_leaf: np.ndarray    # uint8
    digit: np.ndarray      # octant of the node inside its parent (0 for the root)
    ix: np.ndarray
    iy: np.ndarray
    iz: np.ndarray
    level_offset: np.ndarray  # start of each level in node order; length depth+2

    @property
    def n_nodes(self) -> int:
        return int(self.level.shape[0])


def build(x, y, z, leaf_max: int = 64, max_depth: int = DEPTH) -> Octree:
    """Adaptive octree exactly as described in the module docstring."""
    n = int(x.shape[0])
    keys_in, lo, side = morton_keys(x, y, z)
    perm = np.argsort(keys_in, kind="stable").astype(np.int64)
    keys = keys_in[perm]

    # level 0: the root covers every point
    lv_first = [np.array([0], np.int64)]
    lv_count = [np.array([n], np.int64)]
    lv_parent = [np.array([-1], np.int64)]
    lv_digit = [np.array([0], np.int64)]
    level = 0
    while level < max_depth:
        f, c = lv_first[-1], lv_count[-1]
        split = np.nonzero(c > leaf_max)[0]
        if split.size == 0:
            break
        shift = np.uint64(3 * (DEPTH - level - 1))
        sf, sc = f[split], c[split]
        # the parent's key prefix at `level`, then the 8 child prefixes
        pref = keys[sf] >> np.uint64(3 * (DEPTH - level))
        bounds = np.empty((split.size, 9), np.int64)
        for d in range(8):
            child_lo = ((pref << np.uint64(3)) | np.uint64(d)) << shift
            bounds[:, d] = np.searchsorted(keys, child_lo, side="left")
        bounds[:, 8] = sf + sc
        bounds[:, 0] = sf
        cf, cc, cp, cd = [], [], [], []
        node_base = sum(a.size for a in lv_first[:-1])   # index of this level's first node
        for d in range(8):
            cnt = bounds[:, d + 1] - bounds[:, d]
            keep = cnt > 0
            cf.append(np.stack([bounds[keep, d], cnt[keep], node_base + split[keep],
                                np.full(int(keep.sum()), d)], axis=1))
        allc = np.concatenate(cf, axis=0)
        # breadth-first within the level means Morton order = order of first point
        allc = allc[np.argsort(allc[:, 0], kind="stable")]
        lv_first.append(allc[:, 0].copy())
        lv_count.append(allc[:, 1].copy())
        lv_parent.append(allc[:, 2].copy())
        lv_digit.append(allc[:, 3].copy())
        level += 1

    sizes = [a.size for a in lv_first]
    level_offset = np.zeros(len(sizes) + 1, np.int64)
    level_offset[1:] = np.cumsum(sizes)
    first = np.concatenate(lv_first)
    count = np.concatenate(lv_count)
    parent = np.concatenate(lv_parent)
    digit = np.concatenate(lv_digit)
    lev = np.concatenate([np.full(s, l, np.int32) for l, s in enumerate(sizes)])
    nn = first.size
    first_child = np.full(nn, -1, np.int64)
    n_children = np.zeros(nn, np.int64)
    if nn > 1:
        ch = np.arange(1, nn)
        par = parent[1:]
        # children of one parent are contiguous; record the first and count
        np.add.at(n_children, par, 1)
        firsts = np.full(nn, nn, np.int64)
        np.minimum.at(firsts, par, ch)
        has = n_children > 0
        first_child[has] = firsts[has]
    is_leaf = (n_children == 0).astype(np.uint8)
    ix = np.zeros(nn, np.int64)
    iy = np.zeros(nn, np.int64)
    iz = np.zeros(nn, np.int64)
    for l in range(len(sizes)):
        s, e = level_offset[l], level_offset[l + 1]
        pref = keys[first[s:e]] >> np.uint64(3 * (DEPTH - l))
        ix[s:e], iy[s:e], iz[s:e] = deinterleave(pref, l)
    return Octree(keys, perm, lo, side, lev, first, count, parent, first_child, n_children,
                  is_leaf, digit, ix, iy, iz, level_offset)


def node_box(tree: Octree, node: int):
    """Geometric centre and half-side (float64) of a node's cell."""
    l = int(tree.level[node])
    h = tree.side / (1 << l)
    c = tree.lo + (np.array([tree.ix[node], tree.iy[node], tree.iz[node]], np.float64) + 0.5) * h
    return c, 0.5 * h
