"""Oracle child probabilities for the proportional partner choice (Algorithm 2).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

For a query (target neuron i, octree node X) the attraction of each child c of
X is the restricted direct sum S_c = sum_{j in c} w_j exp(-|t_i - s_j|^2/sigma^2)
(Eq. (8) over the sources below c), and the probability of c is S_c divided by
the sum over X's children.  Probabilities are indexed by the child's octant
(0..7, bit 2 = x, bit 1 = y, bit 0 = z); absent children get 0.

The choice draws r in [0, 1) and takes the first child, in octant order, whose
inclusive running sum of S exceeds r * total (the paper's upper_bound over the
probabilities, read as a search in their running sums).  A node whose children
carry no weight (total 0), or a leaf, gives choice -1.
"""
from __future__ import annotations

import numpy as np

from . import gauss_sum


def probabilities(tree, pos, w, sigma, target_idx, node_idx, uniforms=None, exclude_self=False):
    """Returns (P[nq, 8] float64, S[nq, 8] float64, choice[nq] int64 node ids)."""
    pos = np.asarray(pos, np.float64)
    w = np.asarray(w, np.float64)
    nq = len(target_idx)
    P = np.zeros((nq, 8))
    S = np.zeros((nq, 8))
    choice = np.full(nq, -1, np.int64)
    for q in range(nq):
        i, X = int(target_idx[q]), int(node_idx[q])
        if tree.is_leaf[X]:
            continue
        fc, nc = int(tree.first_child[X]), int(tree.n_children[X])
        t = pos[i:i + 1]
        for c in range(fc, fc + nc):
            idx = tree.perm[tree.first[c]:tree.first[c] + tree.count[c]]
            keep = w[idx] != 0
            if exclude_self:
                keep &= idx != i
            idx = idx[keep]
            if idx.size:
                S[q, tree.digit[c]] = gauss_sum(t, pos[idx], w[idx], sigma)[0]
        total = S[q].sum()
        if total > 0:
            P[q] = S[q] / total
            if uniforms is not None:
                target = float(uniforms[q]) * total
                run = np.cumsum(S[q])
                d = int(np.nonzero(run > target)[0][0]) if np.any(run > target) else int(np.nonzero(S[q])[0][-1])
                # the child node with octant d
                for c in range(fc, fc + nc):
                    if tree.digit[c] == d:
                        choice[q] = c
    return P, S, choice
