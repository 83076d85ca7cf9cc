"""Oracle of the paper's partner descent: Algorithm 1 (pairs of an axon-side and
a dendrite-side item of the octree, descended step by step) driven by the
proportional choice of Algorithm 2, then the acceptance of the requests at the
dendrites.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Items.  An item is an octree node v (encoded v >= 0) or one neuron with input
index i (encoded -(i + 1)).  A neuron is the paper's leaf.  The children of an
inner node are its child nodes in octant order; the children of a leaf node of
the octree (which holds up to leaf_max neurons) are its neurons in key order; a
neuron has none ("single").

Attraction between the axons of an item S and the dendrites of an item C:
    Att(S, C) = sum_{i in S} sum_{j in C, j != i} a_i w_j exp(-|t_i - s_j|^2 / sigma^2)
(the kernel of Eq. (8) weighted by vacant axonal elements a and vacant dendritic
elements w; no self pair).  Algorithm 2 evaluates this sum directly or from
Hermite / Taylor expansions depending on the element counts; the oracle sums it
directly in FP64.

One step maps a frontier of pairs (S, T) to the next frontier and a list of
requests:
  S, T single                   request (S -> T)
  S single, T not               T' = choice over the children C of T with values
                                Att(S, C); pair (S, T')
  S not single, T single        S' = choice over the children of S with values
                                Att(child, T); pair (S', T)
  neither single                for every child S_c of S that holds axons:
                                T' = choice over the children C of T with values
                                Att(S_c, C); pair (S_c, T')
A choice whose values are all 0 drops its pair.  A choice draws r in [0, 1)
from the counter-based generator below, keyed by (seed, step, choosing item),
and takes the first candidate whose inclusive running sum exceeds r * total
(the last positive one if rounding leaves none).  The descent starts from
(root, root) and steps until the frontier is empty.

Acceptance: dendrite neuron j takes at most floor(w_j) of the requests naming
it, those with the smallest priority (generator keyed by (seed, axon input
index)), ties by axon index.

Generator: SplitMix64 (the published generator of Steele, Lea and Flood, 2014,
as in its reference C implementation): state += 0x9E3779B97F4A7C15, then
z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9, z = (z ^ (z >> 27)) * 0x94D049BB133111EB,
output z ^ (z >> 31), all modulo 2^64.  mix(x) is the output for state x.
    uniform(seed, step, item) = (mix(mix(seed ^ ((step + 1) * 0x9E3779B97F4A7C15)) ^ item) >> 11) * 2^-53
    priority(seed, axon)      = mix(mix(seed ^ 0xD1B54A32D192ED03) ^ axon)
with item and axon taken modulo 2^64 (two's complement).
"""
from __future__ import annotations

import numpy as np

from . import gauss_sum

M64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
PRIORITY_STREAM = 0xD1B54A32D192ED03


def splitmix64_next(state: int):
    """One step of SplitMix64: returns (new state, output)."""
    state = (state + GAMMA) & M64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return state, z ^ (z >> 31)


def mix(x: int) -> int:
    return splitmix64_next(x & M64)[1]


def uniform(seed: int, step: int, item: int) -> float:
    v = mix(mix((seed ^ (((step + 1) * GAMMA) & M64)) & M64) ^ (item & M64))
    return (v >> 11) * (2.0 ** -53)


def priority(seed: int, axon: int) -> int:
    return mix(mix((seed ^ PRIORITY_STREAM) & M64) ^ (axon & M64))


def choose(values, r: float) -> int:
    """Index chosen by r in [0, 1) from non-negative values, or -1 (all zero)."""
    v = np.asarray(values, np.float64)
    total = float(v.sum())
    if not total > 0.0:
        return -1
    target = r * total
    run = 0.0
    last = -1
    for k, x in enumerate(v):
        if x > 0.0:
            last = k
        run += x
        if run > target and x > 0.0:
            return k
    return last


def margin(values, r: float) -> float:
    """Distance of r * total to the nearest interior boundary of the running sums,
    relative to the total (inf when there is at most one positive value)."""
    v = np.asarray(values, np.float64)
    total = float(v.sum())
    pos = np.nonzero(v > 0)[0]
    if total <= 0.0 or pos.size < 2:
        return float("inf")
    run = np.cumsum(v)[pos[:-1]]
    return float(np.min(np.abs(run - r * total)) / total)


class Descent:
    """The tree and the neuron data of one descent (positions, a, w, sigma)."""

    def __init__(self, tree, pos, a, w, sigma):
        self.tree = tree
        self.pos = np.asarray(pos, np.float64)
        self.a = np.asarray(a, np.float64)
        self.w = np.asarray(w, np.float64)
        self.sigma = float(sigma)

    # items -------------------------------------------------------------------
    def children(self, item: int):
        t = self.tree
        if item < 0:
            return []
        if t.n_children[item] > 0:
            fc, nc = int(t.first_child[item]), int(t.n_children[item])
            return sorted(range(fc, fc + nc), key=lambda c: int(t.digit[c]))
        f, c = int(t.first[item]), int(t.count[item])
        return [-(int(i) + 1) for i in t.perm[f:f + c]]

    def neurons(self, item: int) -> np.ndarray:
        if item < 0:
            return np.array([-item - 1], np.int64)
        t = self.tree
        f, c = int(t.first[item]), int(t.count[item])
        return np.asarray(t.perm[f:f + c], np.int64)

    def att(self, S: int, C: int) -> float:
        si = self.neurons(S)
        si = si[self.a[si] > 0]
        cj = self.neurons(C)
        cj = cj[self.w[cj] > 0]
        if si.size == 0 or cj.size == 0:
            return 0.0
        where = np.full(self.pos.shape[0], -1, np.int64)
        where[cj] = np.arange(cj.size)
        u = gauss_sum(self.pos[si], self.pos[cj], self.w[cj], self.sigma, self_idx=where[si])
        return float(np.dot(self.a[si], u))

    def has_axons(self, item: int) -> bool:
        return bool(np.any(self.a[self.neurons(item)] > 0))

    # one step ----------------------------------------------------------------
    def step(self, frontier, step_no: int, seed: int):
        """Returns (next frontier, requests [(axon, dendrite)], decisions
        [(item, chosen index, margin)])."""
        nxt, req, dec = [], [], []

        def decide(item, values):
            r = uniform(seed, step_no, item)
            k = choose(values, r)
            dec.append((item, k, margin(values, r)))
            return k

        for S, T in frontier:
            sS, sT = S < 0, T < 0
            if sS and sT:
                req.append((-S - 1, -T - 1))
            elif sS:
                ch = self.children(T)
                k = decide(S, [self.att(S, C) for C in ch])
                if k >= 0:
                    nxt.append((S, ch[k]))
            elif sT:
                ch = self.children(S)
                k = decide(S, [self.att(c, T) for c in ch])
                if k >= 0:
                    nxt.append((ch[k], T))
            else:
                ch_t = self.children(T)
                for Sc in self.children(S):
                    if not self.has_axons(Sc):
                        continue
                    k = decide(Sc, [self.att(Sc, C) for C in ch_t])
                    if k >= 0:
                        nxt.append((Sc, ch_t[k]))
        return nxt, req, dec

    def run(self, seed: int, max_steps: int = 200):
        """Whole descent from (root, root): requests [(axon, dendrite)] sorted by axon."""
        frontier = [(0, 0)] if self.tree.n_nodes > 0 else []
        req = []
        for s in range(max_steps):
            if not frontier:
                break
            frontier, r, _ = self.step(frontier, s, seed)
            req += r
        return sorted(req)


def accept(requests, w, seed: int) -> np.ndarray:
    """Acceptance at the dendrites: bool per request."""
    w = np.asarray(w, np.float64)
    acc = np.zeros(len(requests), bool)
    by_j = {}
    for k, (i, j) in enumerate(requests):
        by_j.setdefault(int(j), []).append(k)
    for j, ks in by_j.items():
        ks.sort(key=lambda k: (priority(seed, int(requests[k][0])), int(requests[k][0])))
        for k in ks[:int(np.floor(w[j]))]:
            acc[k] = True
    return acc
