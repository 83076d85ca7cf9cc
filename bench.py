#!/usr/bin/env python3
"""Throughput of the Gaussian attraction sums on one MI355X.

A step is one pass of the whole hot path over the 4,194,304-neuron slab
(10 x 10 x 2 mm, sigma = 750 um, p = 8, leaf <= 64): octree build (root cube,
Morton keys, radix sort, node table), staging, the forward sum (expansion route
chosen by the cost model) and the scatter back to input order, plus child
probabilities (Algorithm 2) for 65,536 partner queries in the proportions of
its descent (one query per inner node visited).
fwd_bwd_ms times tree build + forward + backward (weights, positions, sigma).  value = targets evaluated per
second (attraction sums/s), inputs resident in HBM before the timed region.

Prints one JSON line.  Extra keys: per-phase times, the accuracy of this run
against the FP64 oracle on sampled targets, the all-pairs GPU direct sum on a
sample of targets (for the speedup), the oracle timed on host cores, the batch
of 256 populations and the partner descent.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"hbm": 8.0e12, "fp32_vector": 157.3e12, "fp32_mfma": 157.3e12, "fp64_vector": 78.6e12}
# work model of the partner kernels (per unit of counted work)
PAIR_FLOPS = 12.0        # walk pairs in float64: offsets, square, scale, exponential (as one), weight, sum
PAIR_FLOPS32 = 13.0      # direct-pass pairs in float32: 3 offsets, square (5), minus g0^2, scale,
                         # exponential (as one), weight multiply-add (2)
P2P_FLOPS32 = 11.0       # leaf P2P pairs in float32 (offsets scaled once per point): 3 offsets,
                         # square (5), exponential (as one), weight multiply-add (2)
PAIR_BYTES = 16.0        # the point record (x, y, z, staged w)
NODE_BYTES = 36.0        # level, cell coordinates, first point, count, children, moment flag
def m2p_flops(p):        # Hermite rows (3 p recurrence steps) and the p^3 contraction, 2 per multiply-add
    return 2.0 * p ** 3 + 2.0 * p * p + 2.0 * p + 9.0 * p


# phase -> kernel it times (one kernel per launch of the phase)
KERNEL_OF_PHASE = {"sort_scatter": "k_rs_scatter", "sort_hist": "k_rs_hist", "sort_runs": "k_seg_sort",
                   "p2m": "k_p2m_mfma8",
                   "l2p": "k_l2p", "m2l_x": "k_m2l_gemm", "m2l_y": "k_m2l_gemm",
                   "m2l_z": "k_m2l_gemm", "morton": "k_morton", "stage": "k_stage",
                   "partner": "k_partner", "partner_direct": "k_partner_direct",
                   "partner_wave": "k_partner_wave",
                   "scatter": "k_finish_u4"}   # (expansion route: flags and self term in input order)


def _algorithmic(phase, ctx):
    """(bound, unit, amount per launch) for a single-kernel phase, or None.

    Amounts count what the method must do: flops of the contraction it performs
    (2 per multiply-add) or bytes it must move at least once."""
    n, ns, nt, p = ctx["n"], ctx["n_src"], ctx["n_tgt"], ctx["p"]
    p3 = p ** 3
    if phase == "p2m":
        # p = 8: moments as a matrix-core product (k_p2m_mfma8)
        return ("mfma" if p == 8 else "alu"), "TFLOP/s", 2.0 * p3 * ns
    if phase == "l2p":
        return "alu", "TFLOP/s", 2.0 * p3 * nt
    if phase in ("m2l_x", "m2l_y", "m2l_z"):
        G = ctx["grid"]
        k = {"m2l_x": 0, "m2l_y": 1, "m2l_z": 2}[phase]
        U = G[k] * p
        R = G[0] * G[1] * G[2] * p3 // U
        return "mfma", "TFLOP/s", 2.0 * R * U * U
    if phase == "sort_scatter":
        # each pass reads and writes every (key, index) pair once
        return "hbm", "GB/s", n * 24.0
    if phase == "sort_runs":
        # (key, index) read and written once, positions gathered into key order
        return "hbm", "GB/s", n * (24.0 + 32.0)
    if phase in ("partner_direct", "partner_wave"):
        # the counted point pairs, each term in float32 (bound by the vector units)
        pairs = ctx["work"]["direct_pairs" if phase == "partner_direct" else "wave_pairs"]
        return "alu", "TFLOP/s", pairs * PAIR_FLOPS32
    if phase == "partner":
        # the walk: node records, moment blocks and point records it must read, and
        # its arithmetic; the bound is whichever needs more time at peak
        wk = ctx["work"]
        nbytes = wk["walk_nodes"] * NODE_BYTES + wk["walk_expansions"] * 4.0 * p3 + wk["walk_pairs"] * PAIR_BYTES
        t_alu = wk["walk_pairs"] * PAIR_FLOPS / PEAK["fp64_vector"] + wk["walk_expansions"] * m2p_flops(p) / PEAK["fp32_vector"]
        if nbytes / PEAK["hbm"] >= t_alu:
            return "hbm", "GB/s", nbytes
        # flops at the float64 rate that take the same time at peak
        return "alu64", "TFLOP/s", t_alu * PEAK["fp64_vector"]
    if phase == "sort_hist":
        return "hbm", "GB/s", n * 8.0
    if phase == "morton":
        return "hbm", "GB/s", n * (12 + 8 + 4 + 16.0)
    if phase == "stage":
        return "hbm", "GB/s", n * (4 + 1 + 4 + 16 + 1.0)
    if phase == "scatter":
        # target flag read, u read and written in input order
        return "hbm", "GB/s", n * (1 + 4 + 4.0)
    return None


def _partner_work(work, p, phases, steps):
    """The partner kernels' counted work per step, what it costs at each unit's
    peak, and the measured time: the 8-outputs-per-query figure beside the work
    the queries actually did."""
    def ms_of(ph):
        return phases[ph][0] / steps if ph in phases else None
    out = {"counts": work, "outputs_bytes": (work["direct_queries"] + work["wave_queries"] + work["walk_queries"]) * 36.0}
    for name, ph, pairs in (("eight_lane_pass", "partner_direct", work["direct_pairs"]),
                            ("wavefront_pass", "partner_wave", work["wave_pairs"])):
        out[name] = {"kernel": "k_partner_direct" if ph == "partner_direct" else "k_partner_wave",
                     "pairs": pairs, "flops32": pairs * PAIR_FLOPS32, "bytes": pairs * PAIR_BYTES,
                     "t_alu_ms": 1e3 * pairs * PAIR_FLOPS32 / PEAK["fp32_vector"],
                     "t_hbm_ms": 1e3 * pairs * PAIR_BYTES / PEAK["hbm"], "measured_ms": ms_of(ph)}
    nb = work["walk_nodes"] * NODE_BYTES + work["walk_expansions"] * 4.0 * p ** 3 + work["walk_pairs"] * PAIR_BYTES
    out["walk"] = {"kernel": "k_partner", "queries": work["walk_queries"], "nodes": work["walk_nodes"],
                   "expansions": work["walk_expansions"], "expansion_flops32": work["walk_expansions"] * m2p_flops(p),
                   "pairs": work["walk_pairs"], "pair_flops64": work["walk_pairs"] * PAIR_FLOPS, "bytes": nb,
                   "t_alu_ms": 1e3 * (work["walk_pairs"] * PAIR_FLOPS / PEAK["fp64_vector"]
                                      + work["walk_expansions"] * m2p_flops(p) / PEAK["fp32_vector"]),
                   "t_hbm_ms": 1e3 * nb / PEAK["hbm"],
                   "rounds_per_query": work["walk_rounds"] / max(work["walk_queries"], 1),
                   "measured_ms": ms_of("partner"),
                   "bound_by": "latency: each stack round waits on dependent loads of node records and "
                               "moment blocks, and the launch lasts as long as its longest query (the root's)"}
    return out


def _peak_of(bound):
    return {"mfma": PEAK["fp32_mfma"], "alu": PEAK["fp32_vector"], "alu64": PEAK["fp64_vector"]}[bound]


def _traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or None
    when there is none or the kernel's source has changed since it was taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_slab4M.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_src = re.search(r"source_sha256:\s*(\S+)\s+(\S+)", text)
    m_val = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not (m_src and m_val):
        return None
    src = os.path.join(ROOT, m_src.group(1))
    if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != m_src.group(2):
        return None
    return float(m_val.group(1))


def _partner_queries(tree, k, seed):
    """k (target, node) queries in the proportions of the descent of Algorithm 2,
    which asks one query per (axon box, dendrite node) pair on every level: the
    node is drawn uniformly from the inner nodes (so levels appear in proportion
    to their node counts) and the target uniformly from the node's points."""
    import numpy as np
    import torch
    ex = {kk: v.cpu().numpy() for kk, v in tree.export().items()}
    if k <= 0 or tree.n == 0:
        e = torch.zeros(0, dtype=torch.int32, device="cuda")
        return e, e
    rng = np.random.default_rng(seed)
    inner = np.nonzero(ex["node_n_children"] > 0)[0]
    node = inner[rng.integers(0, inner.size, k)]
    first, count = ex["node_first"][node], ex["node_count"][node]
    pos = first + (rng.random(k) * count).astype(np.int64)
    tq = ex["perm"][pos]
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()
    return T(tq), T(node)


def _descent_bench(args, dev):
    """The partner descent (Algorithm 1 with Algorithm 2's proportional choice, then
    the acceptance at the dendrites) over the 262,144 neurons in 64 Gaussian blobs
    (sigma 200 um, p 8): whole descents from (root, root) timed with the device
    synchronised, plus validity checks of the result."""
    import numpy as np
    import torch
    import paper_2301_10570_amd as msp
    import synth
    wl = synth.blobs262k()
    T = lambda v: torch.from_numpy(np.ascontiguousarray(v)).to(dev)
    tree = msp.Tree()
    tree.build(T(wl.x), T(wl.y), T(wl.z), leaf_max=wl.leaf_max)
    w, a = T(wl.w), T(wl.a)
    reps = 3

    def timed(cutoff):
        r = tree.partner_descent(w, a, wl.sigma, 11, p=wl.p, cutoff_sigmas=cutoff)   # first call: allocations
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for rep in range(reps):
            r = tree.partner_descent(w, a, wl.sigma, 11 + rep, p=wl.p, cutoff_sigmas=cutoff)
        torch.cuda.synchronize()
        return r, 1000.0 * (time.perf_counter() - t0) / reps

    r0, ms_nocut = timed(0.0)
    r, ms = timed(4.5)
    ax = r["axon"].cpu().numpy()
    dd = r["dendrite"].cpu().numpy()
    acc = r["accepted"].cpu().numpy().astype(bool)
    ok = bool(np.unique(ax).size == ax.size and np.all(wl.a[ax] > 0) and np.all(wl.w[dd] > 0)
              and np.all(ax != dd) and np.all(np.bincount(dd[acc], minlength=wl.n) <= np.floor(wl.w)))
    tree.close()
    return {"workload": "262,144 neurons in 64 Gaussian blobs (4 mm cube, std 50 um), sigma 200 um, p 8, "
                        "leaf <= 64, cutoff 4.5 sigma",
            "axon_neurons": int(np.count_nonzero(wl.a > 0)), "requests": int(ax.size),
            "accepted": int(acc.sum()), "steps": int(r["steps"]), "ms_per_descent": ms,
            "requests_per_s": ax.size / (ms / 1000.0), "valid": ok,
            "no_cutoff": {"ms_per_descent": ms_nocut, "requests": int(r0["axon"].numel())}}


def _timed(fn, steps):
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return 1000.0 * (time.perf_counter() - t0) / steps


def _other_configs(args, dev, threads):
    """The transform against the all-pairs GPU direct sum on the 4,096-neuron cube
    (sigma 100 um) and on the 262,144 neurons in 64 blobs (sigma 200 um), each with
    its accuracy against the FP64 oracle; and forward + backward on the gradient
    workload (1,048,576 sources + 1,048,576 targets in a 2 mm cube, sigma 200 um)."""
    import numpy as np
    import torch

    import paper_2301_10570_amd as msp
    import synth
    out = {}
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    for name, wl, nchk in (("uniform4k", synth.uniform4k(), None), ("blobs262k", synth.blobs262k(), 4096)):
        x, y, z, w, tg = T(wl.x), T(wl.y), T(wl.z), T(wl.w), T((wl.a > 0).astype(np.uint8))
        ti = np.nonzero(wl.a > 0)[0]
        si = np.nonzero(wl.w > 0)[0]
        tree = msp.Tree().build(x, y, z, leaf_max=wl.leaf_max)
        u = torch.empty(wl.n, dtype=torch.float32, device=dev)
        reps = max(args.steps, 100)   # small launches: enough repetitions for a steady clock
        ms_c = _timed(lambda: tree.forward(w, tg, sigma=wl.sigma, p=wl.p, out=u), reps)
        ms_b = _timed(lambda: (tree.build(x, y, z, leaf_max=wl.leaf_max),
                               tree.forward(w, tg, sigma=wl.sigma, p=wl.p, out=u)), reps)
        plan = tree.plan(wl.sigma, p=wl.p)
        dtx, dty, dtz = T(wl.x[ti]), T(wl.y[ti]), T(wl.z[ti])
        dsx, dsy, dsz, dsw = T(wl.x[si]), T(wl.y[si]), T(wl.z[si]), T(wl.w[si])
        ud = torch.empty(ti.size, dtype=torch.float32, device=dev)
        ms_d = _timed(lambda: msp.direct_sum(dtx, dty, dtz, dsx, dsy, dsz, dsw, wl.sigma, out=ud), reps)
        row = {"n": wl.n, "targets": int(ti.size), "sources": int(si.size), "route": plan["route"],
               "level": plan["level"], "fmm_ms_cached_tree": ms_c, "fmm_ms_incl_tree": ms_b,
               "fmm_sums_per_s_cached_tree": ti.size / (ms_c / 1000.0),
               "fmm_sums_per_s_incl_tree": ti.size / (ms_b / 1000.0),
               "direct_gpu_ms": ms_d, "direct_gpu_sums_per_s": ti.size / (ms_d / 1000.0),
               "speedup_cached_tree": ms_d / ms_c, "speedup_incl_tree": ms_d / ms_b}
        if not args.no_check:
            import oracle
            chk = np.arange(ti.size) if nchk is None else synth.sample_indices(ti.size, nchk, seed=786)
            ref = oracle.attraction(wl, ti[chk], threads=threads)
            e_f = np.abs(u.cpu().numpy()[ti[chk]].astype(np.float64) - ref) / ref
            e_d = np.abs(ud.cpu().numpy()[chk].astype(np.float64) - ref) / ref
            row.update({"targets_checked": int(chk.size), "fmm_max_rel_err": float(e_f.max()),
                        "direct_max_rel_err": float(e_d.max()), "pass": bool(max(e_f.max(), e_d.max()) <= 1e-4)})
        out[name] = row
        tree.close()
    wl = synth.sources_targets_1m()
    x, y, z, w, tg = T(wl.x), T(wl.y), T(wl.z), T(wl.w), T((wl.a > 0).astype(np.uint8))
    g = T(wl.extra["g"])
    tree = msp.Tree()
    u = torch.empty(wl.n, dtype=torch.float32, device=dev)
    res = {}

    def fb():
        tree.build(x, y, z, leaf_max=wl.leaf_max)
        tree.forward(w, tg, sigma=wl.sigma, p=wl.p, out=u)
        res.update(tree.backward(w, g, tg, sigma=wl.sigma, p=wl.p))
    ms_fb = _timed(fb, args.steps)
    row = {"n": wl.n, "targets": int((wl.a > 0).sum()), "sources": int((wl.w > 0).sum()),
           "route": tree.plan(wl.sigma, p=wl.p)["route"], "fwd_bwd_ms_incl_tree": ms_fb,
           "gradients": "weights, positions, sigma"}
    if not args.no_check:
        import oracle
        ti = np.nonzero(wl.a > 0)[0]
        si = np.nonzero(wl.w > 0)[0]
        chk = ti[synth.sample_indices(ti.size, 4096, seed=787)]
        ref = oracle.attraction(wl, chk, threads=threads)
        e_f = np.abs(u.cpu().numpy()[chk].astype(np.float64) - ref) / ref
        sw = si[synth.sample_indices(si.size, 256, seed=788)]
        pos = wl.pos64()
        gh = wl.extra["g"].astype(np.float64)
        rw = oracle.gauss_grad(pos[ti], gh[ti], pos[sw], wl.w[sw], wl.sigma, want=("w",), threads=threads)["w"]
        e_w = np.abs(res["w"].cpu().numpy()[sw].astype(np.float64) - rw) / rw
        row.update({"forward_targets_checked": int(chk.size), "forward_max_rel_err": float(e_f.max()),
                    "grad_w_points_checked": int(sw.size), "grad_w_max_rel_err": float(e_w.max()),
                    "pass": bool(max(e_f.max(), e_w.max()) <= 1e-4)})
    out["sources_targets_1m"] = row
    tree.close()
    return out


def _batch_bench(args, dev, oracle_threads):
    """256 independent populations (sizes log-uniform in [1024, 65536], sigma
    log-uniform in [50, 300] um, each in its own 1 mm cube): autotuned leaf size
    and route per population, the forward as one captured hipGraph (all
    direct-route populations in one persistent launch), per-population latency
    from device timestamps, forward + backward, and accuracy on sampled targets."""
    import numpy as np
    import torch

    import paper_2301_10570_amd as msp
    import synth
    pops = synth.populations()
    T = lambda a: torch.from_numpy(np.ascontiguousarray(np.concatenate(a))).to(dev)
    x, y, z, w = (T([getattr(p, k) for p in pops]) for k in ("x", "y", "z", "w"))
    tg = T([(p.a > 0).astype(np.uint8) for p in pops])
    off = np.concatenate([[0], np.cumsum([p.n for p in pops])]).astype(np.int64)
    sig = np.array([p.sigma for p in pops], dtype=np.float32)
    n_tgt = int(sum(int((p.a > 0).sum()) for p in pops))
    b = msp.Batch()
    t0 = time.perf_counter()
    leaf, routes = b.autotune(x, y, z, off, w, sig, is_target=tg, p=args.p, candidates=(32, 64, 128))
    tune_s = time.perf_counter() - t0
    u = torch.empty(int(off[-1]), dtype=torch.float32, device=dev)
    b.forward(w, sig, is_target=tg, p=args.p, out=u)        # eager, then captured
    launches = b.info()["launches_last_eager_forward"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.forward(w, sig, is_target=tg, p=args.p, out=u)    # graph replay
    torch.cuda.synchronize()
    ms_graph = 1000.0 * (time.perf_counter() - t0) / args.steps
    inst = b.instance_ms()
    pairs, span = b.pair_count()   # the direct-route populations of the last replay
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.forward(w, sig, is_target=tg, p=args.p, out=u, use_graph=False)
    torch.cuda.synchronize()
    ms_eager = 1000.0 * (time.perf_counter() - t0) / args.steps
    gone = torch.ones(int(off[-1]), dtype=torch.float32, device=dev)
    grads = b.backward(w, gone, sig, is_target=tg, p=args.p, use_graph=True)   # eager + capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.forward(w, sig, is_target=tg, p=args.p, out=u)
        grads = b.backward(w, gone, sig, is_target=tg, p=args.p, out=grads, use_graph=True)
    torch.cuda.synchronize()
    ms_fb = 1000.0 * (time.perf_counter() - t0) / args.steps
    # the same forward and forward + backward with the translation as split bfloat16
    # products (graph replays)
    u16 = torch.empty_like(u)
    b.forward(w, sig, is_target=tg, p=args.p, out=u16, m2l="bf16x3")
    ms_graph16 = _timed(lambda: b.forward(w, sig, is_target=tg, p=args.p, out=u16, m2l="bf16x3"), args.steps)
    g16 = b.backward(w, gone, sig, is_target=tg, p=args.p, use_graph=True, m2l="bf16x3")
    ms_fb16 = _timed(lambda: (b.forward(w, sig, is_target=tg, p=args.p, out=u16, m2l="bf16x3"),
                              b.backward(w, gone, sig, is_target=tg, p=args.p, out=g16, use_graph=True,
                                         m2l="bf16x3")), args.steps)
    res = {"workload": "256 populations, n log-uniform 1024-65536, sigma log-uniform 50-300 um, 1 mm cubes",
           "points": int(off[-1]), "targets": n_tgt, "autotune_s": tune_s,
           "routes": {"fgt": routes.count("fgt"), "direct": routes.count("direct")},
           "leaf_sizes": {str(k): int((leaf == k).sum()) for k in (32, 64, 128)},
           "forward_ms_graph": ms_graph, "forward_ms_eager": ms_eager,
           "sums_per_s": n_tgt / (ms_graph / 1000.0), "launches_per_forward_eager": launches,
           "instance_ms_p50": float(np.percentile(inst, 50)), "instance_ms_p99": float(np.percentile(inst, 99)),
           "fwd_bwd_ms": ms_fb,
           "m2l_bf16x3": {"forward_ms_graph": ms_graph16, "fwd_bwd_ms": ms_fb16},
           # k_batch_p2p: the point pairs of the direct-route populations over the span from
           # the launch's first to its last work item (beside the expansion-route branch)
           "direct_route": {"pairs": pairs, "span_ms": span,
                            "pairs_per_s": pairs / (span / 1000.0) if span > 0 else None,
                            "bound": "alu", "peak_tflops": PEAK["fp32_vector"] / 1e12,
                            "achieved_tflops": pairs * P2P_FLOPS32 / (span / 1000.0) / 1e12 if span > 0 else None,
                            "frac": pairs * P2P_FLOPS32 / (span / 1000.0) / PEAK["fp32_vector"] if span > 0
                            else None}}
    if not args.no_check:
        import oracle
        u_h = u.cpu().numpy()
        errs = []
        for k in synth.sample_indices(len(pops), 32, seed=783):
            wl = pops[k]
            tgt = np.nonzero(wl.a > 0)[0]
            sel = tgt[synth.sample_indices(tgt.size, 8, seed=784 + int(k))]
            ref = oracle.attraction(wl, sel, threads=oracle_threads)
            errs.append(np.abs(u_h[off[k]:off[k + 1]][sel].astype(np.float64) - ref) / ref)
        e = np.concatenate(errs)
        res["accuracy"] = {"targets_checked": int(e.size), "max_rel_err": float(e.max()), "bar": 1e-4,
                           "pass": bool(e.max() <= 1e-4)}
        u16_h = u16.cpu().numpy()
        e16 = []
        for k in synth.sample_indices(len(pops), 32, seed=783):
            wl = pops[k]
            tgt = np.nonzero(wl.a > 0)[0]
            sel = tgt[synth.sample_indices(tgt.size, 8, seed=784 + int(k))]
            ref = oracle.attraction(wl, sel, threads=oracle_threads)
            e16.append(np.abs(u16_h[off[k]:off[k + 1]][sel].astype(np.float64) - ref) / ref)
        e16 = np.concatenate(e16)
        res["m2l_bf16x3"]["max_rel_err"] = float(e16.max())
    b.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--p", type=int, default=8)
    ap.add_argument("--route", default="auto")
    ap.add_argument("--scale", type=float, default=1.0, help="shrink the neuron count (testing only)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-direct", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="budget for the oracle sample, from a short probe (which overestimates)")
    ap.add_argument("--queries", type=int, default=65536, help="partner queries per step")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-population batch")
    ap.add_argument("--no-descent", action="store_true", help="skip the partner descent")
    ap.add_argument("--no-configs", action="store_true", help="skip the cube, blob and gradient workloads")
    ap.add_argument("--serial", action="store_true",
                    help="forward and partner probabilities on one stream, one after the other")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with three copies of 1 GiB (counter calibration runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); the octree "
              "transform shards by space with a halo exchange, which is not built here.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2301_10570_amd as msp
    import synth

    print("bench: generating the 4,194,304-neuron slab", file=sys.stderr, flush=True)
    wl = synth.slab4m(args.scale)
    wl.p = args.p
    dev = torch.device("cuda", 0)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    x, y, z, w = T(wl.x), T(wl.y), T(wl.z), T(wl.w)
    tgt = T((wl.a > 0).astype(np.uint8))
    n_tgt = int((wl.a > 0).sum())
    n_src = int((wl.w > 0).sum())
    u = torch.empty(wl.n, dtype=torch.float32, device=dev)
    tree = msp.Tree()
    tree.build(x, y, z, leaf_max=wl.leaf_max)
    tq, nq = _partner_queries(tree, args.queries, seed=781)
    uni = T(synth.uniforms(tq.numel(), 782))

    # the forward and the partner probabilities both read the tree and the weights
    # the weighted build put into key order, and write nothing the other reads: the
    # partner call runs on a second stream beside the forward (--serial: one stream)
    side = torch.cuda.Stream()

    probs = torch.empty(tq.numel() * 8, dtype=torch.float32, device=dev)
    choice = torch.empty(tq.numel(), dtype=torch.int32, device=dev)

    def step(serial=args.serial):
        # the vacant element counts ride into key order with the positions
        tree.build(x, y, z, leaf_max=wl.leaf_max, w=w)
        main = torch.cuda.current_stream()
        two = tq.numel() > 0 and not serial
        if two:
            side.wait_stream(main)   # the partner call follows the build, not the forward
        # the forward first: its few launches reach the GPU while the host issues
        # the partner call's
        tree.forward(w, tgt, sigma=wl.sigma, p=wl.p, route=args.route, out=u, weights_staged=True)
        if tq.numel():
            with torch.cuda.stream(side if two else main):
                tree.partner_probabilities(w, tq, nq, wl.sigma, p=wl.p, uniforms=uni, weights_staged=True,
                                           out=(probs, choice))
        if two:
            main.wait_stream(side)   # the next build rewrites what the partner call reads

    print("bench: warmup", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan = tree.plan(wl.sigma, p=wl.p, route=args.route)

    # timed region
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1000.0 * elapsed / args.steps
    value = n_tgt / (ms_per_step / 1000.0)
    print(f"bench: {ms_per_step:.3f} ms/step, {value:.3e} sums/s", file=sys.stderr, flush=True)

    # the same steps again with HIP events around every library phase and sort
    # pass, recorded live on the streams that run them: once as timed (phases that
    # overlap share the GPU), once with every pass alone (one stream, the
    # library's side-stream passes one after another), which the kernel
    # rooflines use
    def event_pass(isolated):
        tree.set_timing(True, isolated=isolated)
        tree.timing(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(serial=args.serial or isolated)
        torch.cuda.synchronize()
        ms = 1000.0 * (time.perf_counter() - t0) / args.steps
        ph = tree.timing(reset=True)
        tree.set_timing(False)
        return ph, ms
    phases_timed, ms_events = event_pass(False)
    phases, ms_alone = event_pass(True)

    # forward only, cached tree
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        tree.forward(w, tgt, sigma=wl.sigma, p=wl.p, route=args.route, out=u)
    torch.cuda.synchronize()
    ms_fwd = 1000.0 * (time.perf_counter() - t0) / args.steps

    # forward only with the translation (M2L) as split-bfloat16 matrix-core
    # products, against the float32 matrix-core passes
    ub = torch.empty_like(u)
    tree.forward(w, tgt, sigma=wl.sigma, p=wl.p, route=args.route, out=ub, m2l="bf16x3")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        tree.forward(w, tgt, sigma=wl.sigma, p=wl.p, route=args.route, out=ub, m2l="bf16x3")
    torch.cuda.synchronize()
    ms_fwd_b = 1000.0 * (time.perf_counter() - t0) / args.steps
    m2l_ms = {}
    for mode in ("mfma", "bf16x3"):
        tree.set_timing(True)
        tree.timing(reset=True)
        for _ in range(args.steps):
            tree.forward(w, tgt, sigma=wl.sigma, p=wl.p, route=args.route, out=ub, m2l=mode)
        ph = tree.timing(reset=True)
        tree.set_timing(False)
        m2l_ms[mode] = sum(ph[k][0] for k in ("m2l_x", "m2l_y", "m2l_z") if k in ph) / args.steps

    # forward + backward (L = sum u_i over targets, g = 1): gradients w.r.t. the
    # weights, the positions and sigma; the tree is rebuilt every step
    gone = torch.ones(wl.n, dtype=torch.float32, device=dev)
    def fwd_bwd():
        tree.build(x, y, z, leaf_max=wl.leaf_max)
        tree.forward(w, tgt, sigma=wl.sigma, p=wl.p, route=args.route, out=u)
        tree.backward(w, gone, tgt, sigma=wl.sigma, p=wl.p, route=args.route)
    fwd_bwd()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fwd_bwd()
    torch.cuda.synchronize()
    ms_fb = 1000.0 * (time.perf_counter() - t0) / args.steps

    # the partner kernels' work, counted on one more (untimed) step
    tree.set_work_counting(True)
    step()
    work = tree.work_counts()
    tree.set_work_counting(False)
    ctx = {"n": wl.n, "n_src": n_src, "n_tgt": n_tgt, "p": wl.p, "grid": plan["grid"],
           "queries": int(tq.numel()), "work": work}
    per_phase = {k: {"ms_per_step": v[0] / args.steps, "launches_per_step": v[1] / args.steps}
                 for k, v in phases_timed.items()}
    per_phase_alone = {k: {"ms_per_step": v[0] / args.steps, "launches_per_step": v[1] / args.steps}
                       for k, v in phases.items()}
    # dominant kernel: the single-kernel phase with the most time per step
    def _roof(ph):
        info = _algorithmic(ph, ctx)
        if info is None:
            return None
        bound, unit, amount = info
        avg_s = phases[ph][0] / phases[ph][1] / 1000.0
        if unit == "GB/s":
            achieved, peak = amount / avg_s / 1e9, PEAK["hbm"] / 1e9
        else:
            achieved = amount / avg_s / 1e12
            peak = _peak_of(bound) / 1e12
        out_bound = "alu" if bound == "alu64" else bound
        return {"bound": out_bound, "achieved": achieved, "peak": peak, "unit": unit,
                "frac": achieved / peak, "traffic": _traffic(KERNEL_OF_PHASE[ph]),
                "kernel": KERNEL_OF_PHASE[ph], "phase": ph, "algorithmic_per_launch": amount,
                "avg_launch_ms": phases[ph][0] / phases[ph][1],
                "ms_per_step": phases[ph][0] / args.steps}

    # dominant kernel: the single-kernel phase with the most time per step
    cands = [k for k in KERNEL_OF_PHASE if k in phases and phases[k][1] > 0]
    dom = max(cands, key=lambda k: phases[k][0]) if cands else None
    roof = _roof(dom) if dom else None
    kernels = {k: _roof(k) for k in sorted(cands, key=lambda k: -phases[k][0])}
    # the step as a whole: T_ideal = sum over the phases with a work model of
    # (launches x algorithmic amount / peak), against the measured step time
    t_ideal, modelled, unmodelled_ms = 0.0, [], 0.0
    for ph, (tot_ms, launches) in phases.items():
        info = _algorithmic(ph, ctx) if launches > 0 else None
        if info is None:
            unmodelled_ms += tot_ms / args.steps
            continue
        bound, unit, amount = info
        pk = PEAK["hbm"] if unit == "GB/s" else _peak_of(bound)
        t_ideal += (launches / args.steps) * amount / pk
        modelled.append(ph)
    step_roof = {"t_ideal_ms": 1000.0 * t_ideal, "t_measured_ms": ms_per_step,
                 "frac": 1000.0 * t_ideal / ms_per_step, "phases_modelled": sorted(modelled),
                 "unmodelled_phase_ms": unmodelled_ms}
    if args.copy_calibration:
        # a plain device copy of known size, for scaling the HBM counters
        a = torch.empty(256 << 20, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"bench: copy calibration 3 x {a.numel() * 4} bytes", file=sys.stderr, flush=True)

    result = {
        "metric": "attraction sums/s at rel-err<=1e-4 (FMM forward incl. octree build)",
        "value": value, "unit": "sums/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "slab 4,194,304 neurons 10x10x2 mm, sigma 750 um, counts 0-5",
                   "n": wl.n, "targets": n_tgt, "sources": n_src, "p": wl.p, "leaf_max": wl.leaf_max,
                   "route": plan["route"], "level": plan["level"], "grid": plan["grid"],
                   "rho": plan["rho"]},
        "roofline": roof,
        "kernel_rooflines": kernels,
        "step_roofline": step_roof,
        "schedule": ("one stream" if args.serial else
                     "forward on the caller's stream, partner probabilities on a second stream"),
        "phases": per_phase,
        "ms_per_step_with_events": ms_events,
        "phases_alone": per_phase_alone,
        "ms_per_step_alone": ms_alone,
        "forward_only_ms": ms_fwd,
        "forward_only_sums_per_s": n_tgt / (ms_fwd / 1000.0),
        "fwd_bwd_ms": ms_fb,
        "partner_queries_per_step": int(tq.numel()),
        "partner_work": _partner_work(work, wl.p, phases, args.steps),
        "m2l_bf16x3": {"forward_only_ms": ms_fwd_b, "m2l_ms": m2l_ms["bf16x3"],
                       "m2l_fp32_mfma_ms": m2l_ms["mfma"]},
    }

    # p sweep of the transform (tree cached), fp32 and split-bf16 translation
    sweep = {}
    for p in (4, 6, 8, 10):
        for mode in ("mfma", "bf16x3"):
            us = torch.empty_like(u)
            tree.forward(w, tgt, sigma=wl.sigma, p=p, route="fgt", out=us, m2l=mode)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                tree.forward(w, tgt, sigma=wl.sigma, p=p, route="fgt", out=us, m2l=mode)
            torch.cuda.synchronize()
            ms_p = 1000.0 * (time.perf_counter() - t0) / args.steps
            pl_p = tree.plan(wl.sigma, p=p, route="fgt")
            sweep[f"p{p}_{mode}"] = {"p": p, "m2l": mode, "level": pl_p["level"], "grid": pl_p["grid"],
                                     "forward_only_ms": ms_p, "sums_per_s": n_tgt / (ms_p / 1000.0),
                                     "_u": us.cpu().numpy()}
    result["p_sweep"] = sweep

    threads = min(16, len(os.sched_getaffinity(0)))
    if not args.no_check or not args.no_cpu:
        import oracle
        ti = np.nonzero(wl.a > 0)[0]
        # accuracy sample: 65,536 seeded targets, every target within one p = 8 cell of
        # a corner of the slab, and 8,192 targets within that reach of an x or y face
        groups = {"uniform": ti[synth.sample_indices(ti.size, min(65536, ti.size), seed=303)]}
        reach = float(max(np.ptp(wl.x), np.ptp(wl.y), np.ptp(wl.z))) / 16.0
        groups.update(synth.boundary_sample(wl, ti, reach, 8192, seed=304))
        sel = np.unique(np.concatenate(list(groups.values())))
        order = sel[np.random.default_rng(785).permutation(sel.size)]
        ref_of = {}
        if not args.no_cpu:
            # the oracle as it stands, timed on a seeded part of the accuracy sample with
            # every host thread, then on one thread
            oracle.attraction(wl, order[:threads], threads=threads)   # threads started, pages touched
            probe = order[:8 * threads]
            t0 = time.perf_counter()
            oracle.attraction(wl, probe, threads=threads)
            per = (time.perf_counter() - t0) / probe.size
            k = int(max(8 * threads, min(sel.size, args.cpu_seconds / max(per, 1e-9))))
            chunk = order[:k]
            print(f"bench: oracle on {k} targets x {n_src} sources, {threads} threads", file=sys.stderr, flush=True)
            t0 = time.perf_counter()
            r = oracle.attraction(wl, chunk, threads=threads)
            dt = time.perf_counter() - t0
            ref_of.update(zip(chunk.tolist(), r.tolist()))
            k1 = int(max(4, min(k, 0.25 * args.cpu_seconds / max(per * threads, 1e-9))))
            print(f"bench: oracle on {k1} targets, 1 thread", file=sys.stderr, flush=True)
            t1 = time.perf_counter()
            oracle.attraction(wl, order[:k1], threads=1)
            dt1 = time.perf_counter() - t1
            model = ""
            try:
                for line in open("/proc/cpuinfo"):
                    if line.startswith("model name"):
                        model = line.split(":", 1)[1].strip()
                        break
            except OSError:
                pass
            result["cpu_baseline"] = {
                "value": k / dt, "unit": "sums/s", "cores": threads, "kind": "oracle",
                "sample": f"{k} seeded targets of the slab (from the accuracy sample), each summed over "
                          f"all {n_src} sources in FP64 ({dt:.1f} s on {threads} threads)",
                "host_cpus": len(os.sched_getaffinity(0)), "cpu_model": model,
                "single_thread": {"value": k1 / dt1, "unit": "sums/s", "cores": 1,
                                  "sample": f"the first {k1} targets of that sample ({dt1:.1f} s)"}}
        if not args.no_check:
            rest = np.array([i for i in order.tolist() if i not in ref_of], dtype=np.int64)
            print(f"bench: oracle reference at {rest.size} more targets", file=sys.stderr, flush=True)
            if rest.size:
                ref_of.update(zip(rest.tolist(), oracle.attraction(wl, rest, threads=threads).tolist()))
            ref = np.array([ref_of[i] for i in sel.tolist()])
            where = {g: np.searchsorted(sel, idx) for g, idx in groups.items()}

            def acc(uu):
                rel = np.abs(uu[sel].astype(np.float64) - ref) / ref
                out = {"targets_checked": int(sel.size), "max_rel_err": float(rel.max()),
                       "p99_rel_err": float(np.quantile(rel, 0.99)), "p50_rel_err": float(np.median(rel)),
                       "bar": 1e-4, "pass": bool(rel.max() <= 1e-4)}
                for g, ix in where.items():
                    out[g] = {"targets": int(ix.size), "max_rel_err": float(rel[ix].max()),
                              "p99_rel_err": float(np.quantile(rel[ix], 0.99))}
                return out
            tree.forward(w, tgt, sigma=wl.sigma, p=wl.p, route=args.route, out=u)
            result["accuracy"] = acc(u.cpu().numpy())
            result["accuracy"]["sample"] = ("65,536 seeded targets, every target within 625 um of a corner of "
                                            "the slab, 8,192 seeded targets within 625 um of an x or y face")
            tree.forward(w, tgt, sigma=wl.sigma, p=wl.p, route=args.route, out=ub, m2l="bf16x3")
            result["m2l_bf16x3"]["accuracy"] = acc(ub.cpu().numpy())
            for key, row in sweep.items():
                a = acc(row["_u"])
                row["max_rel_err"], row["p99_rel_err"], row["pass"] = a["max_rel_err"], a["p99_rel_err"], a["pass"]
    for row in sweep.values():
        row.pop("_u", None)

    if not args.no_direct:
        print("bench: all-pairs GPU direct sum on sampled targets", file=sys.stderr, flush=True)
        ti = np.nonzero(wl.a > 0)[0]
        si = np.nonzero(wl.w > 0)[0]
        k = min(ti.size, 131072)
        ts = ti[synth.sample_indices(ti.size, k, seed=778)]
        dtx, dty, dtz = T(wl.x[ts]), T(wl.y[ts]), T(wl.z[ts])
        dsx, dsy, dsz, dsw = T(wl.x[si]), T(wl.y[si]), T(wl.z[si]), T(wl.w[si])
        ud = msp.direct_sum(dtx, dty, dtz, dsx, dsy, dsz, dsw, wl.sigma)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        msp.direct_sum(dtx, dty, dtz, dsx, dsy, dsz, dsw, wl.sigma, out=ud)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        dsum = k / dt
        result["direct_gpu"] = {"sums_per_s": dsum, "targets_timed": k, "sources": int(si.size),
                                "pairs_per_s": k * si.size / dt,
                                "speedup_fmm_incl_tree": value / dsum,
                                "speedup_fmm_cached_tree": result["forward_only_sums_per_s"] / dsum}

    tree.close()
    if not args.no_configs:
        print("bench: the other workloads (cube 4k, blobs 262k, gradients 1M + 1M)", file=sys.stderr, flush=True)
        result["other_workloads"] = _other_configs(args, dev, threads)
    if not args.no_batch:
        print("bench: 256-population batch", file=sys.stderr, flush=True)
        result["batch"] = _batch_bench(args, dev, min(16, len(os.sched_getaffinity(0))))
    if not args.no_descent:
        print("bench: partner descent", file=sys.stderr, flush=True)
        result["descent"] = _descent_bench(args, dev)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
