// The partner descent of Algorithm 1, driven by the proportional choice of
// Algorithm 2, as a level-synchronous frontier of (axon item, dendrite item)
// pairs, and the acceptance of the resulting requests at the dendrites.
//
// Items: an octree node v (v >= 0) or one neuron with input index i (-(i + 1)).
// A neuron is the paper's leaf.  The children of an inner node are its child
// nodes in octant order; the children of a leaf node of the octree are its
// neurons in key order.  The attraction of the axons of S to the dendrites of C,
//     Att(S, C) = sum_{i in S} sum_{j in C, j != i} a_i w_j exp(-|t_i - s_j|^2 / sigma^2),
// decides every choice (Eq. (8) weighted by vacant axonal and dendritic elements).
// One step, per pair (S, T):
//   S, T neurons             request S -> T
//   S neuron, T node         choose a child C of T by Att(S, C)
//   S node, T neuron         choose a child S' of S by Att(S', T); the other children drop out
//   S, T nodes               every child S_c of S holding axons chooses a child C of T by Att(S_c, C)
// A choice draws r from SplitMix64 keyed by (seed, step, choosing item) and takes
// the first candidate whose running sum exceeds r times the total; all-zero
// values drop the pair.
//
// Evaluation.  While S and T both lie above the box level (below), Att(S_c, C)
// for the children C of T is the sum of box-pair attractions over the boxes of
// S_c and of C: Algorithm 2's expansion case for many axons against many
// dendrites, taken once per descent for every pair of boxes within the cutoff.
// Below it, Att(S_c, C) is the sum over the axon neurons i of S_c of a_i times
// the per-octant attraction of i to T's children, which the partner queries
// compute (node moments where accurate, direct sums otherwise: the accuracy
// contract of the partner probabilities).  For a leaf node T (children =
// neurons) and for a single dendrite neuron T the terms are summed directly in
// FP64.
//
// Frontier.  The frontier lives in device memory and every step runs in kernels:
// per pair, the number of units (one per choice) and requests it makes; their
// offsets by prefix sums; per unit, its queries or direct tasks and their offsets
// by prefix sums; the lists; the partner queries and direct terms; the choices;
// and the next frontier, one entry per unit (kNoItem where the choice dropped the
// pair).  The kernels read the step's sizes from device counters and the tables
// are sized once per descent: the axon items of a frontier are disjoint and each
// holds an axon, so the units, queries and tasks of a step never outnumber the
// neurons with axons.  The host only launches; it stays at most two steps ahead
// of the device and stops once a step has emptied the frontier.
//
// Boxes.  The box level is one below the coarsest level whose half side is
// within rho_max(p) sigma, so that a box there has half side at most
// rho_max(p) sigma / 2.  The boxes are the nodes at or below the box level whose
// parent lies above it, and the leaves above it; they partition the points, and
// the boxes inside a node above the box level are one run of the boxes in key
// order.  For an axon box s (a_i > 0 somewhere) and a dendrite box c (w_j > 0
// somewhere) within the cutoff (box gap <= cutoff_sigmas sigma; every pair
// without a cutoff)
//     Att(s, c) = sum_{i in s} sum_{j in c, j != i} a_i w_j exp(-|t_i - s_j|^2 / sigma^2)
// is summed directly (float32 terms relative to the closest approach of the two
// boxes, each to about 1e-5; float64 sums), or, when both boxes lie at or below
// the box level,
// s holds more than c2 axons and c more than c1 dendrites (Algorithm 2's
// thresholds, 70 each) and their centres are within kBoxAdmitR sigma, taken from
// expansions: with u, v the offsets of s_j, t_i from the centres of c and s in
// units of sigma and d = (centre of s - centre of c) / sigma,
//     Att(s, c) = sum_{alpha, beta} A_alpha Mt_beta h(alpha + beta, d),
//     A_alpha  = sum_j w_j u_j^alpha / alpha!           (Eq. (7), the dendrite box)
//     Mt_beta  = sum_i a_i (-v_i)^beta / beta!          (the axon box)
// i.e. the dendrite box's Hermite series translated to a Taylor series at the
// axon box (the coefficients B_beta of Eq. (6), whose sign factor belongs with
// h's argument taken as target centre minus source) and contracted with the axon box's power sums; a box paired with
// itself has its self terms a_i w_i subtracted.  The truncation error of that
// double series grows with d: for every p it stays below about 3e-5 of the
// pair's value up to |d| = 2.5 at half sides rho_max(p) sigma / 2 (measured on
// corner-heavy point sets), hence kBoxAdmitR.
#include "internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace msp {
namespace {

constexpr int kBlock = 256;
constexpr int64_t kNoItem = INT64_MIN;
enum UnitKind : int32_t { K_OCT = 0, K_LEAF = 1, K_SRC = 2, K_BOX = 3 };
constexpr int kC1 = 70, kC2 = 70;          // Algorithm 2's dendrite and axon thresholds
constexpr int kBoxPMax = 10;               // box pairs by expansion for p up to this
constexpr double kBoxAdmitR = 2.5;         // expansion for box centres within this many sigma
constexpr int64_t kBoxPairsNoCutoff = (int64_t)1 << 22;   // without a cutoff: box path up to this many pairs
constexpr int kBoxStack = 176;             // > 7 kDepth + 1: the traversal's deepest stack
constexpr int64_t kBoxBrute = 16384;       // up to this many boxes, each axon box tests every box
constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// One choice: candidates' values from queries [r0, r1) (K_OCT, 8 octants), from
// direct tasks [r0, r1) against ncand neurons each (K_LEAF), from per-candidate
// task ranges crng[c0 + c] (K_SRC), or from the boxes [r0, r1) of the axon node,
// their pairs binned by the octant of the dendrite box under node c0 (K_BOX, 8
// octants).
struct UnitDesc {
    int64_t item;
    int64_t r0, r1, c0;
    int32_t kind, ncand;
};

__device__ inline uint64_t sm_mix(uint64_t x) {   // SplitMix64 output for state x
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ inline double desc_uniform(uint64_t seed, int step, int64_t item) {
    const uint64_t v = sm_mix(sm_mix(seed ^ ((uint64_t)(step + 1) * 0x9E3779B97F4A7C15ull)) ^ (uint64_t)item);
    return (double)(v >> 11) * 0x1.0p-53;
}

__device__ inline uint64_t desc_priority(uint64_t seed, int64_t axon) {
    return sm_mix(sm_mix(seed ^ 0xD1B54A32D192ED03ull) ^ (uint64_t)axon);
}

// Counters of a descent in device memory (int64 slots).
enum Ctr : int {
    C_M = 0,     // pairs in the current frontier
    C_NU,        // units of the step (scan total)
    C_SNR,       // requests of the step (scan total)
    C_NR,        // requests so far
    C_NQ,        // queries, tasks, direct terms, K_SRC range entries of the step (scan totals)
    C_NT,
    C_NDV,
    C_NCR,
    C_STEPS,     // steps that started with a non-empty frontier
    C_ERR,       // a table would have exceeded its capacity, or an absent octant was chosen
    C_LIVE,      // units of the step whose choice kept their pair
    C_COUNT = 16
};

// direct terms w_j K(t_i, s_j) of one axon neuron i (key order) against the
// neurons cf .. cf + nc - 1 (key order; the pair j = i is 0); one wavefront per
// task, the tasks of the step counted in *ntask
__global__ void __launch_bounds__(256) k_desc_direct(const int64_t *ntask, const int32_t *ti, const int32_t *tcf,
                                                     const int32_t *tnc, const int64_t *toff, const float4 *ps,
                                                     double inv_s2, double *dv) {
    const int lane = threadIdx.x & 63;
    const int64_t nt = *ntask;
    for (int64_t task = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); task < nt; task += (int64_t)gridDim.x * 4) {
        const int32_t i = ti[task], cf = tcf[task], nc = tnc[task];
        const int64_t off = toff[task];
        const float4 q = ps[i];
        for (int k = lane; k < nc; k += 64) {
            const int32_t j = cf + k;
            double v = 0.0;
            if (j != i) {
                const float4 s = ps[j];
                const double dx = (double)q.x - s.x, dy = (double)q.y - s.y, dz = (double)q.z - s.z;
                v = (double)s.w * exp(-(dx * dx + dy * dy + dz * dz) * inv_s2);
            }
            dv[off + k] = v;
        }
    }
}

// value of candidate k of a K_LEAF or K_SRC unit (FP64, fixed summation order)
__device__ inline double unit_value(const UnitDesc &U, int k, const double *raw, const float *qa,
                                    const double *dv, const int64_t *toff, const float *ta, const int64_t *crng) {
    double v = 0.0;
    if (U.kind == K_LEAF) {
        for (int64_t t = U.r0; t < U.r1; ++t) v += (double)ta[t] * dv[toff[t] + k];
    } else {
        const int64_t b = crng[2 * (U.c0 + k)], e = crng[2 * (U.c0 + k) + 1];
        for (int64_t t = b; t < e; ++t) v += (double)ta[t] * dv[toff[t]];
    }
    return v;
}

// acceptance: requests bucketed by dendrite, ranked by (priority, axon)
__global__ void k_desc_zero(int64_t n, int32_t *a, int32_t *b) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g < n) {
        a[g] = 0;
        b[g] = 0;
    }
}

__global__ void k_req_count(int64_t nr, const int32_t *rd, int32_t *cnt) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g < nr) atomicAdd(&cnt[rd[g]], 1);
}

// exclusive prefix sum of cnt[0 .. n) into off (one block, chunks of 1024)
__global__ void __launch_bounds__(1024) k_req_scan(int64_t n, const int32_t *cnt, int32_t *off) {
    __shared__ int32_t part[1024];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < n; c0 += 1024) {
        const int64_t g = c0 + threadIdx.x;
        const int32_t v = g < n ? cnt[g] : 0;
        part[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int32_t t = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0;
            __syncthreads();
            part[threadIdx.x] += t;
            __syncthreads();
        }
        if (g < n) off[g] = carry + part[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 0) carry += part[1023];
        __syncthreads();
    }
}

__global__ void k_req_fill(int64_t nr, const int32_t *rd, const int32_t *off, int32_t *fill, int32_t *bucket) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g < nr) {
        const int32_t j = rd[g];
        bucket[off[j] + atomicAdd(&fill[j], 1)] = (int32_t)g;
    }
}

__global__ void k_req_rank(int64_t nr, const int32_t *ra, const int32_t *rd, const int32_t *off,
                           const int32_t *cnt, const int32_t *bucket, const float *w, uint64_t seed,
                           uint8_t *accepted) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= nr) return;
    const int32_t j = rd[g], i = ra[g];
    const uint64_t pi = desc_priority(seed, i);
    const int32_t b = off[j], e = off[j] + cnt[j];
    int rank = 0;
    for (int32_t k = b; k < e; ++k) {
        const int32_t r = bucket[k];
        if (r == g) continue;
        const int32_t i2 = ra[r];
        const uint64_t p2 = desc_priority(seed, i2);
        rank += (p2 < pi || (p2 == pi && i2 < i)) ? 1 : 0;
    }
    accepted[g] = (double)rank < floor((double)w[j]) ? 1 : 0;
}

// ---- box pairs ------------------------------------------------------------

// What the box kernels read and write.
struct BoxArgs {
    int64_t nbox;
    int level;                                    // the box level
    const int32_t *node_box;                      // node -> box (-1: not a box)
    const int32_t *box_node, *box_na, *box_nd;    // box -> node, axon and dendrite neurons
    const int64_t *pair_off;                      // pairs of axon box s: pair_off[s] .. pair_off[s + 1]
    int32_t *pair_s, *pair_c;                     // axon box, dendrite box of each pair
    double *F;                                    // Att(s, c) of each pair
    float *A, *M;                                 // per box: A_alpha, Mt_beta (p^3 each)
    const int32_t *nlevel, *nix, *niy, *niz, *nfirst, *ncount, *nfchild, *nnchild;
    double lox, loy, loz, side;
    const float4 *ps;                             // key order: positions, staged w
    const float *akey;                            // key order: a
    double inv_sigma;
    double cut;                                   // largest box gap of a pair (length); < 0: none
    const uint64_t *box_key;                      // Morton key of each box's first point
    const double4 *box_geo;                       // centre and half side of each box
    int32_t *box_T, *box_stamp;                   // per box: dendrite node of its unit, and the step
    double *part;                                 // per box: its pairs' sums by octant under box_T (8)
};

__device__ inline void box_geom(const BoxArgs &g, int32_t u, double &cx, double &cy, double &cz, double &half) {
    const double h = g.side / (double)(1ll << g.nlevel[u]);
    cx = g.lox + (g.nix[u] + 0.5) * h;
    cy = g.loy + (g.niy[u] + 0.5) * h;
    cz = g.loz + (g.niz[u] + 0.5) * h;
    half = 0.5 * h;
}

// One thread per axon box: the dendrite boxes within the cutoff, by a walk from
// the root (children in key order, so the list of a box is in key order).  With
// cnt: counts only; otherwise the pairs go to pair_off[s] ...
__global__ void __launch_bounds__(256) k_box_lists(BoxArgs g, int64_t *cnt) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= g.nbox) return;
    int64_t n = 0;
    if (g.box_na[s] > 0) {
        double sx, sy, sz, sh;
        box_geom(g, g.box_node[s], sx, sy, sz, sh);
        const int64_t base = cnt ? 0 : g.pair_off[s];
        int32_t stk[kBoxStack];
        int sp = 0;
        stk[sp++] = 0;
        while (sp > 0) {
            const int32_t u = stk[--sp];
            if (g.cut >= 0.0) {
                double ux, uy, uz, uh;
                box_geom(g, u, ux, uy, uz, uh);
                const double gx = fmax(fabs(ux - sx) - uh - sh, 0.0);
                const double gy = fmax(fabs(uy - sy) - uh - sh, 0.0);
                const double gz = fmax(fabs(uz - sz) - uh - sh, 0.0);
                if (gx * gx + gy * gy + gz * gz > g.cut * g.cut) continue;
            }
            const int32_t bu = g.node_box[u];
            if (bu >= 0) {
                if (g.box_nd[bu] > 0) {
                    if (!cnt) {
                        g.pair_s[base + n] = (int32_t)s;
                        g.pair_c[base + n] = bu;
                    }
                    ++n;
                }
                continue;
            }
            const int32_t nc = g.nnchild[u], fc = g.nfchild[u];
            for (int k = nc - 1; k >= 0 && sp < kBoxStack; --k) stk[sp++] = fc + k;
        }
    }
    if (cnt) cnt[s] = n;
}

// One wavefront per axon box: every dendrite box within the cutoff, tested 64 at
// a time in box order (so each list is in key order).  With cnt: counts only;
// otherwise the pairs go to pair_off[s] ...
__global__ void __launch_bounds__(256) k_box_lists_all(BoxArgs g, int64_t *cnt) {
    const int lane = threadIdx.x & 63;
    const int64_t s = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (s >= g.nbox) return;
    int64_t n = 0;
    if (g.box_na[s] > 0) {
        const double4 gs = g.box_geo[s];
        const int64_t base = cnt ? 0 : g.pair_off[s];
        const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
        for (int64_t c0 = 0; c0 < g.nbox; c0 += 64) {
            const int64_t c = c0 + lane;
            bool ok = c < g.nbox && g.box_nd[c] > 0;
            if (ok && g.cut >= 0.0) {
                const double4 gc = g.box_geo[c];
                const double gx = fmax(fabs(gc.x - gs.x) - gc.w - gs.w, 0.0);
                const double gy = fmax(fabs(gc.y - gs.y) - gc.w - gs.w, 0.0);
                const double gz = fmax(fabs(gc.z - gs.z) - gc.w - gs.w, 0.0);
                ok = gx * gx + gy * gy + gz * gz <= g.cut * g.cut;
            }
            const uint64_t mask = __ballot(ok);
            if (!cnt && ok) {
                const int64_t pos = base + n + __popcll(mask & below);
                g.pair_s[pos] = (int32_t)s;
                g.pair_c[pos] = (int32_t)c;
            }
            n += __popcll(mask);
        }
    }
    if (cnt && lane == 0) cnt[s] = n;
}

// One wavefront per box whose unit this step is a K_BOX unit (box_stamp): its
// pairs binned by the octant of the dendrite box under the unit's node T (pairs
// outside T dropped), by the boxes' key prefixes.
__global__ void __launch_bounds__(256) k_box_partials(BoxArgs g, const uint64_t *keys, int step) {
    const int lane = threadIdx.x & 63;
    for (int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); b < g.nbox; b += (int64_t)gridDim.x * 4) {
        if (g.box_stamp[b] != step) continue;
        const int32_t T = g.box_T[b];
        const int lt = g.nlevel[T];
        const uint64_t kt = keys[g.nfirst[T]];
        const int sh0 = 3 * (kDepth - lt), sh1 = sh0 - 3;
        const uint64_t pt = sh0 >= 64 ? 0ull : kt >> sh0;
        double acc[8];
#pragma unroll
        for (int d = 0; d < 8; ++d) acc[d] = 0.0;
        for (int64_t k = g.pair_off[b] + lane; k < g.pair_off[b + 1]; k += 64) {
            const uint64_t kc = g.box_key[g.pair_c[k]];
            if ((sh0 >= 64 ? 0ull : kc >> sh0) != pt) continue;
            const int d = (int)((kc >> sh1) & 7);
            const double x = g.F[k];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (q == d) acc[q] += x;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
#pragma unroll
            for (int d = 0; d < 8; ++d) acc[d] += __shfl_xor(acc[d], o, 64);
        if (lane < 8) {
            double v = 0.0;
#pragma unroll
            for (int d = 0; d < 8; ++d)
                if (d == lane) v = acc[d];
            g.part[b * 8 + lane] = v;
        }
    }
}

// One wavefront per box at or below the box level: A_alpha (weights w) when the
// box holds more than c1 dendrites, Mt_beta (weights a) when it holds more than
// c2 axons, both about the box centre; the points pass through LDS 64 at a time
// as their powers per axis.
template <int P>
__global__ void __launch_bounds__(64) k_box_moments(BoxArgs g) {
    constexpr int P3 = P * P * P, PER = (P3 + 63) / 64, ROW = 3 * P + 2;
    const int64_t b = blockIdx.x;
    const int lane = threadIdx.x;
    const int32_t v = g.box_node[b];
    if (g.nlevel[v] < g.level) return;
    const bool wantA = g.box_nd[b] > kC1, wantM = g.box_na[b] > kC2;
    if (!wantA && !wantM) return;
    double cx, cy, cz, half;
    box_geom(g, v, cx, cy, cz, half);
    const float fx = (float)cx, fy = (float)cy, fz = (float)cz, is = (float)g.inv_sigma;
    __shared__ float pw[64 * ROW];
    int ia[PER], ib[PER], ic[PER];
    float accA[PER], accM[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int m = lane + 64 * k < P3 ? lane + 64 * k : 0;
        ia[k] = m % P;
        ib[k] = P + (m / P) % P;
        ic[k] = 2 * P + m / (P * P);
        accA[k] = 0.f;
        accM[k] = 0.f;
    }
    const int32_t f = g.nfirst[v], cnt = g.ncount[v];
    for (int32_t c0 = 0; c0 < cnt; c0 += 64) {
        const int32_t j = c0 + lane;
        float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
        float aj = 0.f;
        if (j < cnt) {
            q = g.ps[f + j];
            aj = g.akey[f + j];
        }
        float *r = pw + lane * ROW;
        const float y[3] = {(q.x - fx) * is, (q.y - fy) * is, (q.z - fz) * is};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            float t = 1.f;
#pragma unroll
            for (int k = 0; k < P; ++k) {
                r[d * P + k] = t;
                t *= y[d];
            }
        }
        r[3 * P] = q.w;
        r[3 * P + 1] = aj;
        __syncthreads();
        const int m = cnt - c0 < 64 ? cnt - c0 : 64;
        for (int jj = 0; jj < m; ++jj) {
            const float *rr = pw + jj * ROW;
            const float wj = rr[3 * P], aa = rr[3 * P + 1];
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const float t = rr[ia[k]] * rr[ib[k]] * rr[ic[k]];
                accA[k] = fmaf(wj, t, accA[k]);
                accM[k] = fmaf(aa, t, accM[k]);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int m = lane + 64 * k;
        if (m >= P3) continue;
        const int ax = ia[k], ay = ib[k] - P, az = ic[k] - 2 * P;
        float fact = 1.f;
        for (int e = 2; e <= ax; ++e) fact *= (float)e;
        for (int e = 2; e <= ay; ++e) fact *= (float)e;
        for (int e = 2; e <= az; ++e) fact *= (float)e;
        if (wantA) g.A[b * P3 + m] = accA[k] / fact;
        if (wantM) g.M[b * P3 + m] = ((ax + ay + az) & 1 ? -accM[k] : accM[k]) / fact;
    }
}

__device__ inline double wave_sum_d(double x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// One wavefront per box pair: Att(s, c) by the expansions (the double series,
// contracted one axis at a time in LDS) or directly (float32 terms relative to
// the pair's closest approach, float64 sums).
template <int P>
__global__ void __launch_bounds__(64) k_box_pair_values(BoxArgs g, int64_t npair) {
    constexpr int P2 = P * P, P3 = P2 * P, NH = 2 * P - 1;
    const int64_t k = blockIdx.x;
    const int lane = threadIdx.x;
    if (k >= npair) return;
    const int32_t s = g.pair_s[k], c = g.pair_c[k];
    const int32_t vs = g.box_node[s], vc = g.box_node[c];
    double sx, sy, sz, sh, cx, cy, cz, ch;
    box_geom(g, vs, sx, sy, sz, sh);
    box_geom(g, vc, cx, cy, cz, ch);
    const double dx = (sx - cx) * g.inv_sigma, dy = (sy - cy) * g.inv_sigma, dz = (sz - cz) * g.inv_sigma;
    const bool expo = g.nlevel[vs] >= g.level && g.nlevel[vc] >= g.level && g.box_na[s] > kC2 &&
                      g.box_nd[c] > kC1 && dx * dx + dy * dy + dz * dz <= kBoxAdmitR * kBoxAdmitR;
    const int32_t fs = g.nfirst[vs], ns = g.ncount[vs];
    double val = 0.0;
    if (expo) {
        __shared__ float sA[P3], sM[P3], sX[P3];
        __shared__ float hh[3][NH + 1];
        for (int m = lane; m < P3; m += 64) {
            sA[m] = g.A[(int64_t)c * P3 + m];
            sM[m] = g.M[(int64_t)s * P3 + m];
        }
        if (lane < 3) {   // h_0 .. h_{2p-2} at the centre offset, by the recurrence in FP64
            const double y = lane == 0 ? dx : lane == 1 ? dy : dz;
            double h0 = exp(-y * y), h1 = 2.0 * y * h0;
            hh[lane][0] = (float)h0;
            if (NH > 1) hh[lane][1] = (float)h1;
            for (int n = 1; n + 1 < NH; ++n) {
                const double h2 = 2.0 * y * h1 - 2.0 * n * h0;
                hh[lane][n + 1] = (float)h2;
                h0 = h1;
                h1 = h2;
            }
        }
        __syncthreads();
        // X[az][ay][bx] = sum_ax A[az][ay][ax] h(ax + bx, dx)
        for (int m = lane; m < P3; m += 64) {
            const int bx = m % P, row = m / P;
            float acc = 0.f;
#pragma unroll
            for (int ax = 0; ax < P; ++ax) acc = fmaf(sA[row * P + ax], hh[0][ax + bx], acc);
            sX[m] = acc;
        }
        __syncthreads();
        // Y[az][by][bx] = sum_ay X[az][ay][bx] h(ay + by, dy), into sA
        for (int m = lane; m < P3; m += 64) {
            const int bx = m % P, by = (m / P) % P, az = m / P2;
            float acc = 0.f;
#pragma unroll
            for (int ay = 0; ay < P; ++ay) acc = fmaf(sX[(az * P + ay) * P + bx], hh[1][ay + by], acc);
            sA[m] = acc;
        }
        __syncthreads();
        // sum_beta Mt[bz][by][bx] sum_az Y[az][by][bx] h(az + bz, dz)
        float part = 0.f;
        for (int m = lane; m < P3; m += 64) {
            const int bx = m % P, by = (m / P) % P, bz = m / P2;
            float z = 0.f;
#pragma unroll
            for (int az = 0; az < P; ++az) z = fmaf(sA[(az * P + by) * P + bx], hh[2][az + bz], z);
            part = fmaf(z, sM[m], part);
        }
        val = wave_sum_d((double)part);
        if (s == c) {   // the series includes the pairs j = i: a_i w_i K(0) each
            double self = 0.0;
            for (int32_t i = lane; i < ns; i += 64) self += (double)g.akey[fs + i] * (double)g.ps[fs + i].w;
            val -= wave_sum_d(self);
        }
    } else {
        // exp(-d^2 / sigma^2) = exp(-g^2 / sigma^2) exp(-(d^2 - g^2) / sigma^2) with g the
        // gap between the boxes (d >= g): the second factor in float32 (each term
        // to about 1e-5 at |d| = 6 sigma), the first once per pair in float64
        const int32_t fc = g.nfirst[vc], nc = g.ncount[vc];
        const double gx = fmax(fabs(sx - cx) - sh - ch, 0.0), gy = fmax(fabs(sy - cy) - sh - ch, 0.0),
                     gz = fmax(fabs(sz - cz) - sh - ch, 0.0);
        const double gap2 = gx * gx + gy * gy + gz * gz;
        const float g2 = (float)gap2, ks = (float)(g.inv_sigma * g.inv_sigma * 1.4426950408889634);
        double part = 0.0;
        for (int32_t j0 = 0; j0 < nc; j0 += 256) {
            // up to four dendrite points per lane (as many as the box needs), held while
            // the axon points pass
            const int nb = nc - j0 >= 256 ? 4 : (nc - j0 + 63) / 64;
            float4 q[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int32_t j = j0 + lane + 64 * u;
                q[u] = j < nc ? g.ps[fc + j] : make_float4(0.f, 0.f, 0.f, 0.f);
            }
            for (int32_t i = 0; i < ns; ++i) {
                const float ai = g.akey[fs + i];
                if (ai == 0.f) continue;
                const float4 ti = g.ps[fs + i];
                float row = 0.f;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (u >= nb) break;
                    const int32_t j = j0 + lane + 64 * u;
                    const float ex = ti.x - q[u].x, ey = ti.y - q[u].y, ez = ti.z - q[u].z;
                    const float e = __builtin_amdgcn_exp2f((g2 - (ex * ex + ey * ey + ez * ez)) * ks);
                    // (padding lanes hold no point: their e is not a term and may overflow)
                    row += j < nc && fc + j != fs + i ? q[u].w * e : 0.f;
                }
                part += (double)ai * (double)row;
            }
        }
        val = wave_sum_d(part) * exp(-gap2 * g.inv_sigma * g.inv_sigma);
    }
    if (lane == 0) g.F[k] = val;
}

// one wavefront per unit (the units of the step counted in *nunit).  K_OCT: the
// lanes split the queries; K_BOX: the lanes split the axon node's boxes (their
// per-octant sums from k_box_partials); both end in a butterfly sum (every lane
// ends with all eight values).  Otherwise candidate values 64 at a time (lane per candidate),
// total and running sums in candidate order by lane 0.
__global__ void __launch_bounds__(256) k_desc_choose(const int64_t *nunit, const UnitDesc *units, const double *raw,
                                                     const float *qa, const double *dv, const int64_t *toff,
                                                     const float *ta, const int64_t *crng, BoxArgs g,
                                                     uint64_t seed, int step, int32_t *out) {
    __shared__ double sv[4][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t nu = *nunit;
    for (int64_t u = (int64_t)blockIdx.x * 4 + wave; u < nu; u += (int64_t)gridDim.x * 4) {
        const UnitDesc U = units[u];
        if (U.kind == K_OCT || U.kind == K_BOX) {
            double acc[8];
#pragma unroll
            for (int d = 0; d < 8; ++d) acc[d] = 0.0;
            if (U.kind == K_BOX) {   // the boxes [r0, r1) of the axon node, summed per octant
                for (int64_t b = U.r0 + lane; b < U.r1; b += 64)
#pragma unroll
                    for (int d = 0; d < 8; ++d) acc[d] += g.part[b * 8 + d];
            } else {
                for (int64_t q = U.r0 + lane; q < U.r1; q += 64) {
                    const double aq = (double)qa[q];
#pragma unroll
                    for (int d = 0; d < 8; ++d) acc[d] = fma(aq, raw[q * 8 + d], acc[d]);
                }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1)
#pragma unroll
                for (int d = 0; d < 8; ++d) acc[d] += __shfl_xor(acc[d], o, 64);
            double tot = 0.0;
#pragma unroll
            for (int d = 0; d < 8; ++d) tot += acc[d];
            int pk = -1;
            if (tot > 0.0) {
                const double target = desc_uniform(seed, step, U.item) * tot;
                double run = 0.0;
                int last = -1;
#pragma unroll
                for (int d = 0; d < 8; ++d) {
                    if (pk >= 0) continue;
                    if (acc[d] > 0.0) last = d;
                    run += acc[d];
                    if (run > target && acc[d] > 0.0) pk = d;
                }
                if (pk < 0) pk = last;
            }
            if (lane == 0) out[u] = pk;
            continue;
        }
        const int nc = U.ncand;
        double total = 0.0;
        for (int k0 = 0; k0 < nc; k0 += 64) {
            const int k = k0 + lane;
            const double v = k < nc ? unit_value(U, k, raw, qa, dv, toff, ta, crng) : 0.0;
            sv[wave][lane] = v;
            wave_sync();
            if (lane == 0)
                for (int m = 0; m < 64 && k0 + m < nc; ++m) total += sv[wave][m];
            wave_sync();
        }
        total = __shfl(total, 0, 64);
        int pick = -1;
        if (total > 0.0) {
            const double target = desc_uniform(seed, step, U.item) * total;
            double run = 0.0;
            int last = -1;
            for (int k0 = 0; k0 < nc && pick < 0; k0 += 64) {
                const int k = k0 + lane;
                const double v = k < nc ? unit_value(U, k, raw, qa, dv, toff, ta, crng) : 0.0;
                sv[wave][lane] = v;
                wave_sync();
                if (lane == 0)
                    for (int m = 0; m < 64 && k0 + m < nc && pick < 0; ++m) {
                        const double x = sv[wave][m];
                        if (x > 0.0) last = k0 + m;
                        run += x;
                        if (run > target && x > 0.0) pick = k0 + m;
                    }
                pick = __shfl(pick, 0, 64);
                last = __shfl(last, 0, 64);
                run = __shfl(run, 0, 64);
                wave_sync();
            }
            if (pick < 0) pick = last;
        }
        if (lane == 0) out[u] = pick;
    }
}

// ---- device frontier ---------------------------------------------------------

// Exclusive prefix sums, in place, of C int64 columns (column c at data + c *
// stride) over the first *count entries; the column totals go to totals[0 .. C).
// Three launches: per block of kScanBlock entries, over the block sums (one
// block), and the block offsets added back.
constexpr int kScanBlock = 1024;

template <int C>
__global__ void __launch_bounds__(kScanBlock) k_scan_blocks(const int64_t *count, int64_t stride, int64_t *data,
                                                            int64_t *bsum) {
    __shared__ int64_t sh[kScanBlock];
    const int64_t n = *count;
    const int64_t nb = gridDim.x;
    const int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
    for (int c = 0; c < C; ++c) {
        const int64_t v = i < n ? data[c * stride + i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < kScanBlock; o <<= 1) {
            const int64_t t = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < n) data[c * stride + i] = sh[threadIdx.x] - v;
        if (threadIdx.x == kScanBlock - 1) bsum[c * nb + blockIdx.x] = sh[threadIdx.x];
        __syncthreads();
    }
}

template <int C>
__global__ void __launch_bounds__(kScanBlock) k_scan_top(int64_t nb, int64_t *bsum, int64_t *totals) {
    __shared__ int64_t sh[kScanBlock];
    __shared__ int64_t carry;
    for (int c = 0; c < C; ++c) {
        if (threadIdx.x == 0) carry = 0;
        __syncthreads();
        for (int64_t c0 = 0; c0 < nb; c0 += kScanBlock) {
            const int64_t g = c0 + threadIdx.x;
            const int64_t v = g < nb ? bsum[c * nb + g] : 0;
            sh[threadIdx.x] = v;
            __syncthreads();
            for (int o = 1; o < kScanBlock; o <<= 1) {
                const int64_t t = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
                __syncthreads();
                sh[threadIdx.x] += t;
                __syncthreads();
            }
            if (g < nb) bsum[c * nb + g] = carry + sh[threadIdx.x] - v;
            __syncthreads();
            if (threadIdx.x == 0) carry += sh[kScanBlock - 1];
            __syncthreads();
        }
        if (threadIdx.x == 0) totals[c] = carry;
        __syncthreads();
    }
}

template <int C>
__global__ void __launch_bounds__(kScanBlock) k_scan_add(const int64_t *count, int64_t stride, int64_t *data,
                                                         const int64_t *bsum) {
    const int64_t n = *count;
    const int64_t nb = gridDim.x;
    const int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
    if (i >= n) return;
    for (int c = 0; c < C; ++c) data[c * stride + i] += bsum[c * nb + blockIdx.x];
}

// A unit before its lists exist: the choosing item X, the other item of the pair,
// its kind and which side the choice replaces (0: the dendrite side, 1: the axon
// side).
struct UnitSpec {
    int64_t X, Tn;
    int32_t kind, side;
};

// What the step kernels read and write.
struct DescArgs {
    int64_t n, nn;
    const int32_t *perm, *iperm, *nfirst, *ncount, *nfchild, *nnchild, *nlevel, *ndigit;
    const float *akey;          // a in key order
    const int64_t *axc;         // neurons with a > 0 before each key position (n + 1)
    int box_level;              // -1: no box pairs
    int64_t nbox;
    const int32_t *box_first;   // first point of each box (key order)
    int32_t *box_T, *box_stamp; // per box: dendrite node of its K_BOX unit and the step
    int step;
    int64_t fcap, ucap, qcap, tcap, dvcap, crcap, rcap;   // capacities
    int64_t *ctr;
    const int64_t *S, *T;       // frontier
    int64_t *S2, *T2;           // next frontier (one entry per unit; kNoItem: dropped)
    int64_t *pcnt;              // per pair: units, requests (2 columns, stride fcap), then their offsets
    UnitSpec *spec;
    int64_t *ucnt;              // per unit: queries, tasks, terms, range entries (4 columns, stride ucap)
    UnitDesc *units;
    int32_t *qt, *qs, *qn;      // queries: target input index, key position, node
    float *qa;
    int32_t *ti, *tcf, *tnc;    // direct tasks
    int64_t *toff;
    float *ta;
    int64_t *crng;
    int32_t *choice;
    int32_t *req_a, *req_d;
};

__device__ inline void flag_error(const DescArgs &d) { atomicOr(reinterpret_cast<unsigned long long *>(d.ctr + C_ERR), 1ull); }

__device__ inline void item_range(const DescArgs &d, int64_t item, int64_t &f, int64_t &c) {
    if (item >= 0) {
        f = d.nfirst[item];
        c = d.ncount[item];
    } else {
        f = d.iperm[-item - 1];
        c = 1;
    }
}

__device__ inline int64_t axons_in(const DescArgs &d, int64_t f, int64_t c) { return d.axc[f + c] - d.axc[f]; }

__global__ void k_desc_init(int64_t *ctr, int64_t *S, int64_t *T, int64_t m0) {
    if (threadIdx.x < C_COUNT) ctr[threadIdx.x] = threadIdx.x == C_M ? m0 : 0;
    if (threadIdx.x == 0 && m0 > 0) {
        S[0] = 0;
        T[0] = 0;
    }
}

// per pair: how many units and requests it makes
__global__ void __launch_bounds__(256) k_pairs_count(DescArgs d) {
    const int64_t m = d.ctr[C_M];
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m && k < d.fcap;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t Si = d.S[k], Ti = d.T[k];
        int64_t nu = 0, nr = 0;
        if (Si == kNoItem) {
        } else if (Si < 0 && Ti < 0) {
            nr = 1;
        } else if (Si < 0 || Ti < 0) {
            nu = 1;
        } else {
            const int32_t nc = d.nnchild[Si];
            if (nc > 0) {
                const int32_t fc = d.nfchild[Si];
                for (int32_t c = 0; c < nc; ++c) nu += axons_in(d, d.nfirst[fc + c], d.ncount[fc + c]) > 0;
            } else {
                nu = axons_in(d, d.nfirst[Si], d.ncount[Si]);   // its neurons with axons
            }
        }
        d.pcnt[k] = nu;
        d.pcnt[d.fcap + k] = nr;
    }
}

// per pair: its requests, and its units' kinds and list sizes
__global__ void __launch_bounds__(256) k_pairs_fill(DescArgs d) {
    const int64_t m = d.ctr[C_M];
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m && k < d.fcap;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t Si = d.S[k], Ti = d.T[k];
        if (Si == kNoItem) continue;
        if (Si < 0 && Ti < 0) {
            const int64_t pos = d.ctr[C_NR] + d.pcnt[d.fcap + k];
            if (pos >= d.rcap) {
                flag_error(d);
                continue;
            }
            d.req_a[pos] = (int32_t)(-Si - 1);
            d.req_d[pos] = (int32_t)(-Ti - 1);
            continue;
        }
        int64_t u = d.pcnt[k];
        // kind K_OCT here stands for "over the children of Tn": K_OCT or K_LEAF by Tn
        auto emit = [&](int64_t X, int64_t Tn, int32_t kind, int32_t side) {
            if (u >= d.ucap) {
                flag_error(d);
                return;
            }
            int64_t nq = 0, nt = 0, ndv = 0, ncr = 0;
            if (kind == K_SRC) {
                const int32_t nc = d.nnchild[X];
                ncr = 2 * (int64_t)(nc > 0 ? nc : d.ncount[X]);
                nt = axons_in(d, d.nfirst[X], d.ncount[X]);
                ndv = nt;
            } else if (kind != K_BOX) {
                int64_t f, c;
                item_range(d, X, f, c);
                const int64_t ax = axons_in(d, f, c);
                if (d.nnchild[Tn] > 0) {
                    kind = K_OCT;
                    nq = ax;
                } else {
                    kind = K_LEAF;
                    nt = ax;
                    ndv = ax * d.ncount[Tn];
                }
            }
            d.spec[u] = UnitSpec{X, Tn, kind, side};
            d.ucnt[u] = nq;
            d.ucnt[d.ucap + u] = nt;
            d.ucnt[2 * d.ucap + u] = ndv;
            d.ucnt[3 * d.ucap + u] = ncr;
            ++u;
        };
        if (Si < 0) {
            emit(Si, Ti, K_OCT, 0);
        } else if (Ti < 0) {
            emit(Si, Ti, K_SRC, 1);
        } else {
            const int32_t nc = d.nnchild[Si];
            // both above the box level, both with child nodes: box pairs
            const bool boxes = d.box_level >= 0 && nc > 0 && d.nnchild[Ti] > 0 && d.nlevel[Si] < d.box_level &&
                               d.nlevel[Ti] < d.box_level;
            if (nc > 0) {
                const int32_t fc = d.nfchild[Si];
                for (int32_t c = 0; c < nc; ++c)
                    if (axons_in(d, d.nfirst[fc + c], d.ncount[fc + c]) > 0) emit(fc + c, Ti, boxes ? K_BOX : K_OCT, 0);
            } else {
                const int32_t f = d.nfirst[Si], e = f + d.ncount[Si];
                for (int32_t p = f; p < e; ++p)
                    if (d.akey[p] > 0.f) emit(-(int64_t)d.perm[p] - 1, Ti, K_OCT, 0);
            }
        }
    }
}

// the key positions p in [f, f + c) with a_p > 0, in order, to emit(index, p); one
// wavefront; returns how many (wave-uniform)
template <class F>
__device__ inline int64_t each_axon(const DescArgs &d, int64_t f, int64_t c, int lane, F emit) {
    int64_t w = 0;
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (int64_t b = f; b < f + c; b += 64) {
        const int64_t p = b + lane;
        const bool is_ax = p < f + c && d.akey[p] > 0.f;
        const uint64_t mask = __ballot(is_ax);
        if (is_ax) emit(w + __popcll(mask & below), p);
        w += __popcll(mask);
    }
    return w;
}

__device__ inline int64_t lower_bound_i32(const int32_t *a, int64_t n, int32_t key) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// one wavefront per unit: its queries or tasks and its descriptor
__global__ void __launch_bounds__(256) k_units_fill(DescArgs d) {
    const int lane = threadIdx.x & 63;
    const int64_t nu = d.ctr[C_NU];
    for (int64_t u = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); u < nu && u < d.ucap;
         u += (int64_t)gridDim.x * 4) {
        const UnitSpec sp = d.spec[u];
        int64_t off[4], cnt[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            off[c] = d.ucnt[c * d.ucap + u];
            cnt[c] = (u + 1 < nu ? d.ucnt[c * d.ucap + u + 1] : d.ctr[C_NQ + c]) - off[c];
        }
        if (off[0] + cnt[0] > d.qcap || off[1] + cnt[1] > d.tcap || off[2] + cnt[2] > d.dvcap ||
            off[3] + cnt[3] > d.crcap) {
            if (lane == 0) flag_error(d);
            continue;
        }
        const int64_t X = sp.X, Tn = sp.Tn;
        UnitDesc U{X, 0, 0, 0, sp.kind, 8};
        if (sp.kind == K_OCT) {
            int64_t f, c;
            item_range(d, X, f, c);
            const int64_t qo = off[0];
            each_axon(d, f, c, lane, [&](int64_t k, int64_t p) {
                d.qt[qo + k] = d.perm[p];
                d.qs[qo + k] = (int32_t)p;
                d.qn[qo + k] = (int32_t)Tn;
                d.qa[qo + k] = d.akey[p];
            });
            U.r0 = qo;
            U.r1 = qo + cnt[0];
        } else if (sp.kind == K_BOX) {
            const int32_t f = d.nfirst[X], e = f + d.ncount[X];
            U.r0 = lower_bound_i32(d.box_first, d.nbox, f);
            U.r1 = lower_bound_i32(d.box_first, d.nbox, e);
            U.c0 = Tn;
            for (int64_t b = U.r0 + lane; b < U.r1; b += 64) {
                d.box_T[b] = (int32_t)Tn;
                d.box_stamp[b] = d.step;
            }
        } else if (sp.kind == K_LEAF) {
            int64_t f, c;
            item_range(d, X, f, c);
            const int32_t tf = d.nfirst[Tn], tc = d.ncount[Tn];
            const int64_t to = off[1], dvo = off[2];
            each_axon(d, f, c, lane, [&](int64_t k, int64_t p) {
                d.ti[to + k] = (int32_t)p;
                d.tcf[to + k] = tf;
                d.tnc[to + k] = tc;
                d.toff[to + k] = dvo + k * tc;
                d.ta[to + k] = d.akey[p];
            });
            U.r0 = to;
            U.r1 = to + cnt[1];
            U.ncand = tc;
        } else {   // K_SRC: the children of node X against the neuron Tn
            const int32_t pt = d.iperm[-Tn - 1];
            const int32_t nc = d.nnchild[X];
            const int64_t nch = nc > 0 ? nc : d.ncount[X];
            const int64_t to = off[1], dvo = off[2], cro = off[3];
            int64_t w = 0;
            for (int64_t k = 0; k < nch; ++k) {
                int64_t cf, cc;
                if (nc > 0) {
                    cf = d.nfirst[d.nfchild[X] + k];
                    cc = d.ncount[d.nfchild[X] + k];
                } else {
                    cf = d.nfirst[X] + k;
                    cc = 1;
                }
                const int64_t w0 = w;
                w += each_axon(d, cf, cc, lane, [&](int64_t kk, int64_t p) {
                    d.ti[to + w0 + kk] = (int32_t)p;
                    d.tcf[to + w0 + kk] = pt;
                    d.tnc[to + w0 + kk] = 1;
                    d.toff[to + w0 + kk] = dvo + w0 + kk;
                    d.ta[to + w0 + kk] = d.akey[p];
                });
                if (lane == 0) {
                    d.crng[cro + 2 * k] = to + w0;
                    d.crng[cro + 2 * k + 1] = to + w;
                }
            }
            U.r0 = to;
            U.r1 = to + cnt[1];
            U.c0 = cro / 2;
            U.ncand = (int32_t)nch;
        }
        if (lane == 0) d.units[u] = U;
    }
}

// per unit: the next pair from the choice (candidate k of the unit: the child of
// Tn in octant k for K_OCT and K_BOX, neuron k of the leaf Tn for K_LEAF, child k
// of X for K_SRC), or kNoItem when the choice dropped it
__global__ void __launch_bounds__(256) k_next(DescArgs d) {
    const int64_t nu = d.ctr[C_NU];
    unsigned long long live = 0;
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < nu && u < d.ucap;
         u += (int64_t)gridDim.x * blockDim.x) {
        const UnitSpec sp = d.spec[u];
        const int32_t k = d.choice[u];
        int64_t s2 = kNoItem, t2 = kNoItem;
        if (k >= 0) {
            int64_t nxt = kNoItem;
            if (sp.kind == K_OCT || sp.kind == K_BOX) {
                const int32_t fc = d.nfchild[sp.Tn], nc = d.nnchild[sp.Tn];
                for (int32_t c = 0; c < nc; ++c)
                    if (d.ndigit[fc + c] == k) nxt = fc + c;
            } else if (sp.kind == K_LEAF) {
                nxt = -(int64_t)d.perm[d.nfirst[sp.Tn] + k] - 1;
            } else {
                const int32_t nc = d.nnchild[sp.X];
                nxt = nc > 0 ? (int64_t)d.nfchild[sp.X] + k : -(int64_t)d.perm[d.nfirst[sp.X] + k] - 1;
            }
            if (nxt == kNoItem) {
                flag_error(d);
            } else if (sp.side == 0) {
                s2 = sp.X;
                t2 = nxt;
            } else {
                s2 = nxt;
                t2 = sp.Tn;
            }
        }
        d.S2[u] = s2;
        d.T2[u] = t2;
        live += s2 != kNoItem;
    }
    for (int o = 32; o > 0; o >>= 1) live += __shfl_xor(live, o, 64);
    if ((threadIdx.x & 63) == 0 && live > 0)
        atomicAdd(reinterpret_cast<unsigned long long *>(d.ctr + C_LIVE), live);
}

// After the prefix sums: a step whose tables would not fit stops the descent
// (the error flag is set and the step's counts are cleared, so that the later
// kernels of the step do nothing).
__global__ void k_clamp_pairs(int64_t *ctr, int64_t ucap, int64_t rcap) {
    if (threadIdx.x != 0) return;
    if (ctr[C_NU] > ucap || ctr[C_NR] + ctr[C_SNR] > rcap) {
        ctr[C_ERR] = 1;
        ctr[C_NU] = 0;
        ctr[C_SNR] = 0;
    }
}

__global__ void k_clamp_units(int64_t *ctr, int64_t qcap, int64_t tcap, int64_t dvcap, int64_t crcap) {
    if (threadIdx.x != 0) return;
    if (ctr[C_NQ] > qcap || ctr[C_NT] > tcap || ctr[C_NDV] > dvcap || ctr[C_NCR] > crcap) {
        ctr[C_ERR] = 1;
        ctr[C_NU] = 0;
        ctr[C_NQ] = ctr[C_NT] = ctr[C_NDV] = ctr[C_NCR] = 0;
    }
}

// the next frontier holds one entry per unit, or none when every choice dropped
// its pair
__global__ void k_step_end(int64_t *ctr) {
    if (threadIdx.x != 0) return;
    if (ctr[C_M] > 0) ctr[C_STEPS] += 1;
    ctr[C_NR] += ctr[C_SNR];
    ctr[C_M] = ctr[C_LIVE] > 0 ? ctr[C_NU] : 0;
    ctr[C_LIVE] = 0;
}

// key order: a gathered, and the prefix counts of neurons with a > 0 (as 0/1 then
// scanned)
__global__ void k_desc_akey(int64_t n, const int32_t *perm, const float *a, float *akey, int64_t *flag) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p > n) return;
    if (p == n) {
        flag[p] = 0;
        return;
    }
    const float v = a[perm[p]];
    akey[p] = v;
    flag[p] = v > 0.f ? 1 : 0;
}

// per box: neurons with a > 0 and with staged w > 0, the key of its first point,
// its centre and half side; no unit yet (stamp -1)
__global__ void k_box_counts(BoxArgs g, const int64_t *axc, const uint64_t *keys, int32_t *na, int32_t *nd,
                             uint64_t *key, double4 *geo) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= g.nbox) return;
    const int32_t v = g.box_node[b], f = g.nfirst[v], e = f + g.ncount[v];
    na[b] = (int32_t)(axc[e] - axc[f]);
    int32_t c = 0;
    for (int32_t p = f; p < e; ++p) c += g.ps[p].w > 0.f;
    nd[b] = c;
    key[b] = keys[f];
    double cx, cy, cz, half;
    box_geom(g, v, cx, cy, cz, half);
    geo[b] = make_double4(cx, cy, cz, half);
    g.box_stamp[b] = -1;
}

__global__ void k_set_i64(int64_t *p, int64_t v) {
    if (threadIdx.x == 0) *p = v;
}

// Exclusive scan of C columns of `stride` entries each (see k_scan_blocks); count
// in device memory, at most stride; bsum: C * ceil(stride / kScanBlock) entries.
template <int C>
int scan_cols(const int64_t *count, int64_t stride, int64_t *data, int64_t *bsum, int64_t *totals, hipStream_t s) {
    const int64_t nb = (stride + kScanBlock - 1) / kScanBlock;
    const unsigned g = (unsigned)(nb > 0 ? nb : 1);
    hipLaunchKernelGGL(k_scan_blocks<C>, dim3(g), dim3(kScanBlock), 0, s, count, stride, data, bsum);
    MSP_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_scan_top<C>, dim3(1), dim3(kScanBlock), 0, s, (int64_t)g, bsum, totals);
    MSP_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_scan_add<C>, dim3(g), dim3(kScanBlock), 0, s, count, stride, data, bsum);
    MSP_CHECK_LAUNCH();
    return MSP_OK;
}

inline int64_t scan_blocks(int64_t stride) { return (stride + kScanBlock - 1) / kScanBlock > 0 ? (stride + kScanBlock - 1) / kScanBlock : 1; }

template <class T>
int to_host(std::vector<T> &v, const void *dev, int64_t count) {
    v.resize((size_t)(count > 0 ? count : 0));
    if (count > 0) MSP_HIP(hipMemcpy(v.data(), dev, (size_t)count * sizeof(T), hipMemcpyDeviceToHost));
    return MSP_OK;
}

// Host side of one descent: what the setup learnt about the tree and the tables.
struct Descent {
    msp_tree *t = nullptr;
    int64_t n = 0, nn = 0, nax = 0, maxleaf = 1;
    std::vector<int32_t> nfirst, ncount, nfchild, nnchild, nlevel;   // host copies (setup, caps)
    BoxArgs box{};
    int box_level = -1;
    const int32_t *box_first = nullptr;
    const int64_t *axc = nullptr;
};

// Staged weights and node moments, a in key order with its prefix counts, the
// inverse permutation, and the box table with every box pair's attraction.
// Synchronises `s` (the topology for the box table, the axon count, the pair
// counts).  No box pairs (box_level -1) when p is beyond kBoxPMax, when the root
// is a leaf, or, without a cutoff, when the axon boxes times the dendrite boxes
// exceed kBoxPairsNoCutoff.
int desc_setup(Descent &D, msp_tree *t, const float *w, const float *a, const msp_fgt_params *prm, hipStream_t s) {
    D.t = t;
    D.n = t->n;
    D.nn = t->n_nodes;
    t->desc_box_level = -1;
    t->desc_nbox = t->desc_npair = 0;
    MSP_TRY(partner_prepare(t, w, prm, s));   // staged w, node moments
    MSP_TRY(ensure_iperm(t, s));
    const int64_t n = D.n;
    // a in key order and the prefix counts of neurons with a > 0
    MSP_TRY(t->desc_akey.ensure((size_t)(n > 0 ? n : 1) * 4));
    const int64_t nbp = scan_blocks(n + 1);
    MSP_TRY(t->desc_prefix.ensure((size_t)(n + 1 + nbp + 2) * 8));
    int64_t *axc = t->desc_prefix.as<int64_t>();
    int64_t *bsum = axc + n + 1, *cnt = bsum + nbp;
    hipLaunchKernelGGL(k_desc_akey, dim3(grid_for(n + 1, kBlock)), dim3(kBlock), 0, s, n, t->perm.as<int32_t>(), a,
                       t->desc_akey.as<float>(), axc);
    MSP_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(64), 0, s, cnt, n + 1);
    MSP_CHECK_LAUNCH();
    MSP_TRY(scan_cols<1>(cnt, n + 1, axc, bsum, cnt + 1, s));
    D.axc = axc;
    MSP_HIP(hipStreamSynchronize(s));
    // topology on the host: the box table's walk and the largest leaf
    MSP_TRY(to_host(D.nfirst, t->nfirst.p, D.nn));
    MSP_TRY(to_host(D.ncount, t->ncount.p, D.nn));
    MSP_TRY(to_host(D.nfchild, t->nfchild.p, D.nn));
    MSP_TRY(to_host(D.nnchild, t->nnchild.p, D.nn));
    MSP_TRY(to_host(D.nlevel, t->nlevel.p, D.nn));
    D.maxleaf = 1;
    for (int64_t v = 0; v < D.nn; ++v)
        if (D.nnchild[v] == 0 && D.ncount[v] > D.maxleaf) D.maxleaf = D.ncount[v];
    int64_t nax = 0;
    MSP_HIP(hipMemcpy(&nax, axc + n, 8, hipMemcpyDeviceToHost));
    D.nax = nax;
    // the box table
    D.box_level = -1;
    const int p = prm->p;
    if (p < 1 || p > kBoxPMax || D.nn == 0 || D.nnchild[0] == 0 || nax == 0) return MSP_OK;
    const double rmax = rho_max_for_p(p), sigma = prm->sigma;
    int lm = kDepth;
    for (int l = 0; l <= kDepth; ++l)
        if (t->geo.side / std::ldexp(1.0, l + 1) / sigma <= rmax) {
            lm = l;
            break;
        }
    const int L = lm + 1;
    // boxes in key order: a walk from the root that stops at the first node at or
    // below L and at leaves
    std::vector<int32_t> node_box((size_t)D.nn, -1), stk{0}, bnode, bfirst;
    while (!stk.empty()) {
        const int32_t u = stk.back();
        stk.pop_back();
        if (D.nlevel[u] >= L || D.nnchild[u] == 0) {
            bnode.push_back(u);
            continue;
        }
        for (int32_t k = D.nnchild[u] - 1; k >= 0; --k) stk.push_back(D.nfchild[u] + k);
    }
    std::sort(bnode.begin(), bnode.end(), [&](int32_t x, int32_t y) { return D.nfirst[x] < D.nfirst[y]; });
    const int64_t nbox = (int64_t)bnode.size();
    bfirst.resize((size_t)nbox);
    for (int64_t b = 0; b < nbox; ++b) {
        node_box[bnode[b]] = (int32_t)b;
        bfirst[b] = D.nfirst[bnode[b]];
    }
    // device: node -> box, then per box: node, first point, axons, dendrites, pair
    // offsets, pair counts, key, geometry, unit node, stamp, octant sums
    const size_t nb4 = align_up((size_t)nbox * 4), nb8 = align_up((size_t)nbox * 8);
    const size_t o_nb = 0, o_bn = align_up((size_t)D.nn * 4), o_bf = o_bn + nb4, o_na = o_bf + nb4,
                 o_nd = o_na + nb4, o_off = o_nd + nb4, o_cnt = o_off + align_up((size_t)(nbox + 1) * 8),
                 o_key = o_cnt + nb8, o_geo = o_key + nb8, o_T = o_geo + align_up((size_t)nbox * 32),
                 o_st = o_T + nb4, o_part = o_st + nb4, tot = o_part + align_up((size_t)nbox * 64);
    MSP_TRY(t->desc_box.ensure(tot));
    char *db = t->desc_box.as<char>();
    MSP_HIP(hipMemcpyAsync(db + o_nb, node_box.data(), (size_t)D.nn * 4, hipMemcpyHostToDevice, s));
    MSP_HIP(hipMemcpyAsync(db + o_bn, bnode.data(), (size_t)nbox * 4, hipMemcpyHostToDevice, s));
    MSP_HIP(hipMemcpyAsync(db + o_bf, bfirst.data(), (size_t)nbox * 4, hipMemcpyHostToDevice, s));
    int32_t *dna = reinterpret_cast<int32_t *>(db + o_na), *dnd = reinterpret_cast<int32_t *>(db + o_nd);
    BoxArgs &g = D.box;
    g = BoxArgs{};
    g.nbox = nbox;
    g.node_box = reinterpret_cast<const int32_t *>(db + o_nb);
    g.box_node = reinterpret_cast<const int32_t *>(db + o_bn);
    g.box_na = dna;
    g.box_nd = dnd;
    g.pair_off = reinterpret_cast<const int64_t *>(db + o_off);
    g.nlevel = t->nlevel.as<int32_t>();
    g.nix = t->nix.as<int32_t>();
    g.niy = t->niy.as<int32_t>();
    g.niz = t->niz.as<int32_t>();
    g.nfirst = t->nfirst.as<int32_t>();
    g.ncount = t->ncount.as<int32_t>();
    g.nfchild = t->nfchild.as<int32_t>();
    g.nnchild = t->nnchild.as<int32_t>();
    g.lox = t->geo.lo[0];
    g.loy = t->geo.lo[1];
    g.loz = t->geo.lo[2];
    g.side = t->geo.side;
    g.ps = t->ps.as<float4>();
    g.akey = t->desc_akey.as<float>();
    g.box_key = reinterpret_cast<const uint64_t *>(db + o_key);
    g.box_geo = reinterpret_cast<const double4 *>(db + o_geo);
    g.box_T = reinterpret_cast<int32_t *>(db + o_T);
    g.box_stamp = reinterpret_cast<int32_t *>(db + o_st);
    g.part = reinterpret_cast<double *>(db + o_part);
    hipLaunchKernelGGL(k_box_counts, dim3(grid_for(nbox, kBlock)), dim3(kBlock), 0, s, g, axc,
                       t->keys.as<uint64_t>(), dna, dnd, reinterpret_cast<uint64_t *>(db + o_key),
                       reinterpret_cast<double4 *>(db + o_geo));
    MSP_CHECK_LAUNCH();
    const bool unlimited = !(prm->cutoff_sigmas > 0.f);
    if (unlimited) {
        std::vector<int32_t> na((size_t)nbox), nd((size_t)nbox);
        MSP_HIP(hipMemcpyAsync(na.data(), dna, (size_t)nbox * 4, hipMemcpyDeviceToHost, s));
        MSP_HIP(hipMemcpyAsync(nd.data(), dnd, (size_t)nbox * 4, hipMemcpyDeviceToHost, s));
        MSP_HIP(hipStreamSynchronize(s));
        int64_t nab = 0, ndb = 0;
        for (int64_t b = 0; b < nbox; ++b) {
            nab += na[b] > 0;
            ndb += nd[b] > 0;
        }
        if ((double)nab * (double)ndb > (double)kBoxPairsNoCutoff) return MSP_OK;
    }
    g.level = L;
    g.inv_sigma = 1.0 / sigma;
    g.cut = unlimited ? -1.0 : (double)prm->cutoff_sigmas * sigma;
    // pair counts, offsets on the host, pairs
    int64_t *dcnt = reinterpret_cast<int64_t *>(db + o_cnt);
    std::vector<int64_t> pc((size_t)nbox), poff((size_t)nbox + 1, 0);
    const bool brute = nbox <= kBoxBrute;
    {
        PhaseScope ph(&t->timing, PH_DESC_BOXES, s);
        if (brute) hipLaunchKernelGGL(k_box_lists_all, dim3(grid_for(nbox, 4)), dim3(256), 0, s, g, dcnt);
        else hipLaunchKernelGGL(k_box_lists, dim3(grid_for(nbox, kBlock)), dim3(kBlock), 0, s, g, dcnt);
        MSP_CHECK_LAUNCH();
    }
    MSP_HIP(hipMemcpyAsync(pc.data(), dcnt, (size_t)nbox * 8, hipMemcpyDeviceToHost, s));
    MSP_HIP(hipStreamSynchronize(s));
    for (int64_t b = 0; b < nbox; ++b) poff[b + 1] = poff[b] + pc[b];
    const int64_t npair = poff[nbox];
    MSP_HIP(hipMemcpyAsync(db + o_off, poff.data(), (size_t)(nbox + 1) * 8, hipMemcpyHostToDevice, s));
    const size_t q_s = 0, q_c = align_up((size_t)npair * 4), q_f = q_c + align_up((size_t)npair * 4),
                 qtot = q_f + align_up((size_t)npair * 8);
    MSP_TRY(t->desc_pairs.ensure(qtot > 0 ? qtot : kAlign));
    char *dp = t->desc_pairs.as<char>();
    g.pair_s = reinterpret_cast<int32_t *>(dp + q_s);
    g.pair_c = reinterpret_cast<int32_t *>(dp + q_c);
    g.F = reinterpret_cast<double *>(dp + q_f);
    const int64_t P3 = (int64_t)p * p * p;
    MSP_TRY(t->desc_boxmom.ensure((size_t)nbox * P3 * 8));
    g.A = t->desc_boxmom.as<float>();
    g.M = g.A + nbox * P3;
    {
        PhaseScope ph(&t->timing, PH_DESC_BOXES, s);
        if (brute)
            hipLaunchKernelGGL(k_box_lists_all, dim3(grid_for(nbox, 4)), dim3(256), 0, s, g, (int64_t *)nullptr);
        else
            hipLaunchKernelGGL(k_box_lists, dim3(grid_for(nbox, kBlock)), dim3(kBlock), 0, s, g, (int64_t *)nullptr);
        MSP_CHECK_LAUNCH();
    }
    {
        PhaseScope ph(&t->timing, PH_DESC_PAIRS, s);
        switch (p) {
#define CASE(P)                                                                                           \
    case P:                                                                                               \
        hipLaunchKernelGGL(k_box_moments<P>, dim3((unsigned)nbox), dim3(64), 0, s, g);                   \
        MSP_CHECK_LAUNCH();                                                                               \
        if (npair > 0) {                                                                                  \
            hipLaunchKernelGGL(k_box_pair_values<P>, dim3((unsigned)npair), dim3(64), 0, s, g, npair);   \
            MSP_CHECK_LAUNCH();                                                                           \
        }                                                                                                 \
        break;
            CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
#undef CASE
        }
    }
    MSP_HIP(hipStreamSynchronize(s));   // the host vectors above are released on return
    D.box_level = L;
    D.box_first = reinterpret_cast<const int32_t *>(db + o_bf);
    t->desc_box_level = L;
    t->desc_nbox = nbox;
    t->desc_npair = npair;
    return MSP_OK;
}

// Capacities of one step's tables.
struct Caps {
    int64_t f, u, q, tk, dv, cr, r;
};

// The step tables carved from the tree's desc_lists (base NULL: sizes only), with
// the requests going to req_a / req_d (or to a region of the lists when NULL).
size_t carve_lists(Descent &D, const Caps &c, char *base, DescArgs *a, int64_t **bsumF, int64_t **bsumU,
                   int32_t *req_a, int32_t *req_d) {
    Carve cv(base, base ? SIZE_MAX : 0);
    auto take = [&](size_t bytes) { return cv.take(bytes); };
    DescArgs x{};
    x.ctr = static_cast<int64_t *>(take((size_t)C_COUNT * 8));
    x.S = static_cast<int64_t *>(take((size_t)c.f * 8));
    x.T = static_cast<int64_t *>(take((size_t)c.f * 8));
    x.S2 = static_cast<int64_t *>(take((size_t)c.u * 8));
    x.T2 = static_cast<int64_t *>(take((size_t)c.u * 8));
    x.pcnt = static_cast<int64_t *>(take((size_t)c.f * 2 * 8));
    *bsumF = static_cast<int64_t *>(take((size_t)scan_blocks(c.f) * 2 * 8));
    x.spec = static_cast<UnitSpec *>(take((size_t)c.u * sizeof(UnitSpec)));
    x.ucnt = static_cast<int64_t *>(take((size_t)c.u * 4 * 8));
    *bsumU = static_cast<int64_t *>(take((size_t)scan_blocks(c.u) * 4 * 8));
    x.units = static_cast<UnitDesc *>(take((size_t)c.u * sizeof(UnitDesc)));
    x.choice = static_cast<int32_t *>(take((size_t)c.u * 4));
    x.qt = static_cast<int32_t *>(take((size_t)c.q * 4));
    x.qs = static_cast<int32_t *>(take((size_t)c.q * 4));
    x.qn = static_cast<int32_t *>(take((size_t)c.q * 4));
    x.qa = static_cast<float *>(take((size_t)c.q * 4));
    x.ti = static_cast<int32_t *>(take((size_t)c.tk * 4));
    x.tcf = static_cast<int32_t *>(take((size_t)c.tk * 4));
    x.tnc = static_cast<int32_t *>(take((size_t)c.tk * 4));
    x.toff = static_cast<int64_t *>(take((size_t)c.tk * 8));
    x.ta = static_cast<float *>(take((size_t)c.tk * 4));
    x.crng = static_cast<int64_t *>(take((size_t)c.cr * 8));
    if (req_a) {
        x.req_a = req_a;
        x.req_d = req_d;
    } else {
        x.req_a = static_cast<int32_t *>(take((size_t)c.r * 4));
        x.req_d = static_cast<int32_t *>(take((size_t)c.r * 4));
    }
    msp_tree *t = D.t;
    x.n = D.n;
    x.nn = D.nn;
    x.perm = t->perm.as<int32_t>();
    x.iperm = t->iperm.as<int32_t>();
    x.nfirst = t->nfirst.as<int32_t>();
    x.ncount = t->ncount.as<int32_t>();
    x.nfchild = t->nfchild.as<int32_t>();
    x.nnchild = t->nnchild.as<int32_t>();
    x.nlevel = t->nlevel.as<int32_t>();
    x.ndigit = t->ndigit.as<int32_t>();
    x.akey = t->desc_akey.as<float>();
    x.axc = D.axc;
    x.box_level = D.box_level;
    x.nbox = D.box.nbox;
    x.box_first = D.box_first;
    x.box_T = D.box.box_T;
    x.box_stamp = D.box.box_stamp;
    x.fcap = c.f;
    x.ucap = c.u;
    x.qcap = c.q;
    x.tcap = c.tk;
    x.dvcap = c.dv;
    x.crcap = c.cr;
    x.rcap = c.r;
    if (a) *a = x;
    return cv.used;
}

int lists_for(Descent &D, const Caps &c, DescArgs &a, int64_t **bsumF, int64_t **bsumU, int32_t *req_a,
              int32_t *req_d) {
    msp_tree *t = D.t;
    const size_t bytes = carve_lists(D, c, nullptr, nullptr, bsumF, bsumU, req_a, req_d);
    MSP_TRY(t->desc_lists.ensure(bytes));
    carve_lists(D, c, t->desc_lists.as<char>(), &a, bsumF, bsumU, req_a, req_d);
    MSP_TRY(t->desc_raw.ensure((size_t)(c.q > 0 ? c.q : 1) * 8 * sizeof(double)));
    MSP_TRY(t->desc_probs.ensure((size_t)(c.q > 0 ? c.q : 1) * 8 * sizeof(float)));
    MSP_TRY(t->desc_dv.ensure((size_t)(c.dv > 0 ? c.dv : 1) * sizeof(double)));
    return MSP_OK;
}

inline unsigned capped_grid(int64_t items, int per_block, unsigned cap) {
    const unsigned g = grid_for(items > 0 ? items : 1, per_block);
    return g < cap ? g : cap;
}

// One step, all on the device: units and requests per pair, their offsets, the
// units' lists, the partner queries and direct terms, the choices, the next
// frontier (a.S2 / a.T2, one entry per unit) and the counters.
int launch_step(Descent &D, const DescArgs &a_in, int64_t *bsumF, int64_t *bsumU, const msp_fgt_params *q,
                uint64_t seed, int step, hipStream_t s) {
    msp_tree *t = D.t;
    DescArgs a = a_in;
    a.step = step;
    const unsigned gF = capped_grid(a.fcap, kBlock, 2048), gU = capped_grid(a.ucap, kBlock, 2048),
                   gW = capped_grid(a.ucap, 4, 8192), gT = capped_grid(a.tcap, 4, 8192);
    hipLaunchKernelGGL(k_pairs_count, dim3(gF), dim3(kBlock), 0, s, a);
    MSP_CHECK_LAUNCH();
    MSP_TRY(scan_cols<2>(a.ctr + C_M, a.fcap, a.pcnt, bsumF, a.ctr + C_NU, s));
    hipLaunchKernelGGL(k_clamp_pairs, dim3(1), dim3(64), 0, s, a.ctr, a.ucap, a.rcap);
    MSP_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_pairs_fill, dim3(gF), dim3(kBlock), 0, s, a);
    MSP_CHECK_LAUNCH();
    MSP_TRY(scan_cols<4>(a.ctr + C_NU, a.ucap, a.ucnt, bsumU, a.ctr + C_NQ, s));
    hipLaunchKernelGGL(k_clamp_units, dim3(1), dim3(64), 0, s, a.ctr, a.qcap, a.tcap, a.dvcap, a.crcap);
    MSP_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_units_fill, dim3(gW), dim3(256), 0, s, a);
    MSP_CHECK_LAUNCH();
    if (a.qcap > 0)
        MSP_TRY(partner_query_raw(t, q, a.qt, a.qn, a.qcap, t->desc_probs.as<float>(), t->desc_raw.as<double>(),
                                  a.qs, s, a.ctr + C_NQ));
    {
        PhaseScope ph(&t->timing, PH_DESC_CHOOSE, s);
        if (D.box_level >= 0) {
            hipLaunchKernelGGL(k_box_partials, dim3(capped_grid(D.box.nbox, 4, 8192)), dim3(256), 0, s, D.box,
                               t->keys.as<uint64_t>(), step);
            MSP_CHECK_LAUNCH();
        }
        hipLaunchKernelGGL(k_desc_direct, dim3(gT), dim3(256), 0, s, a.ctr + C_NT, a.ti, a.tcf, a.tnc, a.toff,
                           t->ps.as<float4>(), 1.0 / ((double)q->sigma * q->sigma), t->desc_dv.as<double>());
        MSP_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_desc_choose, dim3(gW), dim3(256), 0, s, a.ctr + C_NU, a.units, t->desc_raw.as<double>(),
                           a.qa, t->desc_dv.as<double>(), a.toff, a.ta, a.crng, D.box, seed, step, a.choice);
        MSP_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_next, dim3(gU), dim3(kBlock), 0, s, a);
    MSP_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_step_end, dim3(1), dim3(64), 0, s, a.ctr);
    MSP_CHECK_LAUNCH();
    return MSP_OK;
}

int check_items(const Descent &D, const int64_t *X, int64_t m) {
    for (int64_t k = 0; k < m; ++k)
        if (X[k] >= D.nn || X[k] < -D.n) return fail(MSP_EINVAL, "frontier item %lld out of range", (long long)X[k]);
    return MSP_OK;
}

}  // namespace

int descent_step(msp_tree *t, const float *w, const float *a, const msp_fgt_params *prm, uint64_t seed,
                 int32_t step, const int64_t *S_in, const int64_t *T_in, int64_t m, int64_t *S_out,
                 int64_t *T_out, int64_t cap, int64_t *m_out, int32_t *req_axon, int32_t *req_dendrite,
                 int64_t req_cap, int64_t *n_req, hipStream_t s) {
    msp_fgt_params q = *prm;
    q.flags |= MSP_EXCLUDE_SELF;
    Descent D;
    MSP_TRY(desc_setup(D, t, w, a, &q, s));
    MSP_TRY(check_items(D, S_in, m));
    MSP_TRY(check_items(D, T_in, m));
    // capacities from the given pairs: a pair's units, queries, tasks and range
    // entries stay within its axon item's neurons, its terms within those times
    // the dendrite leaf's neurons
    Caps c{m > 0 ? m : 1, 0, 0, 0, 0, 0, m > 0 ? m : 1};
    for (int64_t k = 0; k < m; ++k) {
        const int64_t Si = S_in[k], Ti = T_in[k];
        const int64_t ns = Si >= 0 ? D.ncount[Si] : 1;
        const int64_t nu = Si >= 0 ? (D.nnchild[Si] > 0 ? D.nnchild[Si] : D.ncount[Si]) : 1;
        const int64_t tl = Ti >= 0 && D.nnchild[Ti] == 0 ? D.ncount[Ti] : 1;
        c.u += nu;
        c.q += ns;
        c.dv += ns * tl;
        c.cr += 2 * nu;
    }
    c.u = c.u > 0 ? c.u : 1;
    c.tk = c.q = c.q > 0 ? c.q : 1;
    c.dv = c.dv > 0 ? c.dv : 1;
    c.cr = c.cr > 0 ? c.cr : 1;
    DescArgs da;
    int64_t *bsumF = nullptr, *bsumU = nullptr;
    MSP_TRY(lists_for(D, c, da, &bsumF, &bsumU, nullptr, nullptr));
    hipLaunchKernelGGL(k_desc_init, dim3(1), dim3(64), 0, s, da.ctr, const_cast<int64_t *>(da.S),
                       const_cast<int64_t *>(da.T), (int64_t)0);
    MSP_CHECK_LAUNCH();
    if (m > 0) {
        MSP_HIP(hipMemcpyAsync(const_cast<int64_t *>(da.S), S_in, (size_t)m * 8, hipMemcpyHostToDevice, s));
        MSP_HIP(hipMemcpyAsync(const_cast<int64_t *>(da.T), T_in, (size_t)m * 8, hipMemcpyHostToDevice, s));
    }
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(64), 0, s, da.ctr + C_M, m);
    MSP_CHECK_LAUNCH();
    MSP_TRY(launch_step(D, da, bsumF, bsumU, &q, seed, step, s));
    int64_t ctr[C_COUNT];
    MSP_HIP(hipMemcpyAsync(ctr, da.ctr, sizeof(ctr), hipMemcpyDeviceToHost, s));
    MSP_HIP(hipStreamSynchronize(s));
    if (ctr[C_ERR]) return fail(MSP_ENOSPC, "descent step tables overflowed");
    const int64_t nu = ctr[C_NU], nr = ctr[C_SNR];
    std::vector<int64_t> S2((size_t)nu), T2((size_t)nu);
    std::vector<int32_t> ra((size_t)nr), rd((size_t)nr);
    if (nu > 0) {
        MSP_HIP(hipMemcpy(S2.data(), da.S2, (size_t)nu * 8, hipMemcpyDeviceToHost));
        MSP_HIP(hipMemcpy(T2.data(), da.T2, (size_t)nu * 8, hipMemcpyDeviceToHost));
    }
    if (nr > 0) {
        MSP_HIP(hipMemcpy(ra.data(), da.req_a, (size_t)nr * 4, hipMemcpyDeviceToHost));
        MSP_HIP(hipMemcpy(rd.data(), da.req_d, (size_t)nr * 4, hipMemcpyDeviceToHost));
    }
    int64_t mo = 0;
    for (int64_t u = 0; u < nu; ++u)
        if (S2[u] != kNoItem) {
            if (mo < cap) {
                S_out[mo] = S2[u];
                T_out[mo] = T2[u];
            }
            ++mo;
        }
    *m_out = mo;
    *n_req = nr;
    if (mo > cap) return fail(MSP_ENOSPC, "next frontier has %lld pairs, capacity %lld", (long long)mo, (long long)cap);
    if (nr > req_cap) return fail(MSP_ENOSPC, "%lld requests, capacity %lld", (long long)nr, (long long)req_cap);
    std::copy(ra.begin(), ra.end(), req_axon);
    std::copy(rd.begin(), rd.end(), req_dendrite);
    return MSP_OK;
}

int partner_descent(msp_tree *t, const float *w, const float *a, const msp_fgt_params *prm, uint64_t seed,
                    int32_t *req_axon, int32_t *req_dendrite, uint8_t *accepted, int64_t *n_req,
                    int32_t *n_steps, hipStream_t s) {
    msp_fgt_params q = *prm;
    q.flags |= MSP_EXCLUDE_SELF;
    Descent D;
    MSP_TRY(desc_setup(D, t, w, a, &q, s));
    // the axon items of a frontier are disjoint and each holds an axon, so every
    // table of a step stays within the axon count (terms: times the largest leaf)
    const int64_t na1 = D.nax > 0 ? D.nax : 1;
    const Caps c{na1, na1, na1, na1, na1 * D.maxleaf, 2 * (D.n > 0 ? D.n : 1), D.n > 0 ? D.n : 1};
    DescArgs da;
    int64_t *bsumF = nullptr, *bsumU = nullptr;
    MSP_TRY(lists_for(D, c, da, &bsumF, &bsumU, req_axon, req_dendrite));
    hipLaunchKernelGGL(k_desc_init, dim3(1), dim3(64), 0, s, da.ctr, const_cast<int64_t *>(da.S),
                       const_cast<int64_t *>(da.T), (int64_t)(D.nn > 0 && D.nax > 0 ? 1 : 0));
    MSP_CHECK_LAUNCH();
    // every step takes at least one side one level down; neurons sit below the
    // deepest level, so 2 (depth + 2) steps empty the frontier.  The host stays at
    // most two steps ahead of the device and stops once a step has emptied the
    // frontier (the frontier size after each step is copied to page-locked memory).
    const int max_steps = 2 * (t->depth + 2) + 2;
    MSP_TRY(t->desc_stage.ensure((size_t)max_steps * 8));
    volatile int64_t *msize = static_cast<volatile int64_t *>(t->desc_stage.p);
    std::vector<hipEvent_t> ev((size_t)max_steps, nullptr);
    int rc = MSP_OK;
    int launched = 0;
    for (int step = 0; step < max_steps; ++step) {
        if (step >= 2) {
            if (hipEventSynchronize(ev[step - 2]) != hipSuccess) {
                rc = fail(MSP_EHIP, "waiting for descent step %d", step - 2);
                break;
            }
            if (msize[step - 2] == 0) break;
        }
        if (hipEventCreateWithFlags(&ev[step], hipEventDisableTiming) != hipSuccess) {
            rc = fail(MSP_EHIP, "hipEventCreateWithFlags");
            break;
        }
        DescArgs sa = da;   // frontier in and out alternate between the two arrays
        if (step & 1) {
            sa.S = da.S2;
            sa.T = da.T2;
            sa.S2 = const_cast<int64_t *>(da.S);
            sa.T2 = const_cast<int64_t *>(da.T);
        }
        rc = launch_step(D, sa, bsumF, bsumU, &q, seed, step, s);
        if (rc != MSP_OK) break;
        ++launched;
        if (hipMemcpyAsync(const_cast<int64_t *>(msize + step), da.ctr + C_M, 8, hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipEventRecord(ev[step], s) != hipSuccess) {
            rc = fail(MSP_EHIP, "recording descent step %d", step);
            break;
        }
    }
    int64_t ctr[C_COUNT] = {};
    if (rc == MSP_OK) {
        if (hipMemcpyAsync(ctr, da.ctr, sizeof(ctr), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            rc = fail(MSP_EHIP, "reading the descent counters");
    }
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    MSP_TRY(rc);
    if (ctr[C_ERR]) return fail(MSP_ENOSPC, "descent tables overflowed");
    if (ctr[C_M] > 0) return fail(MSP_EINVAL, "descent did not finish in %d steps", launched);
    const int64_t nr = ctr[C_NR];
    *n_req = nr;
    if (n_steps) *n_steps = (int32_t)ctr[C_STEPS];
    if (nr == 0) return MSP_OK;
    // acceptance at the dendrites (input indices): counts, offsets, buckets, ranks
    DevBuf cnt, off, fill, bucket;
    MSP_TRY(cnt.ensure((size_t)D.n * 4));
    MSP_TRY(off.ensure((size_t)D.n * 4));
    MSP_TRY(fill.ensure((size_t)D.n * 4));
    MSP_TRY(bucket.ensure((size_t)nr * 4));
    hipLaunchKernelGGL(k_desc_zero, dim3(grid_for(D.n, kBlock)), dim3(kBlock), 0, s, D.n, cnt.as<int32_t>(),
                       fill.as<int32_t>());
    MSP_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_req_count, dim3(grid_for(nr, kBlock)), dim3(kBlock), 0, s, nr, req_dendrite,
                       cnt.as<int32_t>());
    MSP_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_req_scan, dim3(1), dim3(1024), 0, s, D.n, cnt.as<int32_t>(), off.as<int32_t>());
    MSP_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_req_fill, dim3(grid_for(nr, kBlock)), dim3(kBlock), 0, s, nr, req_dendrite,
                       off.as<int32_t>(), fill.as<int32_t>(), bucket.as<int32_t>());
    MSP_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_req_rank, dim3(grid_for(nr, kBlock)), dim3(kBlock), 0, s, nr, req_axon, req_dendrite,
                       off.as<int32_t>(), cnt.as<int32_t>(), bucket.as<int32_t>(), w, seed, accepted);
    MSP_CHECK_LAUNCH();
    MSP_HIP(hipStreamSynchronize(s));   // the scratch above is released on return
    return MSP_OK;
}

}  // namespace msp
