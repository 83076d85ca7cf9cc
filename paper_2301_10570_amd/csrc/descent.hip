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
// FP64.  The frontier and the lists of a step are built on the host (one
// synchronisation per step); the sums, the choices and the acceptance run in
// kernels.
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
// is summed directly (FP64 offsets and sums, each exponential to about 1e-7), or,
// when both boxes lie at or below the box level,
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
constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// One choice: candidates' values from queries [r0, r1) (K_OCT, 8 octants), from
// direct tasks [r0, r1) against ncand neurons each (K_LEAF), from per-candidate
// task ranges crng[c0 + c] (K_SRC), or from the box pairs [r0, r1) binned by the
// octant of the dendrite box under node c0 (K_BOX, 8 octants).
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

// direct terms w_j K(t_i, s_j) of one axon neuron i (key order) against the
// neurons cf .. cf + nc - 1 (key order; the pair j = i is 0); one wavefront per task
__global__ void __launch_bounds__(256) k_desc_direct(int64_t ntask, const int32_t *ti, const int32_t *tcf,
                                                     const int32_t *tnc, const int64_t *toff, const float4 *ps,
                                                     double inv_s2, double *dv) {
    const int lane = threadIdx.x & 63;
    const int64_t task = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (task >= ntask) return;
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

// one wavefront per unit.  K_OCT: the lanes split the queries; otherwise candidate
// values 64 at a time (lane per candidate), total and running sums in candidate
// order by lane 0
__global__ void __launch_bounds__(256) k_desc_choose(int64_t nunit, const UnitDesc *units, const double *raw,
                                                     const float *qa, const double *dv, const int64_t *toff,
                                                     const float *ta, const int64_t *crng, const double *box_att,
                                                     uint64_t seed, int step, int32_t *out) {
    __shared__ double sv[4][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t u = (int64_t)blockIdx.x * 4 + wave;
    if (u >= nunit) return;
    const UnitDesc U = units[u];
    if (U.kind == K_OCT || U.kind == K_BOX) {
        double acc[8];
#pragma unroll
        for (int d = 0; d < 8; ++d) acc[d] = 0.0;
        if (U.kind == K_BOX) {   // summed by k_box_units
#pragma unroll
            for (int d = 0; d < 8; ++d) acc[d] = box_att[u * 8 + d];
        } else {
            // octant values: the lanes split the queries, then a butterfly sum (every
            // lane ends with all eight values)
            for (int64_t q = U.r0 + lane; q < U.r1; q += 64) {
                const double aq = (double)qa[q];
#pragma unroll
                for (int d = 0; d < 8; ++d) acc[d] = fma(aq, raw[q * 8 + d], acc[d]);
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1)
#pragma unroll
                for (int d = 0; d < 8; ++d) acc[d] += __shfl_xor(acc[d], o, 64);
        }
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
        return;
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

// exp(-x) for x >= 0 over the float64 range: 2^-a, a = x log2(e), as the
// hardware exp2 of the fraction of a times 2^-floor(a) (relative error about 1e-7)
__device__ inline double exp_neg2(double x) {
    const double a = x * 1.4426950408889634;
    const double n = floor(a);
    return ldexp((double)__builtin_amdgcn_exp2f(-(float)(a - n)), -(int)fmin(n, 2000.0));
}

__device__ inline double wave_sum_d(double x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// One wavefront per box pair: Att(s, c) by the expansions (the double series,
// contracted one axis at a time in LDS) or directly (offsets and sums in FP64,
// each exponential to about 1e-7).
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
        const int32_t fc = g.nfirst[vc], nc = g.ncount[vc];
        const double k2 = g.inv_sigma * g.inv_sigma;
        double part = 0.0;
        for (int32_t i = 0; i < ns; ++i) {
            const float ai = g.akey[fs + i];
            if (ai == 0.f) continue;
            const float4 ti = g.ps[fs + i];
            double pi = 0.0;
            for (int32_t j = lane; j < nc; j += 64) {
                const float4 sj = g.ps[fc + j];
                if (sj.w == 0.f || fc + j == fs + i) continue;
                const double ex = (double)ti.x - sj.x, ey = (double)ti.y - sj.y, ez = (double)ti.z - sj.z;
                pi += (double)sj.w * exp_neg2((ex * ex + ey * ey + ez * ez) * k2);
            }
            part += (double)ai * pi;
        }
        val = wave_sum_d(part);
    }
    if (lane == 0) g.F[k] = val;
}

// One block per K_BOX unit (list bu): the pairs of the axon node's boxes binned by
// the octant of the dendrite box under node T (pairs outside T dropped), summed
// per thread in pair order and then over the threads in a fixed order.
__global__ void __launch_bounds__(256) k_box_units(int64_t nbu, const int32_t *bu, const UnitDesc *units,
                                                   BoxArgs g, double *att) {
    __shared__ double part[4][8];
    const int64_t e = blockIdx.x;
    if (e >= nbu) return;
    const int32_t u = bu[e];
    const UnitDesc U = units[u];
    const int32_t T = (int32_t)U.c0;
    const int32_t tf = g.nfirst[T], tc = g.ncount[T], lt = g.nlevel[T];
    double acc[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) acc[d] = 0.0;
    for (int64_t k = U.r0 + threadIdx.x; k < U.r1; k += blockDim.x) {
        const int32_t v = g.box_node[g.pair_c[k]];
        const int32_t f = g.nfirst[v];
        if (f < tf || f >= tf + tc) continue;
        const int sh = g.nlevel[v] - lt - 1;
        const int d = (((g.nix[v] >> sh) & 1) << 2) | (((g.niy[v] >> sh) & 1) << 1) | ((g.niz[v] >> sh) & 1);
        const double x = g.F[k];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (q == d) acc[q] += x;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        const double x = wave_sum_d(acc[d]);
        if (lane == 0) part[wave][d] = x;
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        double x = 0.0;
        for (int w = 0; w < 4; ++w) x += part[w][threadIdx.x];
        att[(int64_t)u * 8 + threadIdx.x] = x;
    }
}

// The boxes of a descent and their pair lists (host side; the device arrays live
// in the tree's desc_box, desc_pairs, desc_boxmom and desc_akey).
struct BoxPlan {
    int level = -1;                     // the box level; -1: no box pairs in this descent
    std::vector<int32_t> node, first;   // per box in key order: node, first point
    std::vector<int64_t> pair_off;      // pairs of axon box s: pair_off[s] .. pair_off[s + 1]
    BoxArgs args{};
};

// Host side of one descent: tree topology and the sorted weights.
struct DescentCtx {
    msp_tree *t = nullptr;
    int64_t n = 0, nn = 0;
    std::vector<int32_t> perm, iperm, nfirst, ncount, nfchild, nnchild, ndigit, nlevel;
    std::vector<float> as, ws;          // a and w in key order
    std::vector<int64_t> axc, dnc;      // prefix counts of neurons with a > 0 / w > 0, key order
    BoxPlan box;
    bool has_axons(int64_t first, int64_t count) const { return axc[first + count] - axc[first] > 0; }
    int64_t pos_of(int64_t item) const { return iperm[-item - 1]; }
    // the boxes inside node X (X above the box level, or a box): [b0, b1)
    void box_range(int64_t X, int64_t &b0, int64_t &b1) const {
        const int32_t f = nfirst[X], e = nfirst[X] + ncount[X];
        b0 = std::lower_bound(box.first.begin(), box.first.end(), f) - box.first.begin();
        b1 = std::lower_bound(box.first.begin(), box.first.end(), e) - box.first.begin();
    }
};

template <class T>
int to_host(std::vector<T> &v, const void *dev, int64_t count) {
    v.resize((size_t)(count > 0 ? count : 0));
    if (count > 0) MSP_HIP(hipMemcpy(v.data(), dev, (size_t)count * sizeof(T), hipMemcpyDeviceToHost));
    return MSP_OK;
}

int ctx_init(DescentCtx &c, msp_tree *t, const float *w, const float *a, const msp_fgt_params *prm,
             hipStream_t s) {
    c.t = t;
    c.n = t->n;
    c.nn = t->n_nodes;
    MSP_TRY(partner_prepare(t, w, prm, s));   // staged w, node moments
    MSP_HIP(hipStreamSynchronize(s));
    MSP_TRY(to_host(c.perm, t->perm.p, c.n));
    c.iperm.resize((size_t)c.n);
    for (int64_t p = 0; p < c.n; ++p) c.iperm[c.perm[p]] = (int32_t)p;
    MSP_TRY(to_host(c.nfirst, t->nfirst.p, c.nn));
    MSP_TRY(to_host(c.ncount, t->ncount.p, c.nn));
    MSP_TRY(to_host(c.nfchild, t->nfchild.p, c.nn));
    MSP_TRY(to_host(c.nnchild, t->nnchild.p, c.nn));
    MSP_TRY(to_host(c.ndigit, t->ndigit.p, c.nn));
    MSP_TRY(to_host(c.nlevel, t->nlevel.p, c.nn));
    std::vector<float> ain, win;
    MSP_TRY(to_host(ain, a, c.n));
    MSP_TRY(to_host(win, w, c.n));
    c.as.resize((size_t)c.n);
    c.ws.resize((size_t)c.n);
    c.axc.assign((size_t)c.n + 1, 0);
    c.dnc.assign((size_t)c.n + 1, 0);
    for (int64_t p = 0; p < c.n; ++p) {
        c.as[p] = ain[c.perm[p]];
        c.ws[p] = win[c.perm[p]];
        c.axc[p + 1] = c.axc[p] + (c.as[p] > 0.f ? 1 : 0);
        c.dnc[p + 1] = c.dnc[p] + (c.ws[p] > 0.f ? 1 : 0);
    }
    return MSP_OK;
}

// The boxes, their pairs within the cutoff, the box moments and every pair's
// attraction, once per descent.  Leaves c.box.level at -1 (no box pairs) when p
// is beyond kBoxPMax, when no node lies above the box level, or, without a cutoff,
// when the axon boxes times the dendrite boxes exceed kBoxPairsNoCutoff.
int box_plan(DescentCtx &c, const msp_fgt_params *prm, hipStream_t s) {
    BoxPlan &B = c.box;
    B.level = -1;
    c.t->desc_box_level = -1;
    c.t->desc_nbox = c.t->desc_npair = 0;
    B.node.clear();
    B.first.clear();
    B.pair_off.clear();
    const int p = prm->p;
    if (p < 1 || p > kBoxPMax || c.nn == 0 || c.nnchild[0] == 0) return MSP_OK;
    const double rmax = rho_max_for_p(p), sigma = prm->sigma;
    int lm = kDepth;
    for (int l = 0; l <= kDepth; ++l)
        if (c.t->geo.side / std::ldexp(1.0, l + 1) / sigma <= rmax) {
            lm = l;
            break;
        }
    const int L = lm + 1;
    // boxes in key order: a walk from the root that stops at the first node at or
    // below L and at leaves
    std::vector<int32_t> node_box((size_t)c.nn, -1), stk{0};
    while (!stk.empty()) {
        const int32_t u = stk.back();
        stk.pop_back();
        if (c.nlevel[u] >= L || c.nnchild[u] == 0) {
            B.node.push_back(u);
            continue;
        }
        for (int32_t k = c.nnchild[u] - 1; k >= 0; --k) stk.push_back(c.nfchild[u] + k);
    }
    std::sort(B.node.begin(), B.node.end(), [&](int32_t x, int32_t y) { return c.nfirst[x] < c.nfirst[y]; });
    const int64_t nbox = (int64_t)B.node.size();
    std::vector<int32_t> na((size_t)nbox), nd((size_t)nbox);
    int64_t nab = 0, ndb = 0;
    B.first.resize((size_t)nbox);
    for (int64_t b = 0; b < nbox; ++b) {
        const int32_t v = B.node[b], f = c.nfirst[v], e = f + c.ncount[v];
        node_box[v] = (int32_t)b;
        B.first[b] = f;
        na[b] = (int32_t)(c.axc[e] - c.axc[f]);
        nd[b] = (int32_t)(c.dnc[e] - c.dnc[f]);
        nab += na[b] > 0;
        ndb += nd[b] > 0;
    }
    const bool unlimited = !(prm->cutoff_sigmas > 0.f);
    if (unlimited && (double)nab * (double)ndb > (double)kBoxPairsNoCutoff) return MSP_OK;
    // device tables: node -> box, then per box node, axons, dendrites, pair offsets, counts
    msp_tree *t = c.t;
    const size_t o_nb = 0, o_bn = align_up((size_t)c.nn * 4), o_na = o_bn + align_up((size_t)nbox * 4),
                 o_nd = o_na + align_up((size_t)nbox * 4), o_off = o_nd + align_up((size_t)nbox * 4),
                 o_cnt = o_off + align_up((size_t)(nbox + 1) * 8), tot = o_cnt + align_up((size_t)nbox * 8);
    MSP_TRY(t->desc_box.ensure(tot));
    char *db = t->desc_box.as<char>();
    MSP_HIP(hipMemcpyAsync(db + o_nb, node_box.data(), (size_t)c.nn * 4, hipMemcpyHostToDevice, s));
    MSP_HIP(hipMemcpyAsync(db + o_bn, B.node.data(), (size_t)nbox * 4, hipMemcpyHostToDevice, s));
    MSP_HIP(hipMemcpyAsync(db + o_na, na.data(), (size_t)nbox * 4, hipMemcpyHostToDevice, s));
    MSP_HIP(hipMemcpyAsync(db + o_nd, nd.data(), (size_t)nbox * 4, hipMemcpyHostToDevice, s));
    MSP_TRY(t->desc_akey.ensure((size_t)c.n * 4));
    MSP_HIP(hipMemcpyAsync(t->desc_akey.p, c.as.data(), (size_t)c.n * 4, hipMemcpyHostToDevice, s));
    BoxArgs &g = B.args;
    g = BoxArgs{};
    g.nbox = nbox;
    g.level = L;
    g.node_box = reinterpret_cast<const int32_t *>(db + o_nb);
    g.box_node = reinterpret_cast<const int32_t *>(db + o_bn);
    g.box_na = reinterpret_cast<const int32_t *>(db + o_na);
    g.box_nd = reinterpret_cast<const int32_t *>(db + o_nd);
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
    g.inv_sigma = 1.0 / sigma;
    g.cut = unlimited ? -1.0 : (double)prm->cutoff_sigmas * sigma;
    // pair counts, offsets on the host, pairs
    int64_t *dcnt = reinterpret_cast<int64_t *>(db + o_cnt);
    {
        PhaseScope ph(&t->timing, PH_DESC_BOXES, s);
        hipLaunchKernelGGL(k_box_lists, dim3(grid_for(nbox, kBlock)), dim3(kBlock), 0, s, g, dcnt);
        MSP_CHECK_LAUNCH();
    }
    std::vector<int64_t> cnt((size_t)nbox);
    MSP_HIP(hipMemcpyAsync(cnt.data(), dcnt, (size_t)nbox * 8, hipMemcpyDeviceToHost, s));
    MSP_HIP(hipStreamSynchronize(s));
    B.pair_off.assign((size_t)nbox + 1, 0);
    for (int64_t b = 0; b < nbox; ++b) B.pair_off[b + 1] = B.pair_off[b] + cnt[b];
    const int64_t npair = B.pair_off[nbox];
    MSP_HIP(hipMemcpyAsync(db + o_off, B.pair_off.data(), (size_t)(nbox + 1) * 8, hipMemcpyHostToDevice, s));
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
        hipLaunchKernelGGL(k_box_lists, dim3(grid_for(nbox, kBlock)), dim3(kBlock), 0, s, g, (int64_t *)nullptr);
        MSP_CHECK_LAUNCH();
    }
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
    B.level = L;
    t->desc_box_level = L;
    t->desc_nbox = nbox;
    t->desc_npair = npair;
    return MSP_OK;
}

// children of an item: nodes (octant order) or neurons (key order)
void children(const DescentCtx &c, int64_t item, std::vector<int64_t> &out) {
    out.clear();
    if (item < 0) return;
    const int32_t nc = c.nnchild[item];
    if (nc > 0) {
        const int32_t fc = c.nfchild[item];
        for (int32_t k = 0; k < nc; ++k) out.push_back(fc + k);
        std::sort(out.begin(), out.end(), [&](int64_t x, int64_t y) { return c.ndigit[x] < c.ndigit[y]; });
    } else {
        const int32_t f = c.nfirst[item], m = c.ncount[item];
        for (int32_t p = f; p < f + m; ++p) out.push_back(-(int64_t)c.perm[p] - 1);
    }
}

void range_of(const DescentCtx &c, int64_t item, int64_t &first, int64_t &count) {
    if (item >= 0) {
        first = c.nfirst[item];
        count = c.ncount[item];
    } else {
        first = c.pos_of(item);
        count = 1;
    }
}

// Device arrays of one step (the tree's, kept between descents): the host lists
// travel in one copy from a page-locked staging buffer into `lists` (each array
// at a 256-byte aligned offset).
struct StepBufs {
    DevBuf &lists, &raw, &probs, &dv, &choice, &boxatt;
    HostBuf &stage;
    const int32_t *qt = nullptr, *qs = nullptr, *qn = nullptr, *ti = nullptr, *tcf = nullptr, *tnc = nullptr;
    const float *qa = nullptr, *ta = nullptr;
    const int64_t *toff = nullptr, *crng = nullptr;
    const UnitDesc *units = nullptr;
    const int32_t *bu = nullptr;
};

// The host lists of one step, kept across steps so that their storage is reused.
struct StepHost {
    std::vector<int32_t> qt, qs, qn, ti, tcf, tnc;
    std::vector<float> qa, ta;
    std::vector<int64_t> toff, crng;
    std::vector<UnitDesc> units;
    std::vector<int32_t> bu;   // the K_BOX units
    std::vector<int64_t> keep, cand_off, cand;
    std::vector<int32_t> side, pick;
    std::vector<int64_t> chS;
    void clear() {
        qt.clear(); qs.clear(); qn.clear(); ti.clear(); tcf.clear(); tnc.clear();
        qa.clear(); ta.clear(); toff.clear(); crng.clear(); units.clear(); bu.clear();
        keep.clear(); cand_off.assign(1, 0); cand.clear(); side.clear(); chS.clear();
    }
};


// all lists of the step in one host-to-device copy
int upload_lists(StepBufs &B, StepHost &H, hipStream_t s) {
    struct Item { const void *src; size_t bytes; size_t off; };
    Item it[12] = {{H.qt.data(), H.qt.size() * 4, 0}, {H.qs.data(), H.qs.size() * 4, 0},
                   {H.qn.data(), H.qn.size() * 4, 0}, {H.qa.data(), H.qa.size() * 4, 0},
                   {H.ti.data(), H.ti.size() * 4, 0}, {H.tcf.data(), H.tcf.size() * 4, 0},
                   {H.tnc.data(), H.tnc.size() * 4, 0}, {H.toff.data(), H.toff.size() * 8, 0},
                   {H.ta.data(), H.ta.size() * 4, 0}, {H.crng.data(), H.crng.size() * 8, 0},
                   {H.units.data(), H.units.size() * sizeof(UnitDesc), 0}, {H.bu.data(), H.bu.size() * 4, 0}};
    size_t total = 0;
    for (Item &x : it) {
        x.off = total;
        total += align_up(x.bytes > 0 ? x.bytes : 1);
    }
    MSP_TRY(B.stage.ensure(total));
    MSP_TRY(B.lists.ensure(total));
    char *h = static_cast<char *>(B.stage.p);
    for (const Item &x : it)
        if (x.bytes) std::memcpy(h + x.off, x.src, x.bytes);
    MSP_HIP(hipMemcpyAsync(B.lists.p, B.stage.p, total, hipMemcpyHostToDevice, s));
    const char *d = B.lists.as<char>();
    B.qt = reinterpret_cast<const int32_t *>(d + it[0].off);
    B.qs = reinterpret_cast<const int32_t *>(d + it[1].off);
    B.qn = reinterpret_cast<const int32_t *>(d + it[2].off);
    B.qa = reinterpret_cast<const float *>(d + it[3].off);
    B.ti = reinterpret_cast<const int32_t *>(d + it[4].off);
    B.tcf = reinterpret_cast<const int32_t *>(d + it[5].off);
    B.tnc = reinterpret_cast<const int32_t *>(d + it[6].off);
    B.toff = reinterpret_cast<const int64_t *>(d + it[7].off);
    B.ta = reinterpret_cast<const float *>(d + it[8].off);
    B.crng = reinterpret_cast<const int64_t *>(d + it[9].off);
    B.units = reinterpret_cast<const UnitDesc *>(d + it[10].off);
    B.bu = reinterpret_cast<const int32_t *>(d + it[11].off);
    return MSP_OK;
}

// one step on the host frontier (pairs S[k], T[k]) -> next frontier and requests
int step_once(DescentCtx &c, StepBufs &B, StepHost &H, const msp_fgt_params *prm, uint64_t seed, int step,
              const std::vector<int64_t> &S, const std::vector<int64_t> &T, std::vector<int64_t> &S2,
              std::vector<int64_t> &T2, std::vector<int32_t> &ra, std::vector<int32_t> &rd, hipStream_t s) {
    S2.clear();
    T2.clear();
    H.clear();
    auto &qt = H.qt, &qs = H.qs, &qn = H.qn, &ti = H.ti, &tcf = H.tcf, &tnc = H.tnc;
    auto &qa = H.qa, &ta = H.ta;
    auto &toff = H.toff, &crng = H.crng;
    auto &units = H.units;
    // per unit: the other item of the next pair and the candidate items
    auto &keep = H.keep, &cand_off = H.cand_off, &cand = H.cand;
    auto &side = H.side;   // 0: next pair (keep, cand); 1: (cand, keep)
    int64_t dvn = 0;
    auto &chS = H.chS;
    auto add_task = [&](int64_t p_axon, int64_t cf, int64_t nc) {
        ti.push_back((int32_t)p_axon);
        tcf.push_back((int32_t)cf);
        tnc.push_back((int32_t)nc);
        toff.push_back(dvn);
        ta.push_back(c.as[p_axon]);
        dvn += nc;
    };
    // a unit choosing a child of node T for the axons of item X (neuron or node)
    auto unit_over_T = [&](int64_t X, int64_t Tn) {
        int64_t xf, xc;
        range_of(c, X, xf, xc);
        UnitDesc U{X, 0, 0, 0, K_OCT, 8};
        if (c.nnchild[Tn] > 0) {
            U.r0 = (int64_t)qt.size();
            for (int64_t p = xf; p < xf + xc; ++p)
                if (c.as[p] > 0.f) {
                    qt.push_back(c.perm[p]);
                    qs.push_back((int32_t)p);
                    qn.push_back((int32_t)Tn);
                    qa.push_back(c.as[p]);
                }
            U.r1 = (int64_t)qt.size();
            // octant d -> child node (absent octants carry no value and are never chosen)
            for (int d = 0; d < 8; ++d) cand.push_back(kNoItem);
            const int32_t fc = c.nfchild[Tn], nc = c.nnchild[Tn];
            const size_t base = cand.size() - 8;
            for (int32_t k = 0; k < nc; ++k) cand[base + c.ndigit[fc + k]] = fc + k;
        } else {
            const int64_t tf = c.nfirst[Tn], tc = c.ncount[Tn];
            U.kind = K_LEAF;
            U.ncand = (int32_t)tc;
            U.r0 = (int64_t)ti.size();
            for (int64_t p = xf; p < xf + xc; ++p)
                if (c.as[p] > 0.f) add_task(p, tf, tc);
            U.r1 = (int64_t)ti.size();
            for (int64_t p = tf; p < tf + tc; ++p) cand.push_back(-(int64_t)c.perm[p] - 1);
        }
        units.push_back(U);
        cand_off.push_back((int64_t)cand.size());
        keep.push_back(X);
        side.push_back(0);
    };
    // a unit choosing a child of node T for the axon node X from the box pairs
    // (X and T above the box level)
    auto unit_box = [&](int64_t X, int64_t Tn) {
        int64_t b0, b1;
        c.box_range(X, b0, b1);
        UnitDesc U{X, c.box.pair_off[b0], c.box.pair_off[b1], Tn, K_BOX, 8};
        H.bu.push_back((int32_t)units.size());
        for (int d = 0; d < 8; ++d) cand.push_back(kNoItem);
        const int32_t fc = c.nfchild[Tn], nc = c.nnchild[Tn];
        const size_t base = cand.size() - 8;
        for (int32_t k = 0; k < nc; ++k) cand[base + c.ndigit[fc + k]] = fc + k;
        units.push_back(U);
        cand_off.push_back((int64_t)cand.size());
        keep.push_back(X);
        side.push_back(0);
    };
    for (size_t k = 0; k < S.size(); ++k) {
        const int64_t Si = S[k], Ti = T[k];
        if (Si < 0 && Ti < 0) {
            ra.push_back((int32_t)(-Si - 1));
            rd.push_back((int32_t)(-Ti - 1));
        } else if (Si < 0) {
            unit_over_T(Si, Ti);
        } else if (Ti < 0) {
            // choose the child of S whose axons attract most to the neuron T
            children(c, Si, chS);
            const int64_t pt = c.pos_of(Ti);
            UnitDesc U{Si, 0, 0, (int64_t)crng.size() / 2, K_SRC, (int32_t)chS.size()};
            for (int64_t ch : chS) {
                int64_t f, m;
                range_of(c, ch, f, m);
                crng.push_back((int64_t)ti.size());
                for (int64_t p = f; p < f + m; ++p)
                    if (c.as[p] > 0.f) add_task(p, pt, 1);
                crng.push_back((int64_t)ti.size());
                cand.push_back(ch);
            }
            units.push_back(U);
            cand_off.push_back((int64_t)cand.size());
            keep.push_back(Ti);
            side.push_back(1);
        } else {
            children(c, Si, chS);
            // both above the box level, both with child nodes: box pairs
            const bool boxes = c.box.level >= 0 && c.nnchild[Si] > 0 && c.nnchild[Ti] > 0 &&
                               c.nlevel[Si] < c.box.level && c.nlevel[Ti] < c.box.level;
            for (int64_t ch : chS) {
                int64_t f, m;
                range_of(c, ch, f, m);
                if (!c.has_axons(f, m)) continue;
                if (boxes) unit_box(ch, Ti);
                else unit_over_T(ch, Ti);
            }
        }
    }
    const int64_t nq = (int64_t)qt.size(), ntask = (int64_t)ti.size(), nu = (int64_t)units.size();
    if (nu == 0) return MSP_OK;
    MSP_TRY(upload_lists(B, H, s));
    MSP_TRY(B.raw.ensure((size_t)(nq > 0 ? nq : 1) * 8 * sizeof(double)));
    MSP_TRY(B.probs.ensure((size_t)(nq > 0 ? nq : 1) * 8 * sizeof(float)));
    MSP_TRY(B.dv.ensure((size_t)(dvn > 0 ? dvn : 1) * sizeof(double)));
    MSP_TRY(B.choice.ensure((size_t)nu * sizeof(int32_t)));
    const int64_t nbu = (int64_t)H.bu.size();
    MSP_TRY(B.boxatt.ensure((size_t)(nbu > 0 ? nu : 1) * 8 * sizeof(double)));
    if (nq > 0)
        MSP_TRY(partner_query_raw(c.t, prm, B.qt, B.qn, nq, B.probs.as<float>(), B.raw.as<double>(), B.qs, s));
    {
    PhaseScope ph(&c.t->timing, PH_DESC_CHOOSE, s);
    if (ntask > 0) {
        hipLaunchKernelGGL(k_desc_direct, dim3(grid_for(ntask, 4)), dim3(256), 0, s, ntask, B.ti, B.tcf, B.tnc,
                           B.toff, c.t->ps.as<float4>(),
                           1.0 / ((double)prm->sigma * prm->sigma), B.dv.as<double>());
        MSP_CHECK_LAUNCH();
    }
    if (nbu > 0) {
        hipLaunchKernelGGL(k_box_units, dim3((unsigned)nbu), dim3(256), 0, s, nbu, B.bu, B.units, c.box.args,
                           B.boxatt.as<double>());
        MSP_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_desc_choose, dim3(grid_for(nu, 4)), dim3(256), 0, s, nu, B.units, B.raw.as<double>(),
                       B.qa, B.dv.as<double>(), B.toff, B.ta, B.crng, B.boxatt.as<double>(), seed, step,
                       B.choice.as<int32_t>());
    MSP_CHECK_LAUNCH();
    }
    auto &pick = H.pick;
    pick.resize((size_t)nu);
    MSP_HIP(hipMemcpyAsync(pick.data(), B.choice.p, (size_t)nu * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MSP_HIP(hipStreamSynchronize(s));
    for (int64_t u = 0; u < nu; ++u) {
        const int32_t k = pick[u];
        if (k < 0) continue;
        const int64_t nxt = cand[cand_off[u] + k];
        if (nxt == kNoItem) return fail(MSP_EINVAL, "descent chose an absent octant");
        if (side[u] == 0) {
            S2.push_back(keep[u]);
            T2.push_back(nxt);
        } else {
            S2.push_back(nxt);
            T2.push_back(keep[u]);
        }
    }
    return MSP_OK;
}

int check_items(const DescentCtx &c, const int64_t *X, int64_t m) {
    for (int64_t k = 0; k < m; ++k)
        if (X[k] >= c.nn || X[k] < -c.n) return fail(MSP_EINVAL, "frontier item %lld out of range", (long long)X[k]);
    return MSP_OK;
}

}  // namespace

int descent_step(msp_tree *t, const float *w, const float *a, const msp_fgt_params *prm, uint64_t seed,
                 int32_t step, const int64_t *S_in, const int64_t *T_in, int64_t m, int64_t *S_out,
                 int64_t *T_out, int64_t cap, int64_t *m_out, int32_t *req_axon, int32_t *req_dendrite,
                 int64_t req_cap, int64_t *n_req, hipStream_t s) {
    msp_fgt_params q = *prm;
    q.flags |= MSP_EXCLUDE_SELF;
    DescentCtx c;
    MSP_TRY(ctx_init(c, t, w, a, &q, s));
    MSP_TRY(check_items(c, S_in, m));
    MSP_TRY(check_items(c, T_in, m));
    MSP_TRY(box_plan(c, &q, s));
    StepBufs B{t->desc_lists, t->desc_raw, t->desc_probs, t->desc_dv, t->desc_choice, t->desc_boxatt, t->desc_stage};
    StepHost H;
    std::vector<int64_t> S(S_in, S_in + m), T(T_in, T_in + m), S2, T2;
    std::vector<int32_t> ra, rd;
    MSP_TRY(step_once(c, B, H, &q, seed, step, S, T, S2, T2, ra, rd, s));
    *m_out = (int64_t)S2.size();
    *n_req = (int64_t)ra.size();
    if ((int64_t)S2.size() > cap) return fail(MSP_ENOSPC, "next frontier has %lld pairs, capacity %lld",
                                              (long long)S2.size(), (long long)cap);
    if ((int64_t)ra.size() > req_cap) return fail(MSP_ENOSPC, "%lld requests, capacity %lld",
                                                  (long long)ra.size(), (long long)req_cap);
    std::copy(S2.begin(), S2.end(), S_out);
    std::copy(T2.begin(), T2.end(), T_out);
    std::copy(ra.begin(), ra.end(), req_axon);
    std::copy(rd.begin(), rd.end(), req_dendrite);
    return MSP_OK;
}

int partner_descent(msp_tree *t, const float *w, const float *a, const msp_fgt_params *prm, uint64_t seed,
                    int32_t *req_axon, int32_t *req_dendrite, uint8_t *accepted, int64_t *n_req,
                    int32_t *n_steps, hipStream_t s) {
    msp_fgt_params q = *prm;
    q.flags |= MSP_EXCLUDE_SELF;
    DescentCtx c;
    MSP_TRY(ctx_init(c, t, w, a, &q, s));
    MSP_TRY(box_plan(c, &q, s));
    StepBufs B{t->desc_lists, t->desc_raw, t->desc_probs, t->desc_dv, t->desc_choice, t->desc_boxatt, t->desc_stage};
    StepHost H;
    std::vector<int64_t> S, T, S2, T2;
    std::vector<int32_t> ra, rd;
    if (c.nn > 0 && c.axc[c.n] > 0) {
        S.push_back(0);
        T.push_back(0);
    }
    // every step takes at least one side one level down; neurons sit below the
    // deepest level, so 2 (depth + 2) steps empty the frontier
    const int max_steps = 2 * (t->depth + 2) + 2;
    int step = 0;
    for (; step < max_steps && !S.empty(); ++step) {
        MSP_TRY(step_once(c, B, H, &q, seed, step, S, T, S2, T2, ra, rd, s));
        S.swap(S2);
        T.swap(T2);
    }
    if (!S.empty()) return fail(MSP_EINVAL, "descent did not finish in %d steps", max_steps);
    const int64_t nr = (int64_t)ra.size();
    *n_req = nr;
    if (n_steps) *n_steps = step;
    if (nr == 0) return MSP_OK;
    MSP_HIP(hipMemcpyAsync(req_axon, ra.data(), (size_t)nr * 4, hipMemcpyHostToDevice, s));
    MSP_HIP(hipMemcpyAsync(req_dendrite, rd.data(), (size_t)nr * 4, hipMemcpyHostToDevice, s));
    // acceptance at the dendrites (input indices): counts, offsets, buckets, ranks
    DevBuf cnt, off, fill, bucket;
    MSP_TRY(cnt.ensure((size_t)c.n * 4));
    MSP_TRY(off.ensure((size_t)c.n * 4));
    MSP_TRY(fill.ensure((size_t)c.n * 4));
    MSP_TRY(bucket.ensure((size_t)nr * 4));
    hipLaunchKernelGGL(k_desc_zero, dim3(grid_for(c.n, kBlock)), dim3(kBlock), 0, s, c.n, cnt.as<int32_t>(),
                       fill.as<int32_t>());
    MSP_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_req_count, dim3(grid_for(nr, kBlock)), dim3(kBlock), 0, s, nr, req_dendrite,
                       cnt.as<int32_t>());
    MSP_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_req_scan, dim3(1), dim3(1024), 0, s, c.n, cnt.as<int32_t>(), off.as<int32_t>());
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
