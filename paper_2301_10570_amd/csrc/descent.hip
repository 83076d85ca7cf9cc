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
// Evaluation.  Att(S_c, C) for the children C of an inner node T is the sum over
// the axon neurons i of S_c of a_i times the per-octant attraction of i to T's
// children, which the partner queries compute (node moments where accurate,
// direct sums otherwise: the accuracy contract of the partner probabilities).
// For a leaf node T (children = neurons) and for a single dendrite neuron T the
// terms are summed directly in FP64.  The frontier and the lists of a step are
// built on the host (one synchronisation per step); the sums, the choices and
// the acceptance run in kernels.
#include "internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace msp {
namespace {

constexpr int kBlock = 256;
constexpr int64_t kNoItem = INT64_MIN;
enum UnitKind : int32_t { K_OCT = 0, K_LEAF = 1, K_SRC = 2 };

// One choice: candidates' values from queries [r0, r1) (K_OCT, 8 octants), from
// direct tasks [r0, r1) against ncand neurons each (K_LEAF), or from per-candidate
// task ranges crng[c0 + c] (K_SRC).
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
                                                     const float *ta, const int64_t *crng, uint64_t seed,
                                                     int step, int32_t *out) {
    __shared__ double sv[4][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t u = (int64_t)blockIdx.x * 4 + wave;
    if (u >= nunit) return;
    const UnitDesc U = units[u];
    if (U.kind == K_OCT) {
        // octant values: the lanes split the queries, then a butterfly sum (every lane
        // ends with all eight values)
        double acc[8];
#pragma unroll
        for (int d = 0; d < 8; ++d) acc[d] = 0.0;
        for (int64_t q = U.r0 + lane; q < U.r1; q += 64) {
            const double aq = (double)qa[q];
#pragma unroll
            for (int d = 0; d < 8; ++d) acc[d] = fma(aq, raw[q * 8 + d], acc[d]);
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

// Host side of one descent: tree topology and the sorted weights.
struct DescentCtx {
    msp_tree *t = nullptr;
    int64_t n = 0, nn = 0;
    std::vector<int32_t> perm, iperm, nfirst, ncount, nfchild, nnchild, ndigit;
    std::vector<float> as, ws;          // a and w in key order
    std::vector<int64_t> axc;           // prefix counts of neurons with a > 0, key order
    bool has_axons(int64_t first, int64_t count) const { return axc[first + count] - axc[first] > 0; }
    int64_t pos_of(int64_t item) const { return iperm[-item - 1]; }
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
    std::vector<float> ain, win;
    MSP_TRY(to_host(ain, a, c.n));
    MSP_TRY(to_host(win, w, c.n));
    c.as.resize((size_t)c.n);
    c.ws.resize((size_t)c.n);
    c.axc.assign((size_t)c.n + 1, 0);
    for (int64_t p = 0; p < c.n; ++p) {
        c.as[p] = ain[c.perm[p]];
        c.ws[p] = win[c.perm[p]];
        c.axc[p + 1] = c.axc[p] + (c.as[p] > 0.f ? 1 : 0);
    }
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
    DevBuf &lists, &raw, &probs, &dv, &choice;
    HostBuf &stage;
    const int32_t *qt = nullptr, *qs = nullptr, *qn = nullptr, *ti = nullptr, *tcf = nullptr, *tnc = nullptr;
    const float *qa = nullptr, *ta = nullptr;
    const int64_t *toff = nullptr, *crng = nullptr;
    const UnitDesc *units = nullptr;
};

// The host lists of one step, kept across steps so that their storage is reused.
struct StepHost {
    std::vector<int32_t> qt, qs, qn, ti, tcf, tnc;
    std::vector<float> qa, ta;
    std::vector<int64_t> toff, crng;
    std::vector<UnitDesc> units;
    std::vector<int64_t> keep, cand_off, cand;
    std::vector<int32_t> side, pick;
    std::vector<int64_t> chS;
    void clear() {
        qt.clear(); qs.clear(); qn.clear(); ti.clear(); tcf.clear(); tnc.clear();
        qa.clear(); ta.clear(); toff.clear(); crng.clear(); units.clear();
        keep.clear(); cand_off.assign(1, 0); cand.clear(); side.clear(); chS.clear();
    }
};

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// all lists of the step in one host-to-device copy
int upload_lists(StepBufs &B, StepHost &H, hipStream_t s) {
    struct Item { const void *src; size_t bytes; size_t off; };
    Item it[11] = {{H.qt.data(), H.qt.size() * 4, 0}, {H.qs.data(), H.qs.size() * 4, 0},
                   {H.qn.data(), H.qn.size() * 4, 0}, {H.qa.data(), H.qa.size() * 4, 0},
                   {H.ti.data(), H.ti.size() * 4, 0}, {H.tcf.data(), H.tcf.size() * 4, 0},
                   {H.tnc.data(), H.tnc.size() * 4, 0}, {H.toff.data(), H.toff.size() * 8, 0},
                   {H.ta.data(), H.ta.size() * 4, 0}, {H.crng.data(), H.crng.size() * 8, 0},
                   {H.units.data(), H.units.size() * sizeof(UnitDesc), 0}};
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
            for (int64_t ch : chS) {
                int64_t f, m;
                range_of(c, ch, f, m);
                if (!c.has_axons(f, m)) continue;
                unit_over_T(ch, Ti);
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
    if (nq > 0)
        MSP_TRY(partner_query_raw(c.t, prm, B.qt, B.qn, nq, B.probs.as<float>(), B.raw.as<double>(), B.qs, s));
    if (ntask > 0) {
        hipLaunchKernelGGL(k_desc_direct, dim3(grid_for(ntask, 4)), dim3(256), 0, s, ntask, B.ti, B.tcf, B.tnc,
                           B.toff, c.t->ps.as<float4>(),
                           1.0 / ((double)prm->sigma * prm->sigma), B.dv.as<double>());
        MSP_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_desc_choose, dim3(grid_for(nu, 4)), dim3(256), 0, s, nu, B.units, B.raw.as<double>(),
                       B.qa, B.dv.as<double>(), B.toff, B.ta, B.crng, seed, step, B.choice.as<int32_t>());
    MSP_CHECK_LAUNCH();
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
    StepBufs B{t->desc_lists, t->desc_raw, t->desc_probs, t->desc_dv, t->desc_choice, t->desc_stage};
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
    StepBufs B{t->desc_lists, t->desc_raw, t->desc_probs, t->desc_dv, t->desc_choice, t->desc_stage};
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
