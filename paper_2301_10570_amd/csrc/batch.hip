// Many independent populations in one batch.
//
// Every population keeps its own octree (built from its slice of the caller's
// concatenated arrays) and its own sigma.  A forward call evaluates all of them
// with a fixed, short launch sequence whatever the number of populations:
//   - the expansion-route populations share one launch per pass (translation
//     operators, grid clearing, the occupied-cell list, P2M, three M2L passes,
//     L2P straight into the output slices), each pass locating its work units
//     (population, cell / tile / operator) in prefix sums; they run on a branch
//     stream that forks from the caller's stream and joins it again;
//   - all populations on the direct route share ONE persistent P2P launch: a
//     grid sized to the chip takes work items (population, node) from a global
//     counter until the queue is empty, so small populations do not each pay
//     for a launch and the chip stays busy across the uneven sizes.  One staging
//     launch before it and one scatter launch after it also cover all of them.
// The backward has the same shape: the two fields it needs (weights w, and the
// upstream gradient at the targets) by the batched expansion passes with an L2P
// that also gives gradient and Laplacian, or by one persistent P2P-with-derivatives
// launch per field, then one launch that combines every point's records into its
// gradients and one that reduces the sigma derivative of each population.
// After a first eager call the sequence is captured into a hipGraph on a
// private stream and later calls with the same arguments replay the graph on
// the caller's stream.  The capture holds no memset nodes: the work counter and
// the timestamps are cleared by a kernel.
//
// The autotuner times every population at each candidate leaf size on both
// routes and keeps the fastest pair.
#include "grad_common.hpp"

#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

namespace msp {
namespace {

constexpr int kBlock = 256;

// One direct-route population as the batched kernels read it.
struct PopDesc {
    LeafSet ls;            // tree arrays, staged weights (ls.ps.w), flags, output in key order
    const int32_t *perm;   // key order -> index inside the population
    int64_t base;          // first index of the population in the caller's arrays
    int64_t n;
    int32_t pop;
};

__device__ inline int find_segment(const int64_t *off, int nseg, int64_t x) {
    int lo = 0, hi = nseg;   // off[lo] <= x < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ void k_batch_reset(const PopDesc *desc, int nd, unsigned long long *counter,
                              unsigned long long *stamps) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *counter = 0ull;
    if (i < nd) {
        stamps[2 * desc[i].pop] = ~0ull;
        stamps[2 * desc[i].pop + 1] = 0ull;
    }
}

__global__ void k_batch_stage(const PopDesc *desc, const int64_t *pt_off, int nd, const float *w,
                              const uint8_t *is_target) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= pt_off[nd]) return;
    const int d = find_segment(pt_off, nd, g);
    const PopDesc &D = desc[d];
    const int64_t i = g - pt_off[d];
    const int64_t j = D.base + D.perm[i];
    float4 *ps = const_cast<float4 *>(D.ls.ps);
    ps[i].w = w[j];
    const_cast<uint8_t *>(D.ls.tflag)[i] = is_target ? (is_target[j] != 0) : (uint8_t)1;
}

// Persistent P2P over the nodes of every direct-route population, four independent
// wavefronts per block.  A wave takes kP2PTake consecutive items per atomic addition
// on the shared counter (one item balances the load best: leaves differ widely in
// work) and leaves the loop once the counter passes the last item; population
// timestamps are recorded once per run of items of one population.
constexpr int kP2PTake = 1;
__global__ void __launch_bounds__(256, 8) k_batch_p2p(const PopDesc *desc, const int64_t *item_off, int nd,
                                                   unsigned long long *counter,
                                                   unsigned long long *stamps) {
    __shared__ P2PShared sh[4];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t total = item_off[nd];
    // a wave can take at most `total` batches before the counter passes the end
    for (int64_t it = 0; it <= total; ++it) {
        unsigned long long mine = 0ull;
        if (lane == 0) mine = atomicAdd(counter, (unsigned long long)kP2PTake);
        const int64_t first = (int64_t)__shfl(mine, 0, 64);
        if (first >= total) break;
        const int64_t last = first + kP2PTake < total ? first + kP2PTake : total;
        int pop = -1;
        unsigned long long t_first = 0ull;
        for (int64_t item = first; item < last; ++item) {
            const int d = find_segment(item_off, nd, item);
            const PopDesc &D = desc[d];
            const unsigned long long t0 = wall_clock64();
            if (D.pop != pop) {
                if (pop >= 0 && lane == 0) {
                    atomicMin(&stamps[2 * pop], t_first);
                    atomicMax(&stamps[2 * pop + 1], (unsigned long long)wall_clock64());
                }
                pop = D.pop;
                t_first = t0;
            }
            p2p_leaf(D.ls, item - item_off[d], sh[wave]);
        }
        if (lane == 0) {
            atomicMin(&stamps[2 * pop], t_first);
            atomicMax(&stamps[2 * pop + 1], (unsigned long long)wall_clock64());
        }
    }
}

// Point pairs the direct-route passes evaluate: over every leaf, its point count
// times the point counts of the leaves its interaction list names (the list read
// with the same bounds as the P2P pass), summed into *pairs.
__global__ void __launch_bounds__(256) k_batch_pairs(const PopDesc *desc, const int64_t *item_off, int nd,
                                                     unsigned long long *pairs) {
    __shared__ unsigned long long red[4];
    const int64_t total = item_off[nd];
    unsigned long long acc = 0ull;
    for (int64_t item = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; item < total;
         item += (int64_t)gridDim.x * blockDim.x) {
        const int d = find_segment(item_off, nd, item);
        const LeafSet &L = desc[d].ls;
        const int64_t v = item - item_off[d];
        if (v >= L.n_nodes || L.nnchild[v] != 0) continue;
        const int64_t l0 = L.off[v];
        int64_t l1 = L.off[v + 1];
        if (l1 - l0 > L.n_nodes) l1 = l0 + L.n_nodes;
        unsigned long long src = 0ull;
        for (int64_t e = l0; e < l1; ++e) {
            const int32_t u = L.lst[e];
            if (u >= 0 && u < L.n_nodes) src += (unsigned)L.ncount[u];
        }
        acc += (unsigned long long)(unsigned)L.ncount[v] * src;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(pairs, red[0] + red[1] + red[2] + red[3]);
}

__global__ void k_batch_scatter(const PopDesc *desc, const int64_t *pt_off, int nd, float *u_out) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= pt_off[nd]) return;
    const int d = find_segment(pt_off, nd, g);
    const PopDesc &D = desc[d];
    const int64_t i = g - pt_off[d];
    u_out[D.base + D.perm[i]] = D.ls.usort[i];
}

// ---------------------------------------------------------------------------------
// Batched backward.  One direct-route population as its kernels read it.
struct GradDesc {
    GradLeafSet L;          // tree arrays, staged weights w (L.ps.w), records L.out
    float *g2;              // staged target weights g in key order
    const int32_t *perm;    // key order -> index inside the population
    int64_t base, n;
};

// One population as the combination reads it.
struct CombDesc {
    const int32_t *iperm;   // index inside the population -> key order
    const float *rec;       // records in key order
    int64_t base, n;
    double sigma;
    int exclude_self;
};

// Both fields' weights of every direct-route population into key order (w into
// the w slot of ps, the target weights g into g2).
__global__ void k_bw_stage(const GradDesc *desc, const int64_t *pt_off, int nd, const float *w, const float *gt) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= pt_off[nd]) return;
    const int d = find_segment(pt_off, nd, g);
    const GradDesc &D = desc[d];
    const int64_t i = g - pt_off[d];
    const int64_t j = D.base + D.perm[i];
    const_cast<float4 *>(D.L.ps)[i].w = w[j];
    D.g2[i] = gt[j];
}

__global__ void k_bw_reset(unsigned long long *counter) { *counter = 0ull; }

// Persistent P2P with derivatives of both fields over the nodes of every
// direct-route population (four independent wavefronts per block, one item per
// counter addition).
__global__ void __launch_bounds__(256, 7) k_batch_p2p_grad(const GradDesc *desc, const int64_t *item_off, int nd,
                                                        unsigned long long *counter, int want_lap) {
    __shared__ GradShared sh[4];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t total = item_off[nd];
    for (int64_t it = 0; it <= total; ++it) {
        unsigned long long mine = 0ull;
        if (lane == 0) mine = atomicAdd(counter, 1ull);
        const int64_t item = (int64_t)__shfl(mine, 0, 64);
        if (item >= total) break;
        const int d = find_segment(item_off, nd, item);
        p2p_grad_leaf_t<true>(desc[d].L, desc[d].g2, item - item_off[d], kRec, want_lap, sh[wave]);
    }
}

// Gradients of every point of every population (blocks of 256 points, each within
// one population) and per-block partial sums of the sigma derivative.
__global__ void __launch_bounds__(256) k_batch_combine(const CombDesc *desc, const int64_t *blk_off, int np,
                                                       const float *gt, const float *w, int want_w, int want_pos,
                                                       int want_sigma, float *grad_w, float *grad_x,
                                                       float *grad_y, float *grad_z, double *partial) {
    __shared__ double red[kBlock];
    const int d = find_segment(blk_off, np, (int64_t)blockIdx.x);
    const CombDesc &D = desc[d];
    const int64_t j = (blockIdx.x - blk_off[d]) * (int64_t)kBlock + threadIdx.x;
    double ds = 0.0;
    if (j < D.n) {
        const int64_t o = D.base + j;
        ds = combine_point(reinterpret_cast<const float4 *>(D.rec + (int64_t)D.iperm[j] * kRec), gt[o],
                           want_pos ? w[o] : 0.f, want_w, want_pos, want_sigma, D.sigma, D.exclude_self,
                           want_w ? grad_w + o : nullptr, want_pos ? grad_x + o : nullptr,
                           want_pos ? grad_y + o : nullptr, want_pos ? grad_z + o : nullptr);
    }
    red[threadIdx.x] = ds;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0 && partial) partial[blockIdx.x] = red[0];
}

// Sigma derivative of population blockIdx.x: its block partials in order.
__global__ void __launch_bounds__(256) k_batch_sigma(const int64_t *blk_off, const double *partial,
                                                     double *grad_sigma) {
    __shared__ double red[kBlock];
    const int k = blockIdx.x;
    double s = 0.0;
    for (int64_t b = blk_off[k] + threadIdx.x; b < blk_off[k + 1]; b += kBlock) s += partial[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) grad_sigma[k] = red[0];
}

__global__ void k_bw_target_weights(const float *g, const uint8_t *is_target, int64_t n, float *gt) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    gt[i] = (!is_target || is_target[i]) ? g[i] : 0.f;
}

}  // namespace
}  // namespace msp

namespace msp {

namespace {

struct PopPlan {
    msp_fgt_params prm;
    FgtPlan pl;
};

int plan_batch(msp_batch *b, const float *sigma, const msp_fgt_params *prm, std::vector<PopPlan> &plans) {
    plans.resize(b->npop);
    for (int k = 0; k < b->npop; ++k) {
        PopPlan &pp = plans[k];
        pp.prm = *prm;
        pp.prm.sigma = sigma[k];
        if (!(sigma[k] > 0.f) || !std::isfinite(sigma[k]))
            return fail(MSP_EINVAL, "sigma[%d] must be finite and > 0", k);
        if (prm->route == MSP_ROUTE_AUTO && b->route[k] != MSP_ROUTE_AUTO) pp.prm.route = b->route[k];
        MSP_TRY(plan_fgt(b->pops[k].get(), &pp.prm, &pp.pl));
    }
    return MSP_OK;
}

// Expansion-route populations: their descriptors (weights w, flags, outputs u_out)
// into fp, and the device offsets of the batched passes uploaded into foff; bp
// gets everything but its descriptor pointer.  Host synchronisations allowed.
int prepare_fgt(msp_batch *b, const std::vector<PopPlan> &plans, const float *w, const uint8_t *is_target,
                float *u_out, std::vector<FgtPop> &fp, DevBuf &foff, DevBuf &franges, DevBuf &stamps,
                FgtBatchPlan &bp) {
    fp.clear();
    std::vector<int64_t> ops_off{0}, pw_off{0}, grid_off{0}, tile_off[3] = {{0}, {0}, {0}};
    int64_t n_pts = 0;
    int p = 0;
    for (int k = 0; k < b->npop; ++k) {
        msp_tree *t = b->pops[k].get();
        const PopPlan &pp = plans[k];
        if (pp.pl.route != MSP_ROUTE_FGT || t->n == 0) continue;
        FgtPop f;
        MSP_TRY(fgt_pop_prepare(t, pp.pl, &pp.prm, &f));
        const int64_t o = b->off[k];
        f.w = w + o;
        f.is_target = is_target ? is_target + o : nullptr;
        f.u_out = u_out ? u_out + o : nullptr;
        f.pop = k;
        p = pp.pl.p;
        fp.push_back(f);
        ops_off.push_back(ops_off.back() + 2 * (f.G[0] + f.G[1] + f.G[2]) - 3);
        pw_off.push_back(pw_off.back() + (t->n + 63) / 64);
        n_pts += t->n;
        grid_off.push_back(grid_off.back() + (int64_t)f.G[0] * f.G[1] * f.G[2] * p * p * p);
    }
    // M2L as whole-K GEMM tiles when every population's operator and tile fit in LDS
    const bool split = !plans.empty() && (plans[0].prm.flags & MSP_M2L_BF16X3) != 0;
    size_t gemm_lds = 0;
    for (const FgtPop &f : fp) {
        const size_t l = fgt_pop_gemm_lds(f, p, split);
        gemm_lds = l > gemm_lds ? l : gemm_lds;
    }
    const bool gemm = gemm_lds <= 64 * 1024;
    if (split && !fp.empty() && (p != 8 || !gemm))
        return fail(MSP_ENOTSUP, "split-bfloat16 translation in a batch needs p = 8 and tiles that fit in LDS");
    for (const FgtPop &f : fp)
        for (int pass = 0; pass < 3; ++pass)
            tile_off[pass].push_back(tile_off[pass].back() + fgt_pop_tiles(f, p, pass, gemm));
    const int nf = (int)fp.size();
    MSP_TRY(foff.ensure((size_t)6 * (nf + 1) * 8));
    MSP_TRY(franges.ensure((size_t)(n_pts + 1) * sizeof(int4) + 16));
    MSP_TRY(stamps.ensure((size_t)(b->npop > 0 ? b->npop : 1) * 16));
    bp = FgtBatchPlan{};
    bp.npop = nf;
    bp.p = p;
    bp.cus = b->cus;
    bp.gemm = gemm ? 1 : 0;
    bp.split = split ? 1 : 0;
    bp.gemm_lds = gemm_lds;
    if (nf > 0) {
        int64_t *off = foff.as<int64_t>();
        const std::vector<int64_t> *arrs[6] = {&ops_off, &pw_off, &grid_off, &tile_off[0], &tile_off[1], &tile_off[2]};
        for (int a = 0; a < 6; ++a)
            MSP_HIP(hipMemcpy(off + (size_t)a * (nf + 1), arrs[a]->data(), (size_t)(nf + 1) * 8, hipMemcpyHostToDevice));
        bp.ops_off = off;
        bp.pw_off = off + (nf + 1);
        bp.grid_off = off + 2 * (nf + 1);
        for (int pass = 0; pass < 3; ++pass) {
            bp.tile_off[pass] = off + (size_t)(3 + pass) * (nf + 1);
            bp.n_tiles[pass] = tile_off[pass].back();
        }
        bp.n_ops = ops_off.back();
        bp.n_pw = pw_off.back();
        bp.n_grid = grid_off.back();
        bp.cap = n_pts + 1;   // a cell holds at least one point
        bp.cells = franges.as<int4>();
        bp.ncells = reinterpret_cast<int32_t *>(franges.as<int4>() + bp.cap);
        bp.stamps = stamps.as<unsigned long long>();
    }
    return MSP_OK;
}

// Allocations, interaction lists and the descriptors of the direct-route
// populations (host synchronisations allowed: never under capture).
int prepare_batch(msp_batch *b, const std::vector<PopPlan> &plans, const float *w, const uint8_t *is_target,
                  float *u_out, hipStream_t s) {
    std::vector<PopDesc> d;
    std::vector<int64_t> poff{0}, ioff{0};
    (void)hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, b->device);
    // earlier work on s may still read the descriptors about to be replaced
    MSP_HIP(hipStreamSynchronize(s));
    std::vector<FgtPop> fp;
    MSP_TRY(prepare_fgt(b, plans, w, is_target, u_out, fp, b->foff, b->franges, b->stamps, b->fplan));
    MSP_TRY(b->fdesc.ensure((fp.size() + 1) * sizeof(FgtPop)));
    if (!fp.empty()) {
        MSP_HIP(hipMemcpy(b->fdesc.p, fp.data(), fp.size() * sizeof(FgtPop), hipMemcpyHostToDevice));
        b->fplan.pops = b->fdesc.as<FgtPop>();
    }
    for (int k = 0; k < b->npop; ++k) {
        msp_tree *t = b->pops[k].get();
        const PopPlan &pp = plans[k];
        if (pp.pl.route == MSP_ROUTE_FGT || t->n == 0) continue;
        const int64_t nb = t->n > 0 ? t->n : 1;
        MSP_TRY(t->tflag.ensure(nb));
        MSP_TRY(t->usort.ensure(nb * 4));
        MSP_TRY(direct_route_lists(t, &pp.prm, s));
        PopDesc q;
        q.ls = LeafSet{t->n_nodes, t->nfirst.as<int32_t>(), t->ncount.as<int32_t>(), t->nnchild.as<int32_t>(),
                       t->nlevel.as<int32_t>(), t->nix.as<int32_t>(), t->niy.as<int32_t>(), t->niz.as<int32_t>(),
                       BoxGeo{{t->geo.lo[0], t->geo.lo[1], t->geo.lo[2]}, t->geo.side},
                       t->list_off.as<int64_t>(), t->list_idx.as<int32_t>(), t->ps.as<float4>(),
                       t->tflag.as<uint8_t>(), (float)(std::sqrt(1.4426950408889634) / (double)pp.prm.sigma),
                       (pp.prm.flags & MSP_EXCLUDE_SELF) ? 1 : 0, t->usort.as<float>()};
        q.perm = t->perm.as<int32_t>();
        q.base = b->off[k];
        q.n = t->n;
        q.pop = k;
        d.push_back(q);
        poff.push_back(poff.back() + t->n);
        ioff.push_back(ioff.back() + t->n_nodes);
    }
    if (!b->fork) {
        MSP_HIP(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
        for (int r = 0; r < msp_batch::kBranches; ++r) {
            MSP_HIP(hipStreamCreateWithFlags(&b->side[r], hipStreamNonBlocking));
            MSP_HIP(hipEventCreateWithFlags(&b->join[r], hipEventDisableTiming));
        }
    }
    b->n_direct = (int32_t)d.size();
    b->direct_pops.clear();
    for (const PopDesc &q : d) b->direct_pops.push_back(q.pop);
    b->direct_points = poff.back();
    b->direct_items = ioff.back();
    MSP_TRY(b->desc.ensure((d.size() + 1) * sizeof(PopDesc)));
    MSP_TRY(b->pt_off.ensure(poff.size() * 8));
    MSP_TRY(b->item_off.ensure(ioff.size() * 8));
    MSP_TRY(b->counter.ensure(8));
    MSP_HIP(hipStreamSynchronize(s));
    if (!d.empty()) MSP_HIP(hipMemcpy(b->desc.p, d.data(), d.size() * sizeof(PopDesc), hipMemcpyHostToDevice));
    MSP_HIP(hipMemcpy(b->pt_off.p, poff.data(), poff.size() * 8, hipMemcpyHostToDevice));
    MSP_HIP(hipMemcpy(b->item_off.p, ioff.data(), ioff.size() * 8, hipMemcpyHostToDevice));
    std::vector<uint64_t> zero((size_t)(b->npop > 0 ? b->npop : 1) * 2, 0);
    MSP_HIP(hipMemcpy(b->stamps.p, zero.data(), zero.size() * 8, hipMemcpyHostToDevice));
    return MSP_OK;
}

// The whole forward as a launch sequence on s (no synchronisation, no allocation
// once prepare_batch has run for the same plans).
int enqueue_forward(msp_batch *b, const std::vector<PopPlan> &plans, const float *w,
                    const uint8_t *is_target, float *u_out, hipStream_t s) {
    int64_t launches = 0;
    uint64_t *stamps = b->stamps.as<uint64_t>();
    // all expansion-route populations on a branch stream that forks from s here and
    // joins it at the end (also under capture), beside the direct-route launch
    MSP_HIP(hipEventRecord(b->fork, s));
    MSP_HIP(hipStreamWaitEvent(b->side[0], b->fork, 0));
    MSP_TRY(fgt_batch_forward(b->fplan, b->side[0]));
    if (b->fplan.npop > 0) launches += 8;
    (void)stamps;
    const int nd = b->n_direct;
    if (nd > 0) {
        const PopDesc *desc = b->desc.as<PopDesc>();
        auto *counter = b->counter.as<unsigned long long>();
        auto *st = b->stamps.as<unsigned long long>();
        hipLaunchKernelGGL(k_batch_reset, dim3(grid_for(nd, 64)), dim3(64), 0, s, desc, nd, counter, st);
        MSP_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_batch_stage, dim3(grid_for(b->direct_points, kBlock)), dim3(kBlock), 0, s, desc,
                           b->pt_off.as<int64_t>(), nd, w, is_target);
        MSP_CHECK_LAUNCH();
        const int64_t waves = (int64_t)b->cus * 32;
        const int64_t want = b->direct_items < waves ? b->direct_items : waves;
        const int64_t grid = (want + 3) / 4;
        if (grid > 0) {
            hipLaunchKernelGGL(k_batch_p2p, dim3((unsigned)grid), dim3(256), 0, s, desc,
                               b->item_off.as<int64_t>(), nd, counter, st);
            MSP_CHECK_LAUNCH();
        }
        hipLaunchKernelGGL(k_batch_scatter, dim3(grid_for(b->direct_points, kBlock)), dim3(kBlock), 0, s, desc,
                           b->pt_off.as<int64_t>(), nd, u_out);
        MSP_CHECK_LAUNCH();
        launches += 4;
    }
    MSP_HIP(hipEventRecord(b->join[0], b->side[0]));
    MSP_HIP(hipStreamWaitEvent(s, b->join[0], 0));
    b->launches = launches;
    return MSP_OK;
}

void append_bytes(std::vector<unsigned char> &k, const void *p, size_t n) {
    const unsigned char *c = static_cast<const unsigned char *>(p);
    k.insert(k.end(), c, c + n);
}

// What a captured graph takes from the populations' trees: the addresses of their
// buffers and the parameters of their interaction lists.  A graph is replayed only
// while this is unchanged (the other call's preparation may reallocate or rebuild).
std::vector<uintptr_t> state_signature(const msp_batch *b) {
    std::vector<uintptr_t> sig;
    sig.reserve(b->pops.size() * 24);
    for (const auto &tp : b->pops) {
        const msp_tree *t = tp.get();
        const msp::DevBuf *bufs[] = {&t->keys, &t->ps, &t->perm, &t->iperm, &t->nfirst, &t->ncount, &t->nnchild,
                                     &t->nlevel, &t->nix, &t->niy, &t->niz, &t->gridA, &t->gridB, &t->ops,
                                     &t->list_off, &t->list_idx, &t->tflag, &t->usort, &t->bwd};
        for (const msp::DevBuf *d : bufs) sig.push_back(reinterpret_cast<uintptr_t>(d->p));
        uint32_t ls, lc;
        std::memcpy(&ls, &t->list_sigma, 4);
        std::memcpy(&lc, &t->list_cutoff, 4);
        sig.push_back(((uintptr_t)ls << 32) | lc);
        sig.push_back((uintptr_t)t->lists_valid | ((uintptr_t)t->iperm_valid << 1));
    }
    return sig;
}

}  // namespace

int batch_build(msp_batch *b, const float *x, const float *y, const float *z, const int64_t *offsets,
                int32_t npop, const int32_t *leaf_max, int32_t max_depth, hipStream_t s) {
    b->drop_graph();
    b->pops.clear();
    b->npop = npop;
    b->off.assign(offsets, offsets + npop + 1);
    b->leaf_max.resize(npop);
    b->route.assign(npop, MSP_ROUTE_AUTO);
    MSP_HIP(hipGetDevice(&b->device));
    for (int k = 0; k < npop; ++k) {
        b->leaf_max[k] = leaf_max ? leaf_max[k] : 64;
        auto t = std::make_unique<msp_tree>();
        t->device = b->device;
        const int64_t o = offsets[k], n = offsets[k + 1] - offsets[k];
        MSP_TRY(build_tree(t.get(), x + o, y + o, z + o, n, b->leaf_max[k], max_depth, s));
        b->pops.push_back(std::move(t));
    }
    ++b->generation;
    return MSP_OK;
}

int batch_forward(msp_batch *b, const float *w, const uint8_t *is_target, const float *sigma,
                  const msp_fgt_params *prm, float *u_out, int use_graph, hipStream_t s) {
    std::vector<PopPlan> plans;
    MSP_TRY(plan_batch(b, sigma, prm, plans));
    std::vector<unsigned char> key;
    append_bytes(key, &b->generation, sizeof(b->generation));
    append_bytes(key, &w, sizeof(w));
    append_bytes(key, &is_target, sizeof(is_target));
    append_bytes(key, &u_out, sizeof(u_out));
    append_bytes(key, prm, sizeof(*prm));
    append_bytes(key, sigma, sizeof(float) * b->npop);
    append_bytes(key, b->route.data(), sizeof(int32_t) * b->route.size());
    if (use_graph && b->exec && key == b->key && state_signature(b) == b->fsig) {
        MSP_HIP(hipGraphLaunch(b->exec, s));
        return MSP_OK;
    }
    b->drop_fwd_graph();
    b->pair_gen = -1;
    MSP_TRY(prepare_batch(b, plans, w, is_target, u_out, s));
    b->pair_gen = b->generation;
    b->dsig = state_signature(b);
    MSP_TRY(enqueue_forward(b, plans, w, is_target, u_out, s));
    if (!use_graph) return MSP_OK;
    // capture the same sequence for later calls
    if (!b->cap) MSP_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    MSP_HIP(hipStreamSynchronize(s));
    MSP_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_forward(b, plans, w, is_target, u_out, b->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (rc != MSP_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess || !g) return fail(MSP_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    b->graph = g;
    MSP_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->key = key;
    b->fsig = state_signature(b);
    return MSP_OK;
}

namespace {

// Backward descriptors in the batch's own buffers (the forward's graph keeps
// reading the forward's): expansion-route populations twice (weights w, then the
// target weights g), direct-route populations once, every population for the
// combination.  Interaction lists, inverse permutations and record buffers are
// made here.  Host synchronisations allowed: never under capture.
int prepare_backward(msp_batch *b, const std::vector<PopPlan> &plans, const float *w, hipStream_t s) {
    (void)hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, b->device);
    MSP_HIP(hipStreamSynchronize(s));
    const int64_t N = b->npop > 0 ? b->off[b->npop] : 0;
    MSP_TRY(b->bw_gt.ensure((size_t)(N > 0 ? N : 1) * 4));
    const float *gt = b->bw_gt.as<float>();
    std::vector<CombDesc> cd;
    std::vector<int64_t> boff{0};
    for (int k = 0; k < b->npop; ++k) {
        msp_tree *t = b->pops[k].get();
        CombDesc c{nullptr, nullptr, b->off[k], t->n, (double)plans[k].prm.sigma,
                   (plans[k].prm.flags & MSP_EXCLUDE_SELF) ? 1 : 0};
        if (t->n > 0) {
            MSP_TRY(t->bwd.ensure((size_t)t->n * (kRec + 1) * 4));   // records, then g in key order
            MSP_TRY(ensure_iperm(t, s));
            c.iperm = t->iperm.as<int32_t>();
            c.rec = t->bwd.as<float>();
        }
        cd.push_back(c);
        boff.push_back(boff.back() + (t->n + kBlock - 1) / kBlock);
    }
    // expansion route: one plan, two descriptor sets
    std::vector<FgtPop> fp;
    MSP_TRY(prepare_fgt(b, plans, w, nullptr, nullptr, fp, b->bw_foff, b->bw_franges, b->bw_stamps, b->bw_plan[0]));
    const size_t nf = fp.size();
    for (FgtPop &f : fp) f.rec = b->pops[f.pop]->bwd.as<float>();
    std::vector<FgtPop> both(fp);
    for (FgtPop f : fp) {
        f.w = gt + b->off[f.pop];
        both.push_back(f);
    }
    MSP_TRY(b->bw_fdesc.ensure((both.size() + 1) * sizeof(FgtPop)));
    b->bw_plan[1] = b->bw_plan[0];
    if (nf > 0) {
        MSP_HIP(hipMemcpy(b->bw_fdesc.p, both.data(), both.size() * sizeof(FgtPop), hipMemcpyHostToDevice));
        b->bw_plan[0].pops = b->bw_fdesc.as<FgtPop>();
        b->bw_plan[1].pops = b->bw_fdesc.as<FgtPop>() + nf;
    }
    // direct route
    std::vector<GradDesc> gd;
    std::vector<int64_t> poff{0}, ioff{0};
    for (int k = 0; k < b->npop; ++k) {
        msp_tree *t = b->pops[k].get();
        const PopPlan &pp = plans[k];
        if (pp.pl.route == MSP_ROUTE_FGT || t->n == 0) continue;
        MSP_TRY(direct_route_lists(t, &pp.prm, s));
        const double sig = pp.prm.sigma;
        GradDesc g;
        g.L = GradLeafSet{t->n_nodes, t->nfirst.as<int32_t>(), t->ncount.as<int32_t>(), t->nnchild.as<int32_t>(),
                          t->nlevel.as<int32_t>(), t->nix.as<int32_t>(), t->niy.as<int32_t>(), t->niz.as<int32_t>(),
                          BoxGeo{{t->geo.lo[0], t->geo.lo[1], t->geo.lo[2]}, t->geo.side},
                          t->list_off.as<int64_t>(), t->list_idx.as<int32_t>(), t->ps.as<float4>(),
                          (float)(-1.4426950408889634 / (sig * sig)), (float)(1.0 / (sig * sig)),
                          t->bwd.as<float>()};
        g.g2 = t->bwd.as<float>() + (size_t)t->n * kRec;
        g.perm = t->perm.as<int32_t>();
        g.base = b->off[k];
        g.n = t->n;
        gd.push_back(g);
        poff.push_back(poff.back() + t->n);
        ioff.push_back(ioff.back() + t->n_nodes);
    }
    b->bw_nd = (int32_t)gd.size();
    b->bw_points = poff.back();
    b->bw_items = ioff.back();
    b->bw_nblk = boff.back();
    MSP_TRY(b->bw_desc.ensure((gd.size() + 1) * sizeof(GradDesc)));
    MSP_TRY(b->bw_pt_off.ensure(poff.size() * 8));
    MSP_TRY(b->bw_item_off.ensure(ioff.size() * 8));
    MSP_TRY(b->bw_counter.ensure(8));
    MSP_TRY(b->bw_comb.ensure((cd.size() + 1) * sizeof(CombDesc)));
    MSP_TRY(b->bw_boff.ensure(boff.size() * 8));
    MSP_TRY(b->bw_partial.ensure((size_t)(b->bw_nblk > 0 ? b->bw_nblk : 1) * 8));
    MSP_HIP(hipStreamSynchronize(s));
    if (!gd.empty()) MSP_HIP(hipMemcpy(b->bw_desc.p, gd.data(), gd.size() * sizeof(GradDesc), hipMemcpyHostToDevice));
    MSP_HIP(hipMemcpy(b->bw_pt_off.p, poff.data(), poff.size() * 8, hipMemcpyHostToDevice));
    MSP_HIP(hipMemcpy(b->bw_item_off.p, ioff.data(), ioff.size() * 8, hipMemcpyHostToDevice));
    if (!cd.empty()) MSP_HIP(hipMemcpy(b->bw_comb.p, cd.data(), cd.size() * sizeof(CombDesc), hipMemcpyHostToDevice));
    MSP_HIP(hipMemcpy(b->bw_boff.p, boff.data(), boff.size() * 8, hipMemcpyHostToDevice));
    if (!b->bfork) {
        MSP_HIP(hipEventCreateWithFlags(&b->bfork, hipEventDisableTiming));
        MSP_HIP(hipStreamCreateWithFlags(&b->bside, hipStreamNonBlocking));
        MSP_HIP(hipEventCreateWithFlags(&b->bjoin, hipEventDisableTiming));
    }
    return MSP_OK;
}

// The whole backward as a launch sequence on s (no synchronisation, no allocation
// once prepare_backward has run for the same plans): the target weights, the two
// fields of the expansion-route populations on a branch stream beside those of
// the direct-route populations, then the combination.
int enqueue_backward(msp_batch *b, const float *w, const uint8_t *is_target, const float *grad_u,
                     float *grad_w, float *grad_x, float *grad_y, float *grad_z, double *grad_sigma,
                     hipStream_t s) {
    const int64_t N = b->npop > 0 ? b->off[b->npop] : 0;
    const bool needA = grad_x || grad_sigma;
    const bool needB = grad_w || grad_x;
    float *gt = b->bw_gt.as<float>();
    if (N > 0) {
        hipLaunchKernelGGL(k_bw_target_weights, dim3(grid_for(N, kBlock)), dim3(kBlock), 0, s, grad_u, is_target, N,
                           gt);
        MSP_CHECK_LAUNCH();
    }
    MSP_HIP(hipEventRecord(b->bfork, s));
    MSP_HIP(hipStreamWaitEvent(b->bside, b->bfork, 0));
    if (needA) MSP_TRY(fgt_batch_field_grad(b->bw_plan[0], kRec, 0, grad_sigma ? 1 : 0, b->bside));
    if (needB) MSP_TRY(fgt_batch_field_grad(b->bw_plan[1], kRec, 5, 0, b->bside));
    const int nd = b->bw_nd;
    if (nd > 0) {
        const GradDesc *desc = b->bw_desc.as<GradDesc>();
        auto *counter = b->bw_counter.as<unsigned long long>();
        const int64_t waves = (int64_t)b->cus * 32;
        const int64_t want = b->bw_items < waves ? b->bw_items : waves;
        const unsigned grid = (unsigned)((want + 3) / 4);
        // both fields in one pass: one exponential per pair serves both
        hipLaunchKernelGGL(k_bw_stage, dim3(grid_for(b->bw_points, kBlock)), dim3(kBlock), 0, s, desc,
                           b->bw_pt_off.as<int64_t>(), nd, w, gt);
        MSP_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_bw_reset, dim3(1), dim3(1), 0, s, counter);
        MSP_CHECK_LAUNCH();
        if (grid > 0) {
            hipLaunchKernelGGL(k_batch_p2p_grad, dim3(grid), dim3(256), 0, s, desc, b->bw_item_off.as<int64_t>(),
                               nd, counter, grad_sigma ? 1 : 0);
            MSP_CHECK_LAUNCH();
        }
    }
    MSP_HIP(hipEventRecord(b->bjoin, b->bside));
    MSP_HIP(hipStreamWaitEvent(s, b->bjoin, 0));
    if (b->npop > 0 && b->bw_nblk > 0) {
        hipLaunchKernelGGL(k_batch_combine, dim3((unsigned)b->bw_nblk), dim3(kBlock), 0, s,
                           b->bw_comb.as<CombDesc>(), b->bw_boff.as<int64_t>(), b->npop, gt, w,
                           grad_w && needB ? 1 : 0, grad_x ? 1 : 0, grad_sigma ? 1 : 0, grad_w, grad_x, grad_y,
                           grad_z, b->bw_partial.as<double>());
        MSP_CHECK_LAUNCH();
    }
    if (grad_sigma && b->npop > 0) {
        hipLaunchKernelGGL(k_batch_sigma, dim3((unsigned)b->npop), dim3(kBlock), 0, s, b->bw_boff.as<int64_t>(),
                           b->bw_partial.as<double>(), grad_sigma);
        MSP_CHECK_LAUNCH();
    }
    return MSP_OK;
}

}  // namespace

// With use_graph, the first call with given arguments runs eagerly (allocations,
// lists, inverse permutations) and the same sequence is captured into a hipGraph;
// later calls replay it while the arguments and the populations' buffers are unchanged.
int batch_backward(msp_batch *b, const float *w, const uint8_t *is_target, const float *sigma,
                   const msp_fgt_params *prm, const float *grad_u, float *grad_w, float *grad_x,
                   float *grad_y, float *grad_z, double *grad_sigma, int use_graph, hipStream_t s) {
    std::vector<PopPlan> plans;
    MSP_TRY(plan_batch(b, sigma, prm, plans));
    std::vector<unsigned char> key;
    append_bytes(key, &b->generation, sizeof(b->generation));
    const void *ptrs[9] = {w, is_target, grad_u, grad_w, grad_x, grad_y, grad_z, grad_sigma, nullptr};
    append_bytes(key, ptrs, sizeof(ptrs));
    append_bytes(key, prm, sizeof(*prm));
    append_bytes(key, sigma, sizeof(float) * b->npop);
    append_bytes(key, b->route.data(), sizeof(int32_t) * b->route.size());
    if (use_graph && b->bexec && key == b->bkey && state_signature(b) == b->bsig) {
        MSP_HIP(hipGraphLaunch(b->bexec, s));
        return MSP_OK;
    }
    b->drop_bwd_graph();
    MSP_TRY(prepare_backward(b, plans, w, s));
    MSP_TRY(enqueue_backward(b, w, is_target, grad_u, grad_w, grad_x, grad_y, grad_z, grad_sigma, s));
    if (!use_graph) return MSP_OK;
    if (!b->cap) MSP_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    MSP_HIP(hipStreamSynchronize(s));
    MSP_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_backward(b, w, is_target, grad_u, grad_w, grad_x, grad_y, grad_z, grad_sigma, b->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (rc != MSP_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess || !g) return fail(MSP_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    b->bgraph = g;
    MSP_HIP(hipGraphInstantiate(&b->bexec, b->bgraph, nullptr, nullptr, 0));
    b->bkey = key;
    b->bsig = state_signature(b);
    return MSP_OK;
}

int batch_autotune(msp_batch *b, const float *x, const float *y, const float *z, const int64_t *offsets,
                   int32_t npop, const float *w, const uint8_t *is_target, const float *sigma,
                   const msp_fgt_params *prm, const int32_t *cand, int32_t ncand, int32_t max_depth,
                   float *scratch_u, int32_t *leaf_out, int32_t *route_out, hipStream_t s) {
    std::vector<int32_t> best_leaf(npop, 64), best_route(npop, MSP_ROUTE_AUTO);
    hipEvent_t e0, e1;
    MSP_HIP(hipEventCreate(&e0));
    MSP_HIP(hipEventCreate(&e1));
    int rc = MSP_OK;
    for (int k = 0; k < npop && rc == MSP_OK; ++k) {
        const int64_t o = offsets[k], n = offsets[k + 1] - offsets[k];
        double best = 1e300;
        for (int c = 0; c < ncand && rc == MSP_OK; ++c) {
            msp_tree t;
            (void)hipGetDevice(&t.device);
            rc = build_tree(&t, x + o, y + o, z + o, n, cand[c], max_depth, s);
            if (rc != MSP_OK) break;
            for (int r : {MSP_ROUTE_FGT, MSP_ROUTE_DIRECT}) {
                msp_fgt_params q = *prm;
                q.sigma = sigma[k];
                q.route = r;
                FgtPlan pl;
                if (plan_fgt(&t, &q, &pl) != MSP_OK) continue;   // grid too large for this route
                auto run = [&]() -> int {
                    if (pl.route == MSP_ROUTE_FGT)
                        return fgt_forward_grid(&t, pl, &q, w + o, is_target ? is_target + o : nullptr,
                                                scratch_u + o, s);
                    MSP_TRY(stage_inputs(&t, w + o, is_target ? is_target + o : nullptr, s));
                    MSP_TRY(direct_route(&t, &q, s));
                    return scatter_output(&t, scratch_u + o, q.flags, false, s);
                };
                rc = run();   // first call: allocations and lists
                if (rc != MSP_OK) break;
                (void)hipEventRecord(e0, s);
                for (int rep = 0; rep < 3 && rc == MSP_OK; ++rep) rc = run();
                (void)hipEventRecord(e1, s);
                if (rc != MSP_OK) break;
                (void)hipEventSynchronize(e1);
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (ms < best) {
                    best = ms;
                    best_leaf[k] = cand[c];
                    best_route[k] = r;
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != MSP_OK) return rc;
    MSP_TRY(batch_build(b, x, y, z, offsets, npop, best_leaf.data(), max_depth, s));
    b->route = best_route;
    if (leaf_out) std::memcpy(leaf_out, best_leaf.data(), sizeof(int32_t) * npop);
    if (route_out) std::memcpy(route_out, best_route.data(), sizeof(int32_t) * npop);
    return MSP_OK;
}

int batch_info(const msp_batch *b, int32_t *npop, int64_t *launches) {
    if (npop) *npop = b->npop;
    if (launches) *launches = b->launches;
    return MSP_OK;
}

int batch_instance_ms(msp_batch *b, double *ms) {
    std::vector<uint64_t> st((size_t)b->npop * 2, 0);
    if (b->npop > 0) MSP_HIP(hipMemcpy(st.data(), b->stamps.p, st.size() * 8, hipMemcpyDeviceToHost));
    int khz = 100000;
    (void)hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, b->device);
    for (int k = 0; k < b->npop; ++k) {
        const uint64_t a = st[2 * k], c = st[2 * k + 1];
        ms[k] = (c > a && a != ~0ull) ? (double)(c - a) / (double)khz : 0.0;
    }
    return MSP_OK;
}

int batch_pair_count(msp_batch *b, int64_t *pairs, double *span_ms, hipStream_t s) {
    if (b->pair_gen != b->generation || state_signature(b) != b->dsig)
        return fail(MSP_ESTATE, "no forward since the populations were built or their lists changed");
    unsigned long long sum = 0ull;
    if (b->n_direct > 0 && b->direct_items > 0) {
        MSP_TRY(b->pair_sum.ensure(8));
        auto *ps = b->pair_sum.as<unsigned long long>();
        MSP_HIP(hipMemsetAsync(ps, 0, 8, s));
        const int64_t want = (b->direct_items + kBlock - 1) / kBlock;
        const int64_t grid = want < 4096 ? want : 4096;
        hipLaunchKernelGGL(k_batch_pairs, dim3((unsigned)grid), dim3(kBlock), 0, s, b->desc.as<PopDesc>(),
                           b->item_off.as<int64_t>(), b->n_direct, ps);
        MSP_CHECK_LAUNCH();
        MSP_HIP(hipMemcpyAsync(&sum, ps, 8, hipMemcpyDeviceToHost, s));
        MSP_HIP(hipStreamSynchronize(s));
    }
    if (pairs) *pairs = (int64_t)sum;
    if (span_ms) {
        *span_ms = 0.0;
        if (!b->direct_pops.empty()) {
            MSP_HIP(hipStreamSynchronize(s));
            std::vector<uint64_t> st((size_t)b->npop * 2, 0);
            MSP_HIP(hipMemcpy(st.data(), b->stamps.p, st.size() * 8, hipMemcpyDeviceToHost));
            uint64_t lo = ~0ull, hi = 0ull;
            for (int32_t k : b->direct_pops) {
                lo = st[2 * k] < lo ? st[2 * k] : lo;
                hi = st[2 * k + 1] > hi ? st[2 * k + 1] : hi;
            }
            int khz = 100000;
            (void)hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, b->device);
            if (hi > lo && lo != ~0ull) *span_ms = (double)(hi - lo) / (double)khz;
        }
    }
    return MSP_OK;
}

}  // namespace msp
