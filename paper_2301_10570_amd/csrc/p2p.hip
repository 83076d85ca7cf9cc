// Direct evaluation of the Gaussian sum (Eq. (8)).
//
// Near-field route: for every leaf of the octree, the list of source leaves whose
// boxes come within the cutoff radius of its box (interaction lists built by a
// depth-first walk of the node table), then P2P: one wavefront per target leaf,
// source leaves staged through LDS.
//
// All-pairs baseline: every target against every source with no tree and no
// cutoff, sources streamed through LDS in tiles.
//
// exp(-d^2/sigma^2) is evaluated as exp2(-(k d)^2) with k^2 = log2(e)/sigma^2.
#include "internal.hpp"
#include "p2p_leaf.hpp"

#include <cmath>

namespace msp {
namespace {

constexpr int kBlock = 256;
constexpr int kStack = 8 * (kDepth + 2);

// Count (fill == nullptr) or write the source leaves within reach of each leaf.
__global__ void k_lists(int64_t n_nodes, const int32_t *nlevel, const int32_t *nix,
                        const int32_t *niy, const int32_t *niz, const int32_t *nfchild,
                        const int32_t *nnchild, BoxGeo geo, float r2, int unlimited,
                        const int64_t *off, int32_t *cnt, int32_t *fill) {
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= n_nodes) return;
    if (nnchild[v] != 0) {
        if (!fill) cnt[v] = 0;
        return;
    }
    float ct[3], ht;
    node_box(geo, nlevel[v], nix[v], niy[v], niz[v], ct, ht);
    int32_t stack[kStack];
    int sp = 0;
    stack[sp++] = 0;
    int64_t k = fill ? off[v] : 0;
    int32_t c = 0;
    while (sp > 0) {
        const int32_t u = stack[--sp];
        float cs[3], hs;
        node_box(geo, nlevel[u], nix[u], niy[u], niz[u], cs, hs);
        float d2 = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float gap = fmaxf(fabsf(ct[a] - cs[a]) - (ht + hs), 0.f);
            d2 = fmaf(gap, gap, d2);
        }
        if (!unlimited && d2 > r2) continue;
        const int nc = nnchild[u];
        if (nc == 0) {
            if (fill) fill[k++] = u;
            ++c;
        } else {
            const int32_t f = nfchild[u];
            // children sit one level deeper, so the walk ends within max_depth
            // levels; the bounds below only protect against a corrupt table
            if (f <= u || f + nc > n_nodes || sp + nc > kStack) continue;
            for (int q = nc - 1; q >= 0; --q) stack[sp++] = f + q;
        }
    }
    if (!fill) cnt[v] = c;
}

__global__ void k_scan_i32_to_i64(const int32_t *cnt, int64_t n, int64_t *off) {
    // single-block exclusive scan (chunked); n up to a few million entries
    __shared__ int64_t part[kBlock];
    const int64_t per = (n + kBlock - 1) / kBlock;
    const int64_t b0 = threadIdx.x * per;
    int64_t s = 0;
    for (int64_t k = 0; k < per; ++k)
        if (b0 + k < n) s += cnt[b0 + k];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int q = 0; q < kBlock; ++q) {
            const int64_t v = part[q];
            part[q] = run;
            run += v;
        }
        off[n] = run;
    }
    __syncthreads();
    int64_t run = part[threadIdx.x];
    for (int64_t k = 0; k < per; ++k)
        if (b0 + k < n) {
            off[b0 + k] = run;
            run += cnt[b0 + k];
        }
}

// One wavefront per target leaf (non-leaf nodes return at once).
__global__ void __launch_bounds__(256, 8) k_p2p(int64_t n_nodes, const int32_t *nfirst,
                                            const int32_t *ncount, const int32_t *nnchild,
                                            const int32_t *nlevel, const int32_t *nix,
                                            const int32_t *niy, const int32_t *niz, BoxGeo geo,
                                            const int64_t *off, const int32_t *lst, const float4 *ps,
                                            const uint8_t *tflag, float k_scale, int exclude_self,
                                            float *usort) {
    __shared__ P2PShared sh[4];
    const LeafSet ls{n_nodes, nfirst, ncount, nnchild, nlevel, nix, niy, niz, geo, off, lst, ps, tflag,
                     k_scale, exclude_self, usort};
    const int wave = threadIdx.x >> 6;
    p2p_leaf(ls, (int64_t)blockIdx.x * 4 + wave, sh[wave]);
}

// All-pairs baseline: one target per thread, 1024 sources per LDS tile.
constexpr int kDirTile = 1024;
__global__ void __launch_bounds__(kBlock) k_direct(const float *tx, const float *ty, const float *tz,
                                                   int64_t nt, const float *sx, const float *sy,
                                                   const float *sz, const float *w, int64_t ns,
                                                   float neg_c, float *u) {
    __shared__ float4 tile[kDirTile];
    const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    const bool valid = i < nt;
    const float x = valid ? tx[i] : 0.f, y = valid ? ty[i] : 0.f, z = valid ? tz[i] : 0.f;
    float total = 0.f, comp = 0.f;
    for (int64_t s0 = 0; s0 < ns; s0 += kDirTile) {
        const int cnt = ns - s0 < kDirTile ? (int)(ns - s0) : kDirTile;
        __syncthreads();
        for (int e = threadIdx.x; e < kDirTile; e += kBlock) {
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (e < cnt) v = make_float4(sx[s0 + e], sy[s0 + e], sz[s0 + e], w[s0 + e]);
            tile[e] = v;
        }
        __syncthreads();
        float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
        // the padded tail has w = 0, so the full tile can be summed
#pragma unroll 4
        for (int j = 0; j < kDirTile; j += 4) {
            float4 a = tile[j], b = tile[j + 1], c = tile[j + 2], d = tile[j + 3];
            float dx, dy, dz;
            dx = x - a.x; dy = y - a.y; dz = z - a.z;
            p0 = fmaf(a.w, __builtin_amdgcn_exp2f(fmaf(dx, dx, fmaf(dy, dy, dz * dz)) * neg_c), p0);
            dx = x - b.x; dy = y - b.y; dz = z - b.z;
            p1 = fmaf(b.w, __builtin_amdgcn_exp2f(fmaf(dx, dx, fmaf(dy, dy, dz * dz)) * neg_c), p1);
            dx = x - c.x; dy = y - c.y; dz = z - c.z;
            p2 = fmaf(c.w, __builtin_amdgcn_exp2f(fmaf(dx, dx, fmaf(dy, dy, dz * dz)) * neg_c), p2);
            dx = x - d.x; dy = y - d.y; dz = z - d.z;
            p3 = fmaf(d.w, __builtin_amdgcn_exp2f(fmaf(dx, dx, fmaf(dy, dy, dz * dz)) * neg_c), p3);
        }
        const float part = (p0 + p1) + (p2 + p3);
        const float yk = part - comp;
        const float t = total + yk;
        comp = (t - total) - yk;
        total = t;
    }
    if (valid) u[i] = total;
}

}  // namespace

int direct_route_counts(msp_tree *t, const msp_fgt_params *prm, hipStream_t s) {
    const int64_t nn = t->n_nodes;
    if (t->n == 0) return MSP_OK;
    if (t->counts_valid && t->list_sigma == prm->sigma && t->list_cutoff == prm->cutoff_sigmas) return MSP_OK;
    BoxGeo geo{{t->geo.lo[0], t->geo.lo[1], t->geo.lo[2]}, t->geo.side};
    const bool unlimited = !(prm->cutoff_sigmas > 0.f);
    const float R = unlimited ? 0.f : prm->cutoff_sigmas * prm->sigma;
    PhaseScope ps(&t->timing, PH_LISTS, s);
    t->lists_valid = false;
    t->counts_valid = false;
    MSP_TRY(t->list_cnt.ensure(nn * 4));
    MSP_TRY(t->list_off.ensure((nn + 1) * 8));
    hipLaunchKernelGGL(k_lists, dim3(grid_for(nn, 128)), dim3(128), 0, s, nn, t->nlevel.as<int32_t>(),
                       t->nix.as<int32_t>(), t->niy.as<int32_t>(), t->niz.as<int32_t>(),
                       t->nfchild.as<int32_t>(), t->nnchild.as<int32_t>(), geo, R * R, unlimited ? 1 : 0,
                       nullptr, t->list_cnt.as<int32_t>(), nullptr);
    MSP_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_scan_i32_to_i64, dim3(1), dim3(kBlock), 0, s, t->list_cnt.as<int32_t>(), nn,
                       t->list_off.as<int64_t>());
    MSP_CHECK_LAUNCH();
    int64_t total = 0;
    MSP_HIP(hipMemcpyAsync(&total, t->list_off.as<int64_t>() + nn, 8, hipMemcpyDeviceToHost, s));
    MSP_HIP(hipStreamSynchronize(s));
    if (total > 0x7fffffffLL)
        return fail(MSP_ENOSPC, "direct route: %lld leaf pairs within the cutoff exceed the list limit",
                    (long long)total);
    t->list_total = total;
    t->list_sigma = prm->sigma;
    t->list_cutoff = prm->cutoff_sigmas;
    t->counts_valid = true;
    return MSP_OK;
}

int direct_route_fill(msp_tree *t, const msp_fgt_params *prm, hipStream_t s) {
    const int64_t nn = t->n_nodes;
    if (t->n == 0) return MSP_OK;
    BoxGeo geo{{t->geo.lo[0], t->geo.lo[1], t->geo.lo[2]}, t->geo.side};
    const bool unlimited = !(prm->cutoff_sigmas > 0.f);
    const float R = unlimited ? 0.f : prm->cutoff_sigmas * prm->sigma;
    PhaseScope ps(&t->timing, PH_LISTS, s);
    MSP_TRY(t->list_idx.ensure((t->list_total > 0 ? t->list_total : 1) * 4));
    hipLaunchKernelGGL(k_lists, dim3(grid_for(nn, 128)), dim3(128), 0, s, nn, t->nlevel.as<int32_t>(),
                       t->nix.as<int32_t>(), t->niy.as<int32_t>(), t->niz.as<int32_t>(),
                       t->nfchild.as<int32_t>(), t->nnchild.as<int32_t>(), geo, R * R, unlimited ? 1 : 0,
                       t->list_off.as<int64_t>(), t->list_cnt.as<int32_t>(), t->list_idx.as<int32_t>());
    MSP_CHECK_LAUNCH();
    return MSP_OK;
}

int direct_route_lists(msp_tree *t, const msp_fgt_params *prm, hipStream_t s) {
    if (t->n == 0) return MSP_OK;
    MSP_TRY(direct_route_counts(t, prm, s));
    if (!t->lists_valid) {
        MSP_TRY(direct_route_fill(t, prm, s));
        t->lists_valid = true;
    }
    return MSP_OK;
}

int direct_route(msp_tree *t, const msp_fgt_params *prm, hipStream_t s, bool lists_ready) {
    const int64_t nn = t->n_nodes;
    if (t->n == 0) return MSP_OK;
    if (!lists_ready) MSP_TRY(direct_route_lists(t, prm, s));
    BoxGeo geo{{t->geo.lo[0], t->geo.lo[1], t->geo.lo[2]}, t->geo.side};
    const float k_scale = (float)(std::sqrt(1.4426950408889634) / (double)prm->sigma);
    PhaseScope ps(&t->timing, PH_P2P, s);
    hipLaunchKernelGGL(k_p2p, dim3((unsigned)((nn + 3) / 4)), dim3(256), 0, s, nn, t->nfirst.as<int32_t>(),
                       t->ncount.as<int32_t>(), t->nnchild.as<int32_t>(), t->nlevel.as<int32_t>(),
                       t->nix.as<int32_t>(), t->niy.as<int32_t>(), t->niz.as<int32_t>(), geo,
                       t->list_off.as<int64_t>(), t->list_idx.as<int32_t>(), t->ps.as<float4>(),
                       t->tflag.as<uint8_t>(), k_scale, (prm->flags & MSP_EXCLUDE_SELF) ? 1 : 0,
                       t->usort.as<float>());
    MSP_CHECK_LAUNCH();
    return MSP_OK;
}

int direct_all_pairs(const float *tx, const float *ty, const float *tz, int64_t nt, const float *sx,
                     const float *sy, const float *sz, const float *w, int64_t ns, float sigma,
                     float *u, hipStream_t s) {
    if (nt == 0) return MSP_OK;
    const float neg_c = (float)(-1.4426950408889634 / ((double)sigma * sigma));
    hipLaunchKernelGGL(k_direct, dim3(grid_for(nt, kBlock)), dim3(kBlock), 0, s, tx, ty, tz, nt, sx,
                       sy, sz, w, ns, neg_c, u);
    MSP_CHECK_LAUNCH();
    return MSP_OK;
}

}  // namespace msp
