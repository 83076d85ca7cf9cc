// Derivatives of L = sum_i g_i u(t_i) (targets i) with respect to the weights, the
// positions and sigma.  With K = exp(-|t - s|^2 / sigma^2):
//   dL/dw_j     = v(s_j),  v(x) = sum_i g_i K(t_i, x)          (the transposed sum)
//   dL/dx_k     = g_k grad u(x_k) + w_k grad v(x_k)             (a point may be both)
//   dL/dsigma   = sum_i g_i [ (sigma/2) lap u(t_i) + (3/sigma) u(t_i) ]
// using dK/dsigma = (sigma/2) lap_t K + (3/sigma) K (the heat equation of the
// Gaussian).  Two field evaluations give everything: u with gradient and
// Laplacian (weights w), and v with gradient (weights g at the targets), both by
// the expansion route (L2P with derivatives) or the direct route (P2P with
// derivatives).
#include "internal.hpp"

#include <cmath>

namespace msp {
namespace {

constexpr int kBlock = 256;
constexpr int kRec = 16;   // floats per point record of the backward pass (64 bytes)

__global__ void k_target_weights(const float *g, const uint8_t *is_target, int64_t n, float *gt) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    gt[i] = (!is_target || is_target[i]) ? g[i] : 0.f;
}

struct BoxGeo {
    double lo[3];
    double side;
};

__device__ inline void node_box(const BoxGeo &g, int level, int ix, int iy, int iz, float c[3]) {
    const double h = g.side / (double)(1ll << level);
    c[0] = (float)(g.lo[0] + (ix + 0.5) * h);
    c[1] = (float)(g.lo[1] + (iy + 0.5) * h);
    c[2] = (float)(g.lo[2] + (iz + 0.5) * h);
}

// P2P with derivatives: for every point of every leaf (key order), the sums over
// the source leaves of its list of e = w exp(-r^2/sigma^2), e*(x-s) and e*r^2.
__global__ void __launch_bounds__(64) k_p2p_grad(int64_t n_nodes, const int32_t *nfirst,
                                                 const int32_t *ncount, const int32_t *nnchild,
                                                 const int32_t *nlevel, const int32_t *nix,
                                                 const int32_t *niy, const int32_t *niz, BoxGeo geo,
                                                 const int64_t *off, const int32_t *lst,
                                                 const float4 *ps, float kexp, float inv_s2,
                                                 float *out, int stride, int want_lap) {
    const int64_t v = blockIdx.x;
    if (v >= n_nodes || nnchild[v] != 0) return;
    __shared__ float4 src[64];
    __shared__ float red[5][64];
    const int lane = threadIdx.x;
    float ct[3];
    node_box(geo, nlevel[v], nix[v], niy[v], niz[v], ct);
    const int32_t tf = nfirst[v], tn = ncount[v];
    const int64_t l0 = off[v], l1 = off[v + 1];
    for (int t0 = 0; t0 < tn; t0 += 64) {
        const int nt = tn - t0 < 64 ? tn - t0 : 64;
        int tp = 1;
        while (tp < nt) tp <<= 1;
        const int G = 64 / tp;
        const int a = lane % tp, grp = lane / tp;
        const int32_t ti = tf + t0 + (a < nt ? a : 0);
        const float4 qt = ps[ti];
        const float tx = qt.x - ct[0], ty = qt.y - ct[1], tz = qt.z - ct[2];
        float su = 0.f, sx = 0.f, sy = 0.f, sz = 0.f, sr = 0.f;
        for (int64_t q = l0; q < l1; ++q) {
            const int32_t u = lst[q];
            if (u < 0 || u >= n_nodes) continue;
            const int32_t sf = nfirst[u], sn = ncount[u];
            for (int s0 = 0; s0 < sn; s0 += 64) {
                const int ns = sn - s0 < 64 ? sn - s0 : 64;
                __syncthreads();
                if (lane < ns) {
                    const float4 qs = ps[sf + s0 + lane];
                    src[lane] = make_float4(qs.x - ct[0], qs.y - ct[1], qs.z - ct[2], qs.w);
                }
                __syncthreads();
                for (int j = grp; j < ns; j += G) {
                    const float4 s4 = src[j];
                    const float dx = tx - s4.x, dy = ty - s4.y, dz = tz - s4.z;
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    const float e = s4.w * __builtin_amdgcn_exp2f(r2 * kexp);
                    su += e;
                    sx = fmaf(e, dx, sx);
                    sy = fmaf(e, dy, sy);
                    sz = fmaf(e, dz, sz);
                    sr = fmaf(e, r2, sr);
                }
            }
        }
        __syncthreads();
        red[0][lane] = su; red[1][lane] = sx; red[2][lane] = sy; red[3][lane] = sz; red[4][lane] = sr;
        __syncthreads();
        if (grp == 0 && a < nt) {
            float r[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
            for (int q = 0; q < G; ++q)
                for (int k = 0; k < 5; ++k) r[k] += red[k][q * tp + a];
            float *o = out + (int64_t)ti * stride;   // value, gradient x y z, Laplacian
            o[0] = r[0];
            o[1] = -2.f * inv_s2 * r[1];
            o[2] = -2.f * inv_s2 * r[2];
            o[3] = -2.f * inv_s2 * r[3];
            if (want_lap) o[4] = 4.f * inv_s2 * inv_s2 * r[4] - 6.f * inv_s2 * r[0];
        }
    }
}

// Per point of the input order j: the key-order record of its point (64 bytes,
// one aligned segment: A value, gradient, Laplacian, then B value, gradient)
// combined into the gradients; per-block partial sums of the sigma derivative.
__global__ void k_combine(int64_t n, const int32_t *iperm, const float *gt, const float *w,
                          const float *rec, int want_w, int want_pos, int want_sigma, double sigma,
                          int exclude_self, float *grad_w, float *grad_x, float *grad_y, float *grad_z,
                          double *partial) {
    __shared__ double red[kBlock];
    const int64_t j = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    double ds = 0.0;
    if (j < n) {
        const float4 *r4 = reinterpret_cast<const float4 *>(rec + (int64_t)iperm[j] * kRec);
        const float4 a = r4[0], b = r4[1], c = r4[2];
        // a = (Av, Agx, Agy, Agz), b = (Alap, Bv, Bgx, Bgy), c = (Bgz, -, -, -)
        const float g = gt[j];
        if (want_w) grad_w[j] = exclude_self ? b.y - g : b.y;
        if (want_pos) {
            const float wj = w[j];
            grad_x[j] = g * a.y + wj * b.z;
            grad_y[j] = g * a.z + wj * b.w;
            grad_z[j] = g * a.w + wj * c.x;
        }
        if (want_sigma) ds = (double)g * (0.5 * sigma * (double)b.x + 3.0 / sigma * (double)a.x);
    }
    red[threadIdx.x] = ds;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0 && partial) partial[blockIdx.x] = red[0];
}

__global__ void k_sum_partials(const double *partial, int64_t m, double *out) {
    __shared__ double red[kBlock];
    double s = 0.0;
    for (int64_t k = threadIdx.x; k < m; k += kBlock) s += partial[k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

}  // namespace

int direct_field_grad(msp_tree *t, const msp_fgt_params *prm, float *out, int stride, int want_lap,
                      hipStream_t s) {
    // the leaf lists of the direct route are built (or reused) by direct_route's
    // list pass; ps.w holds the staged weights of this evaluation
    const int64_t nn = t->n_nodes;
    BoxGeo geo{{t->geo.lo[0], t->geo.lo[1], t->geo.lo[2]}, t->geo.side};
    const double sig = prm->sigma;
    const float kexp = (float)(-1.4426950408889634 / (sig * sig));
    const float inv_s2 = (float)(1.0 / (sig * sig));
    PhaseScope ps(&t->timing, PH_P2P, s);
    hipLaunchKernelGGL(k_p2p_grad, dim3((unsigned)nn), dim3(64), 0, s, nn, t->nfirst.as<int32_t>(),
                       t->ncount.as<int32_t>(), t->nnchild.as<int32_t>(), t->nlevel.as<int32_t>(),
                       t->nix.as<int32_t>(), t->niy.as<int32_t>(), t->niz.as<int32_t>(), geo,
                       t->list_off.as<int64_t>(), t->list_idx.as<int32_t>(), t->ps.as<float4>(), kexp,
                       inv_s2, out, stride, want_lap);
    MSP_CHECK_LAUNCH();
    return MSP_OK;
}

int fgt_backward(msp_tree *t, const float *w, const uint8_t *is_target, const msp_fgt_params *prm,
                 const float *grad_u, float *grad_w, float *grad_x, float *grad_y, float *grad_z,
                 double *grad_sigma, hipStream_t s) {
    const int64_t n = t->n;
    FgtPlan pl;
    MSP_TRY(plan_fgt(t, prm, &pl));
    const int64_t nb = n > 0 ? n : 1;
    const int64_t nblk = (nb + kBlock - 1) / kBlock;
    // scratch: one 64-byte record per point in key order (A: value, gradient,
    // Laplacian; B: value, gradient), gt in input order, block partials
    MSP_TRY(t->bwd.ensure((size_t)nb * kRec * 4 + (size_t)nb * 4 + (size_t)nblk * 8 + 64));
    float *rec = t->bwd.as<float>();
    float *gt = rec + (size_t)nb * kRec;
    double *partial = reinterpret_cast<double *>(gt + nb + (nb & 1));
    if (n == 0) {
        // a kernel rather than a memset, so that the sequence can be captured into a graph
        if (grad_sigma) {
            hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, partial, (int64_t)0, grad_sigma);
            MSP_CHECK_LAUNCH();
        }
        return MSP_OK;
    }
    const bool needA = grad_x || grad_sigma;
    const bool needB = grad_w || grad_x;
    MSP_TRY(ensure_iperm(t, s));
    hipLaunchKernelGGL(k_target_weights, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, grad_u, is_target,
                       n, gt);
    MSP_CHECK_LAUNCH();
    if (pl.route == MSP_ROUTE_FGT) {
        if (needA) MSP_TRY(fgt_field_grad(t, pl, prm, w, rec, kRec, grad_sigma ? 1 : 0, s));
        if (needB) MSP_TRY(fgt_field_grad(t, pl, prm, gt, rec + 5, kRec, 0, s));
    } else {
        msp_fgt_params q = *prm;
        q.flags &= ~(uint32_t)MSP_EXCLUDE_SELF;
        if (needA) {
            MSP_TRY(stage_inputs(t, w, nullptr, s));
            MSP_TRY(direct_route_lists(t, &q, s));
            MSP_TRY(direct_field_grad(t, &q, rec, kRec, grad_sigma ? 1 : 0, s));
        }
        if (needB) {
            MSP_TRY(stage_inputs(t, gt, nullptr, s));
            MSP_TRY(direct_route_lists(t, &q, s));
            MSP_TRY(direct_field_grad(t, &q, rec + 5, kRec, 0, s));
        }
    }
    {
        PhaseScope ps(&t->timing, PH_BACKWARD, s);
        hipLaunchKernelGGL(k_combine, dim3((unsigned)nblk), dim3(kBlock), 0, s, n, t->iperm.as<int32_t>(), gt,
                           w, rec, grad_w && needB ? 1 : 0, grad_x ? 1 : 0, grad_sigma ? 1 : 0,
                           (double)prm->sigma, (prm->flags & MSP_EXCLUDE_SELF) ? 1 : 0, grad_w, grad_x,
                           grad_y, grad_z, partial);
        MSP_CHECK_LAUNCH();
        if (grad_sigma) {
            hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, partial, nblk, grad_sigma);
            MSP_CHECK_LAUNCH();
        }
    }
    return MSP_OK;
}

}  // namespace msp
