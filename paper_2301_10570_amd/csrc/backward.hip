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
#include "grad_common.hpp"

#include <cmath>

namespace msp {
namespace {

constexpr int kBlock = 256;

__global__ void k_target_weights(const float *g, const uint8_t *is_target, int64_t n, float *gt) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    gt[i] = (!is_target || is_target[i]) ? g[i] : 0.f;
}

// P2P with derivatives, one target leaf per block of one wavefront.
__global__ void __launch_bounds__(64) k_p2p_grad(GradLeafSet L, int stride, int want_lap) {
    __shared__ GradShared sh;
    p2p_grad_leaf(L, blockIdx.x, stride, want_lap, sh);
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
    if (j < n)
        ds = combine_point(reinterpret_cast<const float4 *>(rec + (int64_t)iperm[j] * kRec), gt[j],
                           want_pos ? w[j] : 0.f, want_w, want_pos, want_sigma, sigma, exclude_self,
                           want_w ? grad_w + j : nullptr, want_pos ? grad_x + j : nullptr,
                           want_pos ? grad_y + j : nullptr, want_pos ? grad_z + j : nullptr);
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
    const GradLeafSet L{nn, t->nfirst.as<int32_t>(), t->ncount.as<int32_t>(), t->nnchild.as<int32_t>(),
                        t->nlevel.as<int32_t>(), t->nix.as<int32_t>(), t->niy.as<int32_t>(), t->niz.as<int32_t>(),
                        geo, t->list_off.as<int64_t>(), t->list_idx.as<int32_t>(), t->ps.as<float4>(), kexp,
                        inv_s2, out};
    PhaseScope ps(&t->timing, PH_P2P, s);
    hipLaunchKernelGGL(k_p2p_grad, dim3((unsigned)nn), dim3(64), 0, s, L, stride, want_lap);
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
