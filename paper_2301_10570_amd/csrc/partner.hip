// Child probabilities for proportional partner choice (Algorithm 2).
//
// For a query (target t, node X) the attraction of child c of X is the restricted
// sum S_c = sum_{j below c} w_j exp(-|t - s_j|^2 / sigma^2).  Algorithm 2 evaluates
// it directly, by a Hermite expansion, or by a Taylor expansion depending on the
// numbers of elements involved (thresholds c1 = c2 = 70).  For a single target
// the Taylor form reduces to a direct sum, so here a node is evaluated
//   - from its Hermite moments (M2P, Eq. (7)) when it holds more than c1 = 70
//     sources, is small enough for p terms (half-side <= rho_max(p) sigma), and
//     the target is close enough that the truncation stays within 1e-5 of the
//     node's own contribution;
//   - directly (Eq. (8)) when it is a leaf;
//   - otherwise through its children.
//
// Far queries produce sums far below the float32 range, so the sums are
// accumulated in float64: each exponential 2^-a is formed as a float32 exp2 of
// the fraction of a, scaled by 2^-floor(a).  A cutoff drops nodes whose box lies
// more than cutoff_sigmas*sigma beyond the distance d0 from the target to X.
//
// Node moments come from a bottom-up pass over the levels that may carry them:
// a node's moments are the P2M of the points of its children that carry none,
// plus the M2M shift of the moments of those that do (separable:
// A'_a = sum_{g<=a} A_g d^(a-g)/(a-g)! along each axis, d = (c_child - c_node)/sigma).
#include "internal.hpp"

#include <cmath>

namespace msp {

double rho_max_for_p(int p);

namespace {

constexpr int kBlock = 256;
constexpr int kC1 = 70;                    // Algorithm 2's element threshold
constexpr int kStack = 8 * (kDepth + 2);
constexpr double kAdmitTol = 1e-5;   // M2P error vs the node's own smallest contribution
constexpr double kRunTol = 1e-7;     // M2P error vs the running total of the query
constexpr double kSkipTol = 1e-12;   // dropped node's largest contribution vs the running total

// Sources below the nodes of one level: leaves count their points, inner nodes
// add up their children (levels are processed from the deepest up).
__global__ void k_nsrc_level(int64_t v0, int64_t v1, const int32_t *nfirst, const int32_t *ncount,
                             const int32_t *nfchild, const int32_t *nnchild, const float4 *ps,
                             int32_t *nsrc) {
    const int64_t v = v0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= v1) return;
    const int32_t nc = nnchild[v];
    int32_t k = 0;
    if (nc == 0) {
        const int32_t f = nfirst[v], c = ncount[v];
        for (int32_t j = f; j < f + c; ++j) k += ps[j].w != 0.f;
    } else {
        const int32_t fc = nfchild[v];
        for (int q = 0; q < nc; ++q) k += nsrc[fc + q];
    }
    nsrc[v] = k;
}

// One block per node of one level (v0 .. v0 + gridDim.x).  Nodes must be
// processed from the deepest level upward.
template <int P>
__global__ void __launch_bounds__(kBlock)
k_node_moments(int64_t v0, int level, int lh, const int32_t *nfirst, const int32_t *ncount,
               const int32_t *nfchild, const int32_t *nnchild, const int32_t *nix,
               const int32_t *niy, const int32_t *niz, const int32_t *ndigit, double lox,
               double loy, double loz, double side, const float4 *ps, double inv_sigma,
               int32_t *nsrc, uint8_t *hasA,
               float *nodeA, int64_t slot0) {
    constexpr int P2 = P * P, P3 = P * P * P;
    constexpr int NG = kBlock / P2 > 0 ? kBlock / P2 : 1;
    constexpr int STR = 3 * P + 1;
    constexpr int CH = P >= 11 ? 64 : kBlock;      // points staged per round (LDS budget)
    __shared__ float pts[(CH * STR > P3) ? CH * STR : P3];   // reused as bufB for M2M
    __shared__ float tot[P3];
    __shared__ float bufA[P3];
    float *bufB = pts;
    __shared__ float red[NG > 1 ? NG * P2 * P : 1];
    __shared__ float shift[3][P];

    const int64_t v = v0 + blockIdx.x;
    const int tid = threadIdx.x;
    const int32_t nc = nnchild[v];
    const int32_t f = nfirst[v], cnt = ncount[v];
    const bool want = level >= lh && nsrc[v] > kC1;
    if (tid == 0) hasA[v] = want ? 1 : 0;
    if (!want) return;

    const double h = side / (double)(1ll << level);
    const double cx = lox + (nix[v] + 0.5) * h, cy = loy + (niy[v] + 0.5) * h, cz = loz + (niz[v] + 0.5) * h;
    const int grp = tid / P2, yz = tid % P2, ay = yz % P, az = yz / P;
    const bool active = grp < NG;
    float acc[P];
#pragma unroll
    for (int k = 0; k < P; ++k) acc[k] = 0.f;

    // P2M over the points of children that carry no moments (all points for a leaf)
    const int nparts = nc == 0 ? 1 : nc;
    for (int q = 0; q < nparts; ++q) {
        int32_t pf = f, pn = cnt;
        if (nc > 0) {
            const int32_t c = nfchild[v] + q;
            if (hasA[c]) continue;
            pf = nfirst[c];
            pn = ncount[c];
        }
        for (int32_t c0 = 0; c0 < pn; c0 += CH) {
            const int32_t i = pf + c0 + tid;
            __syncthreads();
            if (tid < CH && c0 + tid < pn) {
                const float4 qp = ps[i];
                const float X = (float)(((double)qp.x - cx) * inv_sigma);
                const float Y = (float)(((double)qp.y - cy) * inv_sigma);
                const float Z = (float)(((double)qp.z - cz) * inv_sigma);
                float *r = pts + tid * STR;
                float px = qp.w, py = 1.f, pz = 1.f;
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    r[k] = px; r[P + k] = py; r[2 * P + k] = pz;
                    px *= X; py *= Y; pz *= Z;
                }
            }
            __syncthreads();
            const int m = pn - c0 < CH ? pn - c0 : CH;
            if (active)
                for (int j = grp; j < m; j += NG) {
                    const float *r = pts + j * STR;
                    const float fyz = r[P + ay] * r[2 * P + az];
#pragma unroll
                    for (int k = 0; k < P; ++k) acc[k] = fmaf(fyz, r[k], acc[k]);
                }
        }
    }
    __syncthreads();
    if (NG > 1) {
        if (active)
#pragma unroll
            for (int k = 0; k < P; ++k) red[(grp * P2 + yz) * P + k] = acc[k];
        __syncthreads();
    }
    if (grp == 0) {
        float fy = 1.f, fz = 1.f;
        for (int k = 2; k <= ay; ++k) fy *= (float)k;
        for (int k = 2; k <= az; ++k) fz *= (float)k;
        float fx = 1.f;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            if (k > 1) fx *= (float)k;
            float s = acc[k];
            if (NG > 1) {
                s = 0.f;
                for (int q = 0; q < NG; ++q) s += red[(q * P2 + yz) * P + k];
            }
            tot[(az * P + ay) * P + k] = s / (fx * fy * fz);
        }
    }
    __syncthreads();

    // M2M of the children that carry moments
    if (nc > 0) {
        const double hc = 0.5 * h;
        for (int q = 0; q < nc; ++q) {
            const int32_t c = nfchild[v] + q;
            if (!hasA[c]) continue;
            const float *Ac = nodeA + (int64_t)(c - slot0) * P3;
            for (int e = tid; e < P3; e += kBlock) bufA[e] = Ac[e];
            if (tid < 3 * P) {
                const int axis = tid / P, k = tid % P;
                const int bit = (ndigit[c] >> (2 - axis)) & 1;
                const double d = (bit - 0.5) * hc * inv_sigma;
                double val = 1.0;
                for (int m = 1; m <= k; ++m) val *= d / m;      // d^k / k!
                shift[axis][k] = (float)val;
            }
            __syncthreads();
            // x: bufB[az][ay][ax] = sum_{g<=ax} bufA[az][ay][g] shift_x[ax-g]
            for (int e = tid; e < P3; e += kBlock) {
                const int ax = e % P, rowb = e - ax;
                float s = 0.f;
                for (int g = 0; g <= ax; ++g) s = fmaf(bufA[rowb + g], shift[0][ax - g], s);
                bufB[e] = s;
            }
            __syncthreads();
            for (int e = tid; e < P3; e += kBlock) {
                const int ax = e % P, ay2 = (e / P) % P, az2 = e / P2;
                float s = 0.f;
                for (int g = 0; g <= ay2; ++g) s = fmaf(bufB[(az2 * P + g) * P + ax], shift[1][ay2 - g], s);
                bufA[e] = s;
            }
            __syncthreads();
            for (int e = tid; e < P3; e += kBlock) {
                const int rest = e % P2, az2 = e / P2;
                float s = 0.f;
                for (int g = 0; g <= az2; ++g) s = fmaf(bufA[g * P2 + rest], shift[2][az2 - g], s);
                tot[e] += s;
            }
            __syncthreads();
        }
    }
    float *dst = nodeA + (v - slot0) * P3;
    for (int e = tid; e < P3; e += kBlock) dst[e] = tot[e];
}

__device__ inline double wave_sum(double x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// 2^-a for a >= 0 over the float64 range.
__device__ inline double exp2_neg(double a) {
    const double n = floor(a);
    return ldexp((double)__builtin_amdgcn_exp2f(-(float)(a - n)), -(int)fmin(n, 2000.0));
}

// One wavefront (block of 64) per query.  Children of X are taken nearest
// first, and every walk pushes a node's children so that the nearest is popped
// first; the running total R of what has been summed so far then bounds every
// later decision from below:
//   - a node carrying moments is evaluated by M2P when the truncation model is
//     within kAdmitTol of its own smallest contribution, or within kRunTol of R;
//   - a node carrying moments whose largest possible contribution is below
//     kSkipTol * R is dropped.
template <int P>
__global__ void __launch_bounds__(64)
k_partner(int64_t nq, const int32_t *target_idx, const int32_t *node_id, const float *uniforms,
          int64_t n, int64_t n_nodes, const int32_t *iperm, const int32_t *nlevel,
          const int32_t *nfirst, const int32_t *ncount, const int32_t *nfchild,
          const int32_t *nnchild, const int32_t *ndigit, const int32_t *nix, const int32_t *niy,
          const int32_t *niz, double lox, double loy, double loz, double side, const float4 *ps,
          const uint8_t *hasA, const float *nodeA, int64_t slot0, int lh, double sigma, float cutoff2,
          int unlimited, float rho_ref, int exclude_self, float *probs, int32_t *choice) {
    constexpr int P3 = P * P * P;
    __shared__ int32_t stk[kStack];
    __shared__ float hfun[3][P];
    __shared__ double S[8];
    __shared__ int32_t cid[8];
    __shared__ int32_t order[8];
    __shared__ double dist[8];
    const int64_t q = blockIdx.x;
    const int lane = threadIdx.x;
    if (q >= nq) return;
    const int32_t ti = target_idx[q], X = node_id[q];
    if (lane < 8) { S[lane] = 0.0; cid[lane] = -1; }
    const bool ok = ti >= 0 && ti < n && X >= 0 && X < n_nodes;
    const int nc = ok ? nnchild[X] : 0;
    __syncthreads();
    if (nc == 0) {
        if (lane < 8) probs[q * 8 + lane] = 0.f;
        if (lane == 0 && choice) choice[q] = -1;
        return;
    }
    const int32_t si = iperm[ti];
    const float4 qt = ps[si];
    const double tx = qt.x, ty = qt.y, tz = qt.z;
    const double inv_sigma = 1.0 / sigma;
    const double kexp = 1.4426950408889634 / (sigma * sigma);
    // squared distance from the target to a node's box
    auto box_d2 = [&](int32_t u, double &cxo, double &cyo, double &czo, double &half) {
        const int l = nlevel[u];
        const double h = side / (double)(1ll << l);
        cxo = lox + (nix[u] + 0.5) * h;
        cyo = loy + (niy[u] + 0.5) * h;
        czo = loz + (niz[u] + 0.5) * h;
        half = 0.5 * h;
        const double gx = fmax(fabs(tx - cxo) - half, 0.0), gy = fmax(fabs(ty - cyo) - half, 0.0),
                     gz = fmax(fabs(tz - czo) - half, 0.0);
        return gx * gx + gy * gy + gz * gz;
    };
    double d0sq, dum0, dum1, dum2, dum3;
    d0sq = box_d2(X, dum0, dum1, dum2, dum3);
    const double reach = unlimited ? 0.0 : sqrt(d0sq) + sqrt((double)cutoff2);
    const int32_t fc = nfchild[X];
    // children of X nearest first (ties by index)
    if (lane < nc) {
        double a, b, c, h;
        dist[lane] = box_d2(fc + lane, a, b, c, h);
    }
    __syncthreads();
    if (lane < nc) {
        int rank = 0;
        for (int k = 0; k < nc; ++k)
            rank += (dist[k] < dist[lane]) || (dist[k] == dist[lane] && k < lane);
        order[rank] = lane;
    }
    __syncthreads();
    double run = 0.0;   // wave-uniform running total
    for (int ci = 0; ci < nc; ++ci) {
        const int32_t child = fc + order[ci];
        double csum = 0.0;
        int sp = 0;
        if (lane == 0) stk[0] = child;
        sp = 1;
        __syncthreads();
        while (sp > 0) {
            const int32_t u = stk[sp - 1];
            __syncthreads();
            --sp;
            double ux, uy, uz, half;
            const double g2 = box_d2(u, ux, uy, uz, half);
            if (!unlimited && g2 > reach * reach) continue;
            const int32_t uf = nfirst[u], un = ncount[u], unc = nnchild[u];
            const double dx = tx - ux, dy = ty - uy, dz = tz - uz;
            bool use_m = false;
            const float *A = nullptr;
            if (hasA[u]) {
                A = nodeA + (int64_t)(u - slot0) * P3;
                const double wsum = fabs((double)A[0]);
                // largest possible contribution: every source at the box's nearest point
                if (wsum * exp2_neg(g2 * kexp) <= kSkipTol * run) continue;
                const double rho = half * inv_sigma;
                const double r = sqrt(dx * dx + dy * dy + dz * dz) * inv_sigma;
                const double model = 2e-5 * pow(rho / rho_ref, (double)P);
                const double rel = model * exp(0.5 * r * r + 2.0 * 1.7320508075688772 * rho * r + 3.0 * rho * rho);
                const double abs_err = model * wsum * exp(-0.5 * r * r);
                use_m = rel <= kAdmitTol || abs_err <= kRunTol * run;
            }
            double part = 0.0;
            if (use_m) {
                if (lane < 3 * P) {
                    const int axis = lane / P, k = lane % P;
                    const double yv = (axis == 0 ? dx : axis == 1 ? dy : dz) * inv_sigma;
                    double h0 = exp(-yv * yv), hk = h0;
                    if (k >= 1) {
                        hk = 2.0 * yv * h0;
                        for (int m = 1; m < k; ++m) {
                            const double hn = 2.0 * yv * hk - 2.0 * m * h0;
                            h0 = hk;
                            hk = hn;
                        }
                    }
                    hfun[axis][k] = (float)hk;
                }
                __syncthreads();
                float mp = 0.f;
                for (int e = lane; e < P3; e += 64) {
                    const int ax = e % P, ay = (e / P) % P, az = e / (P * P);
                    mp = fmaf(A[e], hfun[0][ax] * hfun[1][ay] * hfun[2][az], mp);
                }
                // the query's own point inside this node contributes w_self * K(0)
                if (exclude_self && lane == 0 && si >= uf && si < uf + un) mp -= qt.w;
                part = (double)mp;
                __syncthreads();
            } else if (unc == 0) {
                for (int32_t j = uf + lane; j < uf + un; j += 64) {
                    const float4 qj = ps[j];
                    if (qj.w == 0.f || (exclude_self && j == si)) continue;
                    const double ex = tx - qj.x, ey = ty - qj.y, ez = tz - qj.z;
                    part += (double)qj.w * exp2_neg((ex * ex + ey * ey + ez * ez) * kexp);
                }
            } else {
                // push the children farthest first so that the nearest is popped first
                const int32_t f = nfchild[u];
                if (f > u && f + unc <= n_nodes && sp + unc <= kStack) {
                    double cd = 0.0;
                    if (lane < unc) {
                        double a, b, c, h;
                        cd = box_d2(f + lane, a, b, c, h);
                    }
                    if (lane < 8) dist[lane] = cd;
                    __syncthreads();
                    if (lane < unc) {
                        int rank = 0;   // number of children farther away (ties: larger index first)
                        for (int k = 0; k < unc; ++k)
                            rank += (dist[k] > cd) || (dist[k] == cd && k > lane);
                        stk[sp + rank] = f + lane;
                    }
                    sp += unc;
                }
                __syncthreads();
                continue;
            }
            const double node_sum = wave_sum(part);
            csum += node_sum;
            run += node_sum;
        }
        if (lane == 0) {
            S[ndigit[child]] = csum;
            cid[ndigit[child]] = child;
        }
        __syncthreads();
    }
    double total = 0.0;
    for (int d = 0; d < 8; ++d) total += S[d];
    if (lane < 8) probs[q * 8 + lane] = total > 0.0 ? (float)(S[lane] / total) : 0.f;
    if (lane == 0 && choice) {
        int32_t pick = -1;
        if (total > 0.0 && uniforms) {
            const double target = (double)uniforms[q] * total;
            double acc = 0.0;
            int32_t last = -1;
            for (int d = 0; d < 8; ++d) {
                if (S[d] > 0.0) last = cid[d];
                acc += S[d];
                if (acc > target && S[d] > 0.0) { pick = cid[d]; break; }
            }
            if (pick < 0) pick = last;
        }
        choice[q] = pick;
    }
}

template <int P>
int run_partner(msp_tree *t, const msp_fgt_params *prm, const int32_t *target_idx,
                const int32_t *node_id, int64_t nq, const float *uniforms, float *probs,
                int32_t *choice, hipStream_t s) {
    const double sigma = prm->sigma;
    const double rmax = rho_max_for_p(P);
    int lh = kDepth;
    for (int l = 0; l <= kDepth; ++l)
        if (t->geo.side / std::ldexp(1.0, l + 1) / sigma <= rmax) { lh = l; break; }
    const int64_t nn = t->n_nodes;
    const int64_t slot0 = t->level_off[lh < kMaxLevels ? lh : kDepth + 1];
    const int64_t nslots = nn - slot0;
    MSP_TRY(t->node_hasA.ensure(nn));
    MSP_TRY(t->node_nsrc.ensure(nn * 4));
    MSP_TRY(t->nodeA.ensure((size_t)(nslots > 0 ? nslots : 1) * P * P * P * 4));
    MSP_HIP(hipMemsetAsync(t->node_hasA.p, 0, nn, s));
    {
        PhaseScope ps(&t->timing, PH_NODE_MOMENTS, s);
        for (int l = t->depth; l >= lh && l >= 0; --l) {
            const int64_t a = t->level_off[l], b = t->level_off[l + 1];
            if (b <= a) continue;
            hipLaunchKernelGGL(k_nsrc_level, dim3(grid_for(b - a, kBlock)), dim3(kBlock), 0, s, a, b,
                               t->nfirst.as<int32_t>(), t->ncount.as<int32_t>(), t->nfchild.as<int32_t>(),
                               t->nnchild.as<int32_t>(), t->ps.as<float4>(), t->node_nsrc.as<int32_t>());
            MSP_CHECK_LAUNCH();
        }
        for (int l = t->depth; l >= 0; --l) {
            const int64_t a = t->level_off[l], b = t->level_off[l + 1];
            if (b <= a) continue;
            if (l < lh) break;
            // the deepest level holds only leaves, which never exceed leaf_max points
            if (l == t->depth && t->leaf_max <= kC1 && l < t->max_depth) continue;
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_node_moments<P>), dim3((unsigned)(b - a)), dim3(kBlock),
                               0, s, a, l, lh, t->nfirst.as<int32_t>(), t->ncount.as<int32_t>(),
                               t->nfchild.as<int32_t>(), t->nnchild.as<int32_t>(), t->nix.as<int32_t>(),
                               t->niy.as<int32_t>(), t->niz.as<int32_t>(), t->ndigit.as<int32_t>(),
                               t->geo.lo[0], t->geo.lo[1], t->geo.lo[2], t->geo.side, t->ps.as<float4>(), 1.0 / sigma,
                               t->node_nsrc.as<int32_t>(), t->node_hasA.as<uint8_t>(),
                               t->nodeA.as<float>(), slot0);
            MSP_CHECK_LAUNCH();
        }
    }
    t->node_moments_level = lh;
    t->node_moments_p = P;
    t->node_moments_bytes = (int64_t)(nslots > 0 ? nslots : 0) * P * P * P * 4;
    if (nq == 0) return MSP_OK;
    const bool unlimited = !(prm->cutoff_sigmas > 0.f);
    const float R = unlimited ? 0.f : (float)(prm->cutoff_sigmas * sigma);
    PhaseScope ps(&t->timing, PH_PARTNER, s);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_partner<P>), dim3((unsigned)nq), dim3(64), 0, s, nq, target_idx,
                       node_id, uniforms, t->n, nn, t->iperm.as<int32_t>(), t->nlevel.as<int32_t>(),
                       t->nfirst.as<int32_t>(), t->ncount.as<int32_t>(), t->nfchild.as<int32_t>(),
                       t->nnchild.as<int32_t>(), t->ndigit.as<int32_t>(), t->nix.as<int32_t>(),
                       t->niy.as<int32_t>(), t->niz.as<int32_t>(), t->geo.lo[0], t->geo.lo[1],
                       t->geo.lo[2], t->geo.side, t->ps.as<float4>(), t->node_hasA.as<uint8_t>(), t->nodeA.as<float>(), slot0, lh,
                       sigma, R * R, unlimited ? 1 : 0, (float)rmax,
                       (prm->flags & MSP_EXCLUDE_SELF) ? 1 : 0, probs, choice);
    MSP_CHECK_LAUNCH();
    return MSP_OK;
}

}  // namespace

int partner_probabilities(msp_tree *t, const float *w, const msp_fgt_params *prm,
                          const int32_t *target_idx, const int32_t *node_id, int64_t nq,
                          const float *uniforms, float *probs, int32_t *choice, hipStream_t s) {
    if (t->n == 0) {
        if (nq > 0) return fail(MSP_EINVAL, "partner queries on an empty tree");
        return MSP_OK;
    }
    MSP_TRY(stage_inputs(t, w, nullptr, s));
    MSP_TRY(ensure_iperm(t, s));
    switch (prm->p) {
#define CASE(P) case P: return run_partner<P>(t, prm, target_idx, node_id, nq, uniforms, probs, choice, s);
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
        CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16)
#undef CASE
    }
    return fail(MSP_EINVAL, "p out of range");
}

}  // namespace msp
