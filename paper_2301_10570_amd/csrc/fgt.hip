// Expansion route of the forward sum: Hermite moments per cell (P2M, Eq. (7)),
// Hermite-to-Taylor translation between every pair of cells of one octree level
// (M2L), and evaluation of each cell's Taylor series at its targets (L2P, Eq. (6)).
//
// Multi-index notation as in the paper (Eqs. (3)-(5)), tensor range 0 <= n_k < p.
// With h_n(x) = (-1)^n d^n/dx^n exp(-x^2) and cell centres c:
//   P2M  A_a = 1/a! sum_j w_j ((s_j - c_S)/sigma)^a
//   M2L  C_b = (-1)^|b| / b! sum_a A_a h_{a+b}((c_T - c_S)/sigma)
//   L2P  u(t) = sum_b C_b ((t - c_T)/sigma)^b
//
// Because h_{a+b}(x) is a product over the three axes and the cell offset
// c_T - c_S is an integer multiple of the cell side, the translation from every
// cell of the grid to every cell is three 1-D block-Toeplitz matrix products, one
// per axis:  Out[(t,b)][rest] = sum_{(s,a)} T_k[t-s][b][a] In[(s,a)][rest] with
// T_k[o][b][a] = (-1)^b / b! h_{a+b}(o * cell / sigma).  Each pass contracts the
// last index of a row-major tensor and writes its result transposed, so three
// passes return the tensor to its original index order.  All pairs of cells are
// included (no cutoff); operator entries for far offsets underflow to zero.
#include "internal.hpp"

#include <cmath>

namespace msp {

// Cell half-side / sigma at which the transform of p terms per axis keeps the
// per-target relative error of the FP64 transform near 2e-5 on uniform test
// clouds (measured by brute force against the direct sum; the Cramer-type
// bound is far more pessimistic).  Index p - 1.
static const double kRhoMax[kMaxP] = {2e-5, 0.004, 0.025, 0.07, 0.16, 0.25, 0.34, 0.42,
                                      0.50, 0.60, 0.64, 0.68, 0.70, 0.70, 0.70, 0.70};

double rho_max_for_p(int p) { return kRhoMax[p - 1]; }

namespace {

constexpr int kBlock = 256;

// T_k[o][b][a] = (-1)^b / b! * h_{a+b}(o * step), o = -(G_k-1) .. G_k-1, for the three
// axes in one launch (thread -> axis, offset); computed in float64, stored as float32.
__global__ void k_m2l_ops(int p, int Gx, int Gy, int Gz, double step, float *ox, float *oy, float *oz) {
    int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int nx = 2 * Gx - 1, ny = 2 * Gy - 1, nz = 2 * Gz - 1;
    int G;
    float *out;
    if (t < nx) { G = Gx; out = ox; }
    else if (t < nx + ny) { t -= nx; G = Gy; out = oy; }
    else if (t < nx + ny + nz) { t -= nx + ny; G = Gz; out = oz; }
    else return;
    const int o = t - (G - 1);
    const double x = o * step;
    double h[2 * kMaxP];
    h[0] = exp(-x * x);
    if (2 * p - 1 > 1) h[1] = 2.0 * x * h[0];
    for (int n = 1; n + 1 < 2 * p - 1; ++n) h[n + 1] = 2.0 * x * h[n] - 2.0 * n * h[n - 1];
    float *T = out + (size_t)t * p * p;
    double inv_fact = 1.0;
    for (int b = 0; b < p; ++b) {
        if (b > 0) inv_fact /= b;
        const double sgn = (b & 1) ? -inv_fact : inv_fact;
        for (int a = 0; a < p; ++a) T[b * p + a] = (float)(sgn * h[a + b]);
    }
}

// Point range of a grid cell: the points whose level-`level` key prefix is the
// cell's Morton code (contiguous in key order).
__device__ inline void cell_range(const uint64_t *keys, int64_t n, int level, int kx, int ky, int kz,
                                  int64_t &start, int64_t &end) {
    const int sh = 3 * (kDepth - level);
    const uint64_t prefix = morton3((uint32_t)kx, (uint32_t)ky, (uint32_t)kz);
    start = lower_bound_u64(keys, 0, n, prefix << sh);
    end = lower_bound_u64(keys, start, n, (prefix + 1ull) << sh);
}

// One block per cell of the grid; moments written in the grid layout
// [kz][az][ky][ay][kx][ax].  Lane l of a wave owns az = l % P and handles every
// (64/P)-th point of the wave's share; it keeps the P x P moments (ax, ay) of its
// az in registers.  Partial moments are added in a fixed order (lanes, then waves).
template <int P>
__global__ void __launch_bounds__(kBlock) k_p2m(const uint64_t *keys, int64_t n, const float4 *ps,
                                                const int32_t *perm, const float *w,
                                                int level, int Gx, int Gy, int Gz, double lox,
                                                double loy, double loz, double cell,
                                                double inv_sigma, float *A) {
    constexpr int P3 = P * P * P;
    constexpr int PL = 64 / P;            // point lanes per wave
    constexpr int NW = kBlock / 64;
    constexpr int NB = P <= 12 ? NW : 1;  // partial buffers (LDS budget for large P)
    __shared__ float red[NB][P3];
    const int64_t g = blockIdx.x;
    const int kx = (int)(g % Gx), ky = (int)((g / Gx) % Gy), kz = (int)(g / ((int64_t)Gx * Gy));
    int64_t start, end;
    cell_range(keys, n, level, kx, ky, kz, start, end);
    const double cx = lox + (kx + 0.5) * cell, cy = loy + (ky + 0.5) * cell, cz = loz + (kz + 0.5) * cell;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int az = lane % P, pl = lane / P;
    const bool active = pl < PL;
    float acc[P][P];
#pragma unroll
    for (int a = 0; a < P; ++a)
#pragma unroll
        for (int b = 0; b < P; ++b) acc[a][b] = 0.f;
    if (active) {
        for (int64_t j = start + wid * PL + pl; j < end; j += NW * PL) {
            const float4 q = ps[j];
            const float X = (float)(((double)q.x - cx) * inv_sigma);
            const float Y = (float)(((double)q.y - cy) * inv_sigma);
            const float Z = (float)(((double)q.z - cz) * inv_sigma);
            float zw = w[perm[j]];
#pragma unroll
            for (int k = 1; k < P; ++k) zw = k <= az ? zw * Z : zw;
            float px[P], yz[P];
            px[0] = 1.f;
            yz[0] = zw;
#pragma unroll
            for (int k = 1; k < P; ++k) {
                px[k] = px[k - 1] * X;
                yz[k] = yz[k - 1] * Y;
            }
#pragma unroll
            for (int a = 0; a < P; ++a)
#pragma unroll
                for (int b = 0; b < P; ++b) acc[a][b] = fmaf(px[a], yz[b], acc[a][b]);
        }
    }
    // lanes with the same az in point-lane order (per wave, or waves in turn)
    for (int e = tid; e < NB * P3; e += kBlock) (&red[0][0])[e] = 0.f;
    __syncthreads();
    const int wb = NB == NW ? wid : 0;
    for (int w = 0; w < NW / NB; ++w) {
        for (int r = 0; r < PL; ++r) {
            if (active && pl == r && (NB == NW || wid == w)) {
#pragma unroll
                for (int b = 0; b < P; ++b)
#pragma unroll
                    for (int a = 0; a < P; ++a) red[wb][(az * P + b) * P + a] += acc[a][b];
            }
            __syncthreads();
        }
    }
    // waves in order, then 1/(ax! ay! az!) and the grid layout
    const int64_t Rx = (int64_t)Gx * P, Ry = (int64_t)Gy * P;
    for (int e = tid; e < P3; e += kBlock) {
        float s = 0.f;
#pragma unroll
        for (int w = 0; w < NB; ++w) s += red[w][e];
        const int ax = e % P, ay = (e / P) % P, zz = e / (P * P);
        float f = 1.f;
        for (int k = 2; k <= ax; ++k) f *= (float)k;
        for (int k = 2; k <= ay; ++k) f *= (float)k;
        for (int k = 2; k <= zz; ++k) f *= (float)k;
        A[(((int64_t)kz * P + zz) * Ry + (int64_t)ky * P + ay) * Rx + (int64_t)kx * P + ax] = s / f;
    }
}

// Out[v][r] = sum_u In[r][u] * T[(v/p) - (u/p) + G - 1][v%p][u%p], u, v in [0, G*p).
constexpr int TR = 64, TV = 64, TK = 16;
__global__ void __launch_bounds__(kBlock) k_m2l_pass(const float *In, float *Out, int64_t R, int p,
                                                     int G, const float *T) {
    __shared__ float sIn[TK][TR + 4];
    __shared__ float sM[TK][TV + 4];
    const int U = G * p;
    const int64_t r0 = (int64_t)blockIdx.x * TR;
    const int v0 = blockIdx.y * TV;
    const int tid = threadIdx.x;
    const int tr = tid % 16, tv = tid / 16;
    float acc[4][4] = {};
    for (int u0 = 0; u0 < U; u0 += TK) {
        for (int e = tid; e < TR * TK; e += kBlock) {
            const int rr = e / TK, kk = e % TK;
            const int64_t r = r0 + rr;
            const int u = u0 + kk;
            sIn[kk][rr] = (r < R && u < U) ? In[r * U + u] : 0.f;
        }
        for (int e = tid; e < TV * TK; e += kBlock) {
            const int vv = e / TK, kk = e % TK;
            const int v = v0 + vv, u = u0 + kk;
            float m = 0.f;
            if (v < U && u < U) {
                const int t = v / p, b = v % p, s = u / p, a = u % p;
                m = T[((size_t)(t - s + G - 1) * p + b) * p + a];
            }
            sM[kk][vv] = m;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TK; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = sIn[kk][tr * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = sM[kk][tv * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int v = v0 + tv * 4 + j;
        if (v >= U) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t r = r0 + tr * 4 + i;
            if (r < R) Out[(int64_t)v * R + r] = acc[i][j];
        }
    }
}

// The same pass on the matrix cores: D[v][r] = sum_u M[v][u] In[r][u] with
// v_mfma_f32_16x16x4f32 (A = operator tile, B = input tile, both staged in LDS).
// One wavefront per 32 x 32 tile of D, built from 2 x 2 MFMA tiles; K steps of 16.
// Lane layout of the 16x16x4 instruction: lane l supplies A[l%16][l/16] and
// B[l/16][l%16] and receives D[4*(l/16) + i][l%16], i = 0..3.
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int MT = 32, MK = 16;
__global__ void __launch_bounds__(64) k_m2l_pass_mfma(const float *In, float *Out, int64_t R, int p,
                                                      int G, const float *T) {
    __shared__ float sA[MT][MK + 1];   // operator rows v, columns u
    __shared__ float sB[MT][MK + 1];   // input rows r, columns u
    const int U = G * p;
    const int64_t r0 = (int64_t)blockIdx.x * MT;
    const int v0 = blockIdx.y * MT;
    const int lane = threadIdx.x;
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int u0 = 0; u0 < U; u0 += MK) {
#pragma unroll
        for (int e = lane; e < MT * MK; e += 64) {
            const int row = e / MK, kk = e % MK;
            const int u = u0 + kk;
            const int v = v0 + row;
            float m = 0.f;
            if (v < U && u < U) {
                const int t = v / p, b = v % p, sI = u / p, a = u % p;
                m = T[((size_t)(t - sI + G - 1) * p + b) * p + a];
            }
            sA[row][kk] = m;
            const int64_t r = r0 + row;
            sB[row][kk] = (r < R && u < U) ? In[r * U + u] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int k4 = 0; k4 < MK; k4 += 4) {
            const int kk = k4 + (lane >> 4), rr = lane & 15;
            const float a0 = sA[rr][kk], a1 = sA[16 + rr][kk];
            const float b0 = sB[rr][kk], b1 = sB[16 + rr][kk];
            acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int v = v0 + 16 * a + 4 * (lane >> 4) + i;
                const int64_t r = r0 + 16 * b + (lane & 15);
                if (v < U && r < R) Out[(int64_t)v * R + r] = acc[a][b][i];
            }
}

// One block per cell: evaluate the cell's Taylor series at its targets (Horner
// in x, then y, then z), two targets per thread so that every coefficient read
// from LDS feeds two multiply-adds.
template <int P>
__global__ void __launch_bounds__(kBlock) k_l2p(const uint64_t *keys, int64_t n, const float4 *ps,
                                                const int32_t *perm, const uint8_t *is_target,
                                                const float *w, int subtract_self, int level, int Gx,
                                                int Gy, int Gz, double lox, double loy, double loz,
                                                double cell, double inv_sigma, const float *C,
                                                float *u_out) {
    constexpr int P3 = P * P * P;
    __shared__ float sC[P3];
    const int64_t g = blockIdx.x;
    const int kx = (int)(g % Gx), ky = (int)((g / Gx) % Gy), kz = (int)(g / ((int64_t)Gx * Gy));
    int64_t start, end;
    cell_range(keys, n, level, kx, ky, kz, start, end);
    if (start == end) return;
    const int64_t Rx = (int64_t)Gx * P, Ry = (int64_t)Gy * P;
    for (int e = threadIdx.x; e < P3; e += kBlock) {
        const int ax = e % P, ay = (e / P) % P, az = e / (P * P);
        sC[e] = C[(((int64_t)kz * P + az) * Ry + (int64_t)ky * P + ay) * Rx + (int64_t)kx * P + ax];
    }
    __syncthreads();
    const double cx = lox + (kx + 0.5) * cell, cy = loy + (ky + 0.5) * cell, cz = loz + (kz + 0.5) * cell;
    for (int64_t i0 = start + threadIdx.x; i0 < end; i0 += 2 * kBlock) {
        const int64_t i1 = i0 + kBlock;
        const bool has1 = i1 < end;
        const float4 q0 = ps[i0];
        const float4 q1 = has1 ? ps[i1] : q0;
        const float X0 = (float)(((double)q0.x - cx) * inv_sigma), X1 = (float)(((double)q1.x - cx) * inv_sigma);
        const float Y0 = (float)(((double)q0.y - cy) * inv_sigma), Y1 = (float)(((double)q1.y - cy) * inv_sigma);
        const float Z0 = (float)(((double)q0.z - cz) * inv_sigma), Z1 = (float)(((double)q1.z - cz) * inv_sigma);
        float uz0 = 0.f, uz1 = 0.f;
        for (int az = P - 1; az >= 0; --az) {
            float uy0 = 0.f, uy1 = 0.f;
#pragma unroll
            for (int ay = P - 1; ay >= 0; --ay) {
                const float *c = sC + (az * P + ay) * P;
                float ux0 = c[P - 1], ux1 = c[P - 1];
#pragma unroll
                for (int ax = P - 2; ax >= 0; --ax) {
                    const float cv = c[ax];
                    ux0 = fmaf(ux0, X0, cv);
                    ux1 = fmaf(ux1, X1, cv);
                }
                uy0 = fmaf(uy0, Y0, ux0);
                uy1 = fmaf(uy1, Y1, ux1);
            }
            uz0 = fmaf(uz0, Z0, uy0);
            uz1 = fmaf(uz1, Z1, uy1);
        }
        // back to input order; non-targets get 0
        const int32_t j0 = perm[i0];
        const bool t0 = !is_target || is_target[j0];
        u_out[j0] = t0 ? (subtract_self ? uz0 - w[j0] : uz0) : 0.f;
        if (has1) {
            const int32_t j1 = perm[i1];
            const bool t1 = !is_target || is_target[j1];
            u_out[j1] = t1 ? (subtract_self ? uz1 - w[j1] : uz1) : 0.f;
        }
    }
}

// Weights and target flags into key order (the w slot of the sorted positions).
__global__ void k_stage(const float *w, const uint8_t *is_target, const int32_t *perm, int64_t n,
                        float4 *ps, uint8_t *tflag) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t j = perm[i];
    ps[i].w = w[j];
    tflag[i] = is_target ? (is_target[j] != 0) : (uint8_t)1;
}

__global__ void k_scatter(const float *usort, const float4 *ps, const uint8_t *tflag,
                          const int32_t *perm, int64_t n, int subtract_self, float *u_out) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    float u = 0.f;
    if (tflag[i]) u = subtract_self ? usort[i] - ps[i].w : usort[i];
    u_out[perm[i]] = u;
}

struct GridArgs {
    const float *w;
    const uint8_t *is_target;
    int subtract_self;
    float *u_out;
};

template <int P>
int launch_p2m_l2p(msp_tree *t, const FgtPlan &pl, double inv_sigma, bool l2p, const float *C,
                   float *A, const GridArgs &ga, hipStream_t s) {
    const int64_t ncell = (int64_t)pl.G[0] * pl.G[1] * pl.G[2];
    if (!l2p) {
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_p2m<P>), dim3((unsigned)ncell), dim3(kBlock), 0, s,
                           t->keys.as<uint64_t>(), t->n, t->ps.as<float4>(), t->perm.as<int32_t>(),
                           ga.w, pl.level, pl.G[0], pl.G[1], pl.G[2], t->geo.lo[0], t->geo.lo[1],
                           t->geo.lo[2], pl.cell, inv_sigma, A);
    } else {
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_l2p<P>), dim3((unsigned)ncell), dim3(kBlock), 0, s,
                           t->keys.as<uint64_t>(), t->n, t->ps.as<float4>(), t->perm.as<int32_t>(),
                           ga.is_target, ga.w, ga.subtract_self, pl.level, pl.G[0], pl.G[1], pl.G[2],
                           t->geo.lo[0], t->geo.lo[1], t->geo.lo[2], pl.cell, inv_sigma, C, ga.u_out);
    }
    MSP_CHECK_LAUNCH();
    return MSP_OK;
}

int dispatch_p2m_l2p(msp_tree *t, const FgtPlan &pl, double inv_sigma, bool l2p, const float *C,
                     float *A, const GridArgs &ga, hipStream_t s) {
    switch (pl.p) {
#define CASE(P) case P: return launch_p2m_l2p<P>(t, pl, inv_sigma, l2p, C, A, ga, s);
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
        CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16)
#undef CASE
    }
    return fail(MSP_EINVAL, "p out of range");
}

}  // namespace

constexpr double kMaxGridBytes = 48.0e9;   // per expansion grid

int plan_fgt(const msp_tree *t, const msp_fgt_params *prm, FgtPlan *pl) {
    const int p = prm->p;
    const double sigma = prm->sigma;
    const double side = t->geo.side;
    int level = prm->level;
    if (level < 0) {
        const double rmax = rho_max_for_p(p);
        level = kDepth;
        for (int l = 0; l <= kDepth; ++l)
            if (side / std::ldexp(1.0, l + 1) / sigma <= rmax) { level = l; break; }
    }
    pl->p = p;
    pl->level = level;
    pl->cell = side / std::ldexp(1.0, level);
    pl->rho = 0.5 * pl->cell / sigma;
    double ncell = 1.0;
    for (int k = 0; k < 3; ++k) {
        pl->G[k] = (t->geo.qmax[k] >> (kDepth - level)) + 1;
        ncell *= pl->G[k];
    }
    const double p3 = (double)p * p * p;
    const double n = (double)t->n;
    // cost model in units of one float32 vector FMA
    const double gsum = (double)pl->G[0] + pl->G[1] + pl->G[2];
    pl->fgt_cost = 2.0 * p3 * n + (double)p * p3 * ncell * gsum + 2.0e5;
    double frac = 1.0;
    if (prm->cutoff_sigmas > 0.f) {
        const double R = prm->cutoff_sigmas * sigma;
        for (int k = 0; k < 3; ++k) {
            const double ext = side * (t->geo.qmax[k] + 1.0) / 2097152.0;
            frac *= ext > 2.0 * R ? 2.0 * R / ext : 1.0;
        }
    }
    pl->direct_cost = 8.0 * n * n * frac;
    const bool fits = ncell * p3 * 4.0 <= kMaxGridBytes;
    int route = prm->route;
    if (route == MSP_ROUTE_AUTO)
        route = (fits && pl->fgt_cost < pl->direct_cost) ? MSP_ROUTE_FGT : MSP_ROUTE_DIRECT;
    if (route == MSP_ROUTE_FGT && !fits)
        return fail(MSP_ENOSPC, "expansion grid %dx%dx%d at p=%d exceeds %.0f GB", pl->G[0], pl->G[1],
                    pl->G[2], p, kMaxGridBytes / 1e9);
    pl->route = route;
    return MSP_OK;
}

int stage_inputs(msp_tree *t, const float *w, const uint8_t *is_target, hipStream_t s) {
    const int64_t n = t->n, nb = n > 0 ? n : 1;
    MSP_TRY(t->tflag.ensure(nb));
    MSP_TRY(t->usort.ensure(nb * 4));
    if (n == 0) return MSP_OK;
    PhaseScope ps(&t->timing, PH_STAGE, s);
    hipLaunchKernelGGL(k_stage, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, w, is_target,
                       t->perm.as<int32_t>(), n, t->ps.as<float4>(), t->tflag.as<uint8_t>());
    MSP_CHECK_LAUNCH();
    return MSP_OK;
}

int fgt_forward_grid(msp_tree *t, const FgtPlan &pl, const msp_fgt_params *prm, const float *w,
                     const uint8_t *is_target, float *u_out, hipStream_t s) {
    const GridArgs ga{w, is_target, (prm->flags & MSP_EXCLUDE_SELF) ? 1 : 0, u_out};
    const int p = pl.p;
    const int64_t ncell = (int64_t)pl.G[0] * pl.G[1] * pl.G[2];
    const size_t gbytes = (size_t)ncell * p * p * p * 4;
    MSP_TRY(t->gridA.ensure(gbytes));
    MSP_TRY(t->gridB.ensure(gbytes));
    MSP_TRY(t->ops.ensure(gbytes + (size_t)(2 * (pl.G[0] + pl.G[1] + pl.G[2])) * p * p * 4));
    t->grid_bytes_valid = (int64_t)gbytes;
    if (t->n == 0) return MSP_OK;
    float *A = t->gridA.as<float>();
    float *B = t->gridB.as<float>();
    float *Tmp = t->ops.as<float>();                     // second intermediate grid
    float *opsx = Tmp + (size_t)ncell * p * p * p;
    float *opsy = opsx + (size_t)(2 * pl.G[0] - 1) * p * p;
    float *opsz = opsy + (size_t)(2 * pl.G[1] - 1) * p * p;
    const double step = pl.cell / prm->sigma;
    {
        PhaseScope ps(&t->timing, PH_OPS, s);
        const int nops = 2 * (pl.G[0] + pl.G[1] + pl.G[2]) - 3;
        hipLaunchKernelGGL(k_m2l_ops, dim3(grid_for(nops, 64)), dim3(64), 0, s, p, pl.G[0], pl.G[1],
                           pl.G[2], step, opsx, opsy, opsz);
        MSP_CHECK_LAUNCH();
    }
    const double inv_sigma = 1.0 / prm->sigma;
    {
        PhaseScope ps(&t->timing, PH_P2M, s);
        MSP_TRY(dispatch_p2m_l2p(t, pl, inv_sigma, false, nullptr, A, ga, s));
    }
    // three passes: contract x (In [Uz][Uy][Ux]), then y, then z
    const int64_t Ux = (int64_t)pl.G[0] * p, Uy = (int64_t)pl.G[1] * p, Uz = (int64_t)pl.G[2] * p;
    struct Pass { const float *in; float *out; int64_t R; int G; const float *T; int64_t U; };
    const Pass passes[3] = {{A, B, Uz * Uy, pl.G[0], opsx, Ux},
                            {B, Tmp, Ux * Uz, pl.G[1], opsy, Uy},
                            {Tmp, B, Uy * Ux, pl.G[2], opsz, Uz}};
    const bool valu = (prm->flags & MSP_M2L_VALU) != 0;
    for (int k = 0; k < 3; ++k) {
        const Pass &ps = passes[k];
        PhaseScope sc(&t->timing, PH_M2L_X + k, s);
        if (valu) {
            dim3 grid((unsigned)((ps.R + TR - 1) / TR), (unsigned)((ps.U + TV - 1) / TV));
            hipLaunchKernelGGL(k_m2l_pass, grid, dim3(kBlock), 0, s, ps.in, ps.out, ps.R, p, ps.G, ps.T);
        } else {
            dim3 grid((unsigned)((ps.R + MT - 1) / MT), (unsigned)((ps.U + MT - 1) / MT));
            hipLaunchKernelGGL(k_m2l_pass_mfma, grid, dim3(64), 0, s, ps.in, ps.out, ps.R, p, ps.G, ps.T);
        }
        MSP_CHECK_LAUNCH();
    }
    PhaseScope ps(&t->timing, PH_L2P, s);
    return dispatch_p2m_l2p(t, pl, inv_sigma, true, B, nullptr, ga, s);
}

int scatter_output(msp_tree *t, float *u_out, uint32_t flags, bool subtract_self, hipStream_t s) {
    (void)flags;
    if (t->n == 0) return MSP_OK;
    PhaseScope ps(&t->timing, PH_SCATTER, s);
    hipLaunchKernelGGL(k_scatter, dim3(grid_for(t->n, kBlock)), dim3(kBlock), 0, s,
                       t->usort.as<float>(), t->ps.as<float4>(), t->tflag.as<uint8_t>(),
                       t->perm.as<int32_t>(), t->n, subtract_self ? 1 : 0, u_out);
    MSP_CHECK_LAUNCH();
    return MSP_OK;
}

}  // namespace msp
