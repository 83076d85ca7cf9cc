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

#include <algorithm>
#include <cstring>

#include <cmath>

namespace msp {

// Cell half-side / sigma at which the transform of p terms per axis keeps the
// per-target relative error of the FP64 transform near 2e-5 on uniform test
// clouds (measured by brute force against the direct sum; the Cramer-type
// bound is far more pessimistic).  Index p - 1.
static const double kRhoMax[kMaxP] = {2e-5, 0.004, 0.025, 0.07, 0.16, 0.25, 0.34, 0.42,
                                      0.50, 0.60, 0.64, 0.68, 0.70, 0.70, 0.70, 0.70};

double rho_max_for_p(int p) { return kRhoMax[p - 1]; }

// Terms kept at the sub-cells two levels below the expansion level: the smallest
// pf whose per-axis tail sum_{b>=pf} (sqrt2 rho_f)^b / sqrt(b!) (the size of the
// dropped Taylor terms, by Cramer's inequality) is below 1e-5.
static int fine_terms(int p, double rho_f) {
    const double x = std::sqrt(2.0) * rho_f;
    for (int pf = 2; pf < p; ++pf) {
        double tail = 0.0;
        for (int b = pf; b < pf + 60; ++b) tail += std::exp(b * std::log(x) - 0.5 * std::lgamma(b + 1.0));
        if (tail <= 1e-5) return pf;
    }
    return p;
}

static size_t two_level_lds(int p, int pf) {
    const size_t a = 64 * pf * pf * pf + 16 * pf * pf * p + 4 * pf * p * p + 4 * pf * pf * pf;
    const size_t b = (size_t)p * p * p + 4 * pf * p * p + 16 * pf * pf * p + 64 * pf * pf * pf;
    return 4 * (a > b ? a : b);
}


namespace {

constexpr int kBlock = 256;
// batched expansion route: cells of at most this many points are processed eight
// to a wavefront (p <= 8)
constexpr int kSmallCell = 32;

// T_k[o][b][a] = (-1)^b / b! * h_{a+b}(o * step), o = -(G_k-1) .. G_k-1, for the three
// axes in one launch (thread -> axis, offset); computed in float64, stored as float32.
__device__ void m2l_ops_one(int p, int Gx, int Gy, int Gz, double step, float *ox, float *oy, float *oz, int t) {
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

__global__ void k_m2l_ops(int p, int Gx, int Gy, int Gz, double step, float *ox, float *oy, float *oz) {
    m2l_ops_one(p, Gx, Gy, Gz, step, ox, oy, oz, (int)(blockIdx.x * blockDim.x + threadIdx.x));
}

// Largest cell offset along an axis whose translation can matter: the entries
// (-1)^b/b! h_{a+b}(o step) of offset o, weighted by the largest moment and Taylor
// scales rho^a/a! and rho^b of a cell (rho = step/2, so that |A_a| <= W rho^a / a!),
// stay below 1e-9 of the zero-offset term for every larger offset.  The M2L
// contractions skip the blocks beyond it.
int m2l_band(int p, double step, int G) {
    const double rho = 0.5 * step;
    int band = 0;
    for (int o = 1; o < G; ++o) {
        const double x = o * step;
        double h[2 * kMaxP];
        h[0] = std::exp(-x * x);
        if (2 * p - 1 > 1) h[1] = 2.0 * x * h[0];
        for (int n = 1; n + 1 < 2 * p - 1; ++n) h[n + 1] = 2.0 * x * h[n] - 2.0 * n * h[n - 1];
        double worst = 0.0, fa = 1.0, ra = 1.0;
        for (int a = 0; a < p; ++a) {
            if (a > 0) {
                fa *= a;
                ra *= rho;
            }
            double fb = 1.0, rb = 1.0;
            for (int b = 0; b < p; ++b) {
                if (b > 0) {
                    fb *= b;
                    rb *= rho;
                }
                worst = std::fmax(worst, std::fabs(h[a + b]) * ra * rb / (fa * fb));
            }
        }
        if (worst >= 1e-9) band = o;
    }
    return band;
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
// Moments of the points [start, end) of cell (kx, ky, kz) (block-wide).
template <int P>
__device__ void p2m_cell(const float4 *ps, const int32_t *perm, const float *w, int Gx, int Gy,
                         double lox, double loy, double loz, double cell, double inv_sigma, float *A,
                         int kx, int ky, int kz, int64_t start, int64_t end, float4 *stage) {
    constexpr int P3 = P * P * P;
    constexpr int PL = 64 / P;            // point lanes per wave
    constexpr int NW = kBlock / 64;
    constexpr int NB = P <= 12 ? NW : 1;  // partial buffers (LDS budget for large P)
    __shared__ float red[NB][P3];
    const double cx = lox + (kx + 0.5) * cell, cy = loy + (ky + 0.5) * cell, cz = loz + (kz + 0.5) * cell;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int az = lane % P, pl = lane / P;
    const bool active = pl < PL;
    float acc[P][P];
#pragma unroll
    for (int a = 0; a < P; ++a)
#pragma unroll
        for (int b = 0; b < P; ++b) acc[a][b] = 0.f;
    // the cell's points pass through LDS in chunks of kBlock, one point per thread:
    // while a chunk is being accumulated, the threads already hold the next one
    // (position and the weight gathered through the permutation) in registers
    __shared__ float4 chunk[kBlock];
    float4 nxt = make_float4(0.f, 0.f, 0.f, 0.f);
    auto fetch = [&](int64_t c0) {
        const int64_t j = c0 + tid;
        if (j < end) {
            const float4 q = ps[j];
            const float wv = w ? w[perm[j]] : q.w;   // NULL: the weights are staged in the records
            // the weight in key order, for later calls (whole records: full-line writes)
            if (stage) stage[j] = make_float4(q.x, q.y, q.z, wv);
            nxt = make_float4(((q.x - (float)cx) * (float)inv_sigma), ((q.y - (float)cy) * (float)inv_sigma),
                              ((q.z - (float)cz) * (float)inv_sigma), wv);
        }
    };
    fetch(start);
    for (int64_t c0 = start; c0 < end; c0 += kBlock) {
        __syncthreads();
        chunk[tid] = nxt;
        __syncthreads();
        if (c0 + kBlock < end) fetch(c0 + kBlock);
        const int m = end - c0 < kBlock ? (int)(end - c0) : kBlock;
        if (active)
            for (int jj = wid * PL + pl; jj < m; jj += NW * PL) {
                const float4 q = chunk[jj];
                float zw = q.w;
#pragma unroll
                for (int k = 1; k < P; ++k) zw = k <= az ? zw * q.z : zw;
                float px[P], yz[P];
                px[0] = 1.f;
                yz[0] = zw;
#pragma unroll
                for (int k = 1; k < P; ++k) {
                    px[k] = px[k - 1] * q.x;
                    yz[k] = yz[k - 1] * q.y;
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

// One block per cell of the grid; moments written in the grid layout
// [kz][az][ky][ay][kx][ax] (empty cells get zeros).
template <int P>
__global__ void __launch_bounds__(kBlock) k_p2m(const uint64_t *keys, int64_t n, const float4 *ps,
                                                const int32_t *perm, const float *w,
                                                int level, int Gx, int Gy, int Gz, double lox,
                                                double loy, double loz, double cell,
                                                double inv_sigma, float *A, float4 *stage) {
    const int64_t g = blockIdx.x;
    const int kx = (int)(g % Gx), ky = (int)((g / Gx) % Gy), kz = (int)(g / ((int64_t)Gx * Gy));
    int64_t start, end;
    cell_range(keys, n, level, kx, ky, kz, start, end);
    p2m_cell<P>(ps, perm, w, Gx, Gy, lox, loy, loz, cell, inv_sigma, A, kx, ky, kz, start, end, stage);
}

// P2M of one grid cell for p = 8 on the matrix cores.  With ay = 2 ay_hi + ay_lo the
// moments form a 16 x 32 matrix product over the cell's points,
//   M[(ax, ay_lo)][(ay_hi, az)] = sum_j X_j^ax Y_j^ay_lo * w_j Y_j^(2 ay_hi) Z_j^az,
// taken four points at a time by v_mfma_f32_16x16x4f32 (two 16-column tiles).  The
// cell's points pass through LDS 256 at a time with their powers (X^k, Y^k and
// w Z^k, k < 8), one point per thread, the next chunk held in registers; each wave
// takes 64 of them, and the four waves' products are added in wave order at the end.
// One block per cell; output in the grid layout [kz][az][ky][ay][kx][ax].
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kPowStr = 25;   // floats per staged point (24 powers, padded)
__global__ void __launch_bounds__(kBlock) k_p2m_mfma8(const uint64_t *keys, int64_t n, const float4 *ps,
                                                      const int32_t *perm, const float *w, int level, int Gx,
                                                      int Gy, int Gz, double lox, double loy, double loz,
                                                      double cell, double inv_sigma, float *A, float4 *stage) {
    __shared__ float pw[kBlock * kPowStr];
    __shared__ float red[kBlock / 64][512];
    const int64_t g = blockIdx.x;
    const int kx = (int)(g % Gx), ky = (int)((g / Gx) % Gy), kz = (int)(g / ((int64_t)Gx * Gy));
    int64_t start, end;
    cell_range(keys, n, level, kx, ky, kz, start, end);
    const double cx = lox + (kx + 0.5) * cell, cy = loy + (ky + 0.5) * cell, cz = loz + (kz + 0.5) * cell;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    float4 nxt = make_float4(0.f, 0.f, 0.f, 0.f);
    auto fetch = [&](int64_t c0) {
        const int64_t j = c0 + tid;
        nxt = make_float4(0.f, 0.f, 0.f, 0.f);   // past the cell: zero weight
        if (j < end) {
            const float4 q = ps[j];
            const float wv = w ? w[perm[j]] : q.w;   // NULL: the weights are staged in the records
            // the weight in key order, for later calls (whole records: full-line writes)
            if (stage) stage[j] = make_float4(q.x, q.y, q.z, wv);
            nxt = make_float4(((q.x - (float)cx) * (float)inv_sigma), ((q.y - (float)cy) * (float)inv_sigma),
                              ((q.z - (float)cz) * (float)inv_sigma), wv);
        }
    };
    // this lane's operand slots: row m = (ax, ay_lo), column n = (ay_hi within the tile, az)
    const int m = lane & 15, kq = lane >> 4;
    const int ax = m >> 1, aylo = m & 1;
    const int n16 = lane & 15, azc = n16 & 7, ayh0 = n16 >> 3;
    f32x4 acc0 = f32x4{0.f, 0.f, 0.f, 0.f}, acc1 = f32x4{0.f, 0.f, 0.f, 0.f};
    fetch(start);
    // each wavefront stages and reads only its own 64 rows (thread tid writes row
    // tid, wavefront w reads rows 64 w .. 64 w + 63), so the waves synchronise
    // only with themselves
    for (int64_t c0 = start; c0 < end; c0 += kBlock) {
        wave_sync();
        {
            float *r = pw + tid * kPowStr;
            float xp = 1.f, yp = 1.f, wz = nxt.w;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                r[k] = xp;
                r[8 + k] = yp;
                r[16 + k] = wz;
                xp *= nxt.x;
                yp *= nxt.y;
                wz *= nxt.z;
            }
        }
        wave_sync();
        if (c0 + kBlock < end) fetch(c0 + kBlock);
        const int cnt = end - c0 < kBlock ? (int)(end - c0) : kBlock;
        const int w0 = __builtin_amdgcn_readfirstlane(wid) * 64;
        if (w0 < cnt) {
            // rows past the cell weigh 0, so the steps go in groups of eight (a
            // wave-uniform count): all operands of a group are read from LDS
            // before its products
            const int steps = ((cnt - w0 < 64 ? cnt - w0 : 64) + 3) / 4;
            for (int s0 = 0; s0 < steps; s0 += 8) {
                float av[8], b0v[8], b1v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const float *r = pw + (w0 + 4 * (s0 + u) + kq) * kPowStr;
                    av[u] = r[ax] * r[8 + aylo];
                    b0v[u] = r[8 + 2 * ayh0] * r[16 + azc];
                    b1v[u] = r[8 + 2 * (ayh0 + 2)] * r[16 + azc];
                }
                __builtin_amdgcn_sched_barrier(0);   // keep the reads ahead of the products
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u], b0v[u], acc0, 0, 0, 0);
                    acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u], b1v[u], acc1, 0, 0, 0);
                }
            }
        }
    }
    // D[4 kq + i][n16] of both tiles -> red[wave][(az * 8 + ay) * 8 + ax]
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int mm = 4 * kq + i, axo = mm >> 1, aylo_o = mm & 1;
        red[wid][(azc * 8 + 2 * ayh0 + aylo_o) * 8 + axo] = acc0[i];
        red[wid][(azc * 8 + 2 * (ayh0 + 2) + aylo_o) * 8 + axo] = acc1[i];
    }
    __syncthreads();
    const int64_t Rx = (int64_t)Gx * 8, Ry = (int64_t)Gy * 8;
    for (int e = tid; e < 512; e += kBlock) {
        float sum = 0.f;
#pragma unroll
        for (int q = 0; q < kBlock / 64; ++q) sum += red[q][e];
        const int ex = e & 7, ey = (e >> 3) & 7, ez = e >> 6;
        float f = 1.f;
        for (int k = 2; k <= ex; ++k) f *= (float)k;
        for (int k = 2; k <= ey; ++k) f *= (float)k;
        for (int k = 2; k <= ez; ++k) f *= (float)k;
        A[(((int64_t)kz * 8 + ez) * Ry + (int64_t)ky * 8 + ey) * Rx + (int64_t)kx * 8 + ex] = sum / f;
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
constexpr int MT = 32, MK = 16;
__device__ void m2l_tile_mfma(const float *In, float *Out, int64_t R, int p, int G, const float *T, int64_t r0,
                              int v0) {
    __shared__ float sA[MT][MK + 1];   // operator rows v, columns u
    __shared__ float sB[MT][MK + 1];   // input rows r, columns u
    const int U = G * p;
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

__global__ void __launch_bounds__(64) k_m2l_pass_mfma(const float *In, float *Out, int64_t R, int p,
                                                      int G, const float *T) {
    m2l_tile_mfma(In, Out, R, p, G, T, (int64_t)blockIdx.x * MT, (int)blockIdx.y * MT);
}

// Split bfloat16 products (v_mfma_f32_16x16x32_bf16): each FP32 operand x is
// split into hi = bf16(x) and lo = bf16(x - hi), and hi*hi + hi*lo + lo*hi is
// accumulated in FP32.  The dropped lo*lo term and the rounding of lo leave about
// 2^-16 of each product.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
constexpr int MK2 = 32;

__device__ inline unsigned short bf16_bits(float f) {   // round to nearest even
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__device__ inline void split_bf16(const float *src, int stride, bf16x8 &hi, bf16x8 &lo) {
    u16x8 h, l;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const float x = src[j * stride];
        const unsigned short hb = bf16_bits(x);
        h[j] = hb;
        l[j] = bf16_bits(x - __uint_as_float((uint32_t)hb << 16));
    }
    hi = __builtin_bit_cast(bf16x8, h);
    lo = __builtin_bit_cast(bf16x8, l);
}

// The same pass with the whole contraction in LDS: a block of four waves takes RT
// rows r of In (all U columns, staged once) and the operator table T of the axis,
// and produces Out[v][r] for every v.  Each wave owns 16-row slices of v: it keeps
// its slice's operator entries for all K steps in registers (generated from T by
// offset, row and column) and sweeps the r columns in 16-wide MFMA tiles
// (v_mfma_f32_16x16x4f32, same lane layout as above).  LDS: RT x (U + 1) floats of
// In and (2G - 1) p^2 floats of T (dynamic).
__host__ __device__ inline size_t m2l_gemm_lds(int U, int G, int p, int RT) {
    // input rows, operator table, and (cell-major modes) row bases and column offsets
    const size_t nT = (size_t)(2 * G - 1) * p * p;
    return ((size_t)RT * (U + 1) + nT + (nT & 1)) * 4 + (size_t)RT * 8 + (size_t)U * 4;
}

// The split bfloat16 form of the tile (p = 8): the RT input rows and the operator
// table as hi and lo bfloat16 planes, rows padded to whole 32-term K steps plus 8.
__host__ __device__ inline int m2l_split_row(int U) { return ((U + 31) / 32) * 32 + 8; }
__host__ __device__ inline size_t m2l_gemm_lds_split(int U, int G, int RT) {
    const size_t nT = (size_t)(2 * G - 1) * 64;
    size_t b = (size_t)RT * m2l_split_row(U) * 4 + nT * 4;   // two 2-byte planes each
    b = (b + 15) & ~(size_t)15;
    return b + (size_t)RT * 8;
}

// Grid layouts.  The M2L passes read rows along one axis of the interleaved layout
// [kz p + az][ky p + ay][kx p + ax].  The batched route keeps the moment and Taylor
// grids cell-major instead, [kz][ky][kx][az][ay][ax], so that one cell's p^3
// coefficients are one contiguous run for P2M and L2P; its x pass (MODE 1) reads the
// cell-major moments, and its z pass (MODE 2) takes its rows in cell-column order
// (ky, kx, ay, ax) and writes the cell-major Taylor grid.  Ga: the grid's cells along
// y (MODE 1) or x (MODE 2).
// m2l_gemm_tile with split bfloat16 products (p = 8): every staged input and
// operator entry x is split once into hi = bf16(x) and lo = bf16(x - hi), and each
// 16 x 16 output tile accumulates hi*hi + hi*lo + lo*hi over 32-term K steps with
// v_mfma_f32_16x16x32_bf16 (four cells of eight terms per step).  Lane l supplies
// A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16], j < 8, and receives
// D[4 (l / 16) + i][l % 16]: one operator row of one cell and eight consecutive
// terms of one input row, each one 16-byte read from LDS.
template <int RT, int MODE>
__device__ void m2l_gemm_tile_split(const float *In, float *Out, int64_t R, int G, const float *T, int64_t r0,
                                    float *sm, int Ga, int band) {
    constexpr int NR = RT / 16;
    constexpr int p = 8, pp = 64, p3 = 512;
    const int U = G * p;
    const int UH = m2l_split_row(U);
    const int nT = (2 * G - 1) * pp;
    unsigned short *sInH = reinterpret_cast<unsigned short *>(sm);
    unsigned short *sInL = sInH + (size_t)RT * UH;
    unsigned short *sTH = sInL + (size_t)RT * UH;
    unsigned short *sTL = sTH + nT;
    int64_t *rowbase = reinterpret_cast<int64_t *>(
        reinterpret_cast<char *>(sm) + ((((size_t)RT * UH * 4 + (size_t)nT * 4) + 15) & ~(size_t)15));
    auto put = [](unsigned short *h, unsigned short *l, float x) {
        const unsigned short hb = bf16_bits(x);
        *h = hb;
        *l = bf16_bits(x - __uint_as_float((uint32_t)hb << 16));
    };
    for (int e = threadIdx.x; e < nT; e += 256) put(sTH + e, sTL + e, T[e]);
    if constexpr (MODE != 0) {
        for (int rr = threadIdx.x; rr < RT; rr += 256) {
            const int64_t r = r0 + rr;
            int64_t b = -1;
            if (r < R) {
                if constexpr (MODE == 1) {
                    const int Uy = Ga * 8;
                    const int zq = (int)(r / Uy), yq = (int)(r % Uy);
                    b = ((int64_t)(zq >> 3) * Ga + (yq >> 3)) * G * 512 + ((zq & 7) * 8 + (yq & 7)) * 8;
                } else {
                    const int c = (int)(r >> 6), rem = (int)(r & 63);
                    b = ((int64_t)((c / Ga) * 8 + (rem >> 3)) * Ga * 8 + (c % Ga) * 8 + (rem & 7)) * U;
                }
            }
            rowbase[rr] = b;
        }
        __syncthreads();
    }
    // input rows in 16-byte chunks (a chunk never straddles a cell), zeros past U
    const int U4 = UH / 4;
    for (int e = threadIdx.x; e < RT * U4; e += 256) {
        const int rr = e / U4, c4 = e - rr * U4;
        const int64_t r = r0 + rr;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (4 * c4 < U) {
            if constexpr (MODE == 0) {
                if (r < R) v = *reinterpret_cast<const float4 *>(In + r * U + 4 * c4);
            } else {
                const int64_t b = rowbase[rr];
                const int64_t col = MODE == 1 ? (int64_t)(c4 >> 1) * 512 + (c4 & 1) * 4 : 4 * c4;
                if (b >= 0) v = *reinterpret_cast<const float4 *>(In + b + col);
            }
        }
        unsigned short *dh = sInH + (size_t)rr * UH + 4 * c4, *dl = sInL + (size_t)rr * UH + 4 * c4;
        put(dh, dl, v.x);
        put(dh + 1, dl + 1, v.y);
        put(dh + 2, dl + 2, v.z);
        put(dh + 3, dl + 3, v.w);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nk = (U + 31) / 32;   // 32-term K steps
    const int nv = (U + 15) / 16;
    const bf16x8 zero8 = __builtin_bit_cast(bf16x8, u16x8{0, 0, 0, 0, 0, 0, 0, 0});
    for (int vc = wave; vc < nv; vc += 4) {
        const int v = vc * 16 + (lane & 15);
        const int tv = v / p, b = v % p;
        f32x4 acc[NR];
#pragma unroll
        for (int j = 0; j < NR; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
        int kb = 0, ke = nk;
        if (band < G - 1) {
            const int vlast = vc * 16 + 15 < U ? vc * 16 + 15 : U - 1;
            const int c_lo = (vc * 16) / p - band, c_hi = vlast / p + band;
            kb = (c_lo > 0 ? c_lo : 0) / 4;
            const int c_end = c_hi + 1 < G ? c_hi + 1 : G;
            ke = (c_end + 3) / 4 < nk ? (c_end + 3) / 4 : nk;
        }
        for (int ks = kb; ks < ke; ++ks) {
            const int sc = 4 * ks + (lane >> 4);   // the cell of this lane's eight terms
            bf16x8 ah = zero8, al = zero8;
            if (v < U && sc < G) {
                const int row = ((tv - sc + G - 1) * p + b) * p;
                ah = *reinterpret_cast<const bf16x8 *>(sTH + row);
                al = *reinterpret_cast<const bf16x8 *>(sTL + row);
            }
#pragma unroll
            for (int j = 0; j < NR; ++j) {
                const size_t o = (size_t)(16 * j + (lane & 15)) * UH + 32 * ks + 8 * (lane >> 4);
                const bf16x8 bh = *reinterpret_cast<const bf16x8 *>(sInH + o);
                const bf16x8 bl = *reinterpret_cast<const bf16x8 *>(sInL + o);
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[j], 0, 0, 0);
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[j], 0, 0, 0);
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[j], 0, 0, 0);
            }
        }
#pragma unroll
        for (int j = 0; j < NR; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int vo = vc * 16 + 4 * (lane >> 4) + i;
                const int64_t r = r0 + 16 * j + (lane & 15);
                if (vo < U && r < R) {
                    if constexpr (MODE == 2) {
                        const int q = (int)r;
                        Out[(int64_t)(vo / p) * R * p + (vo % p) * pp + (int64_t)(q / pp) * p3 + q % pp] = acc[j][i];
                    } else {
                        Out[(int64_t)vo * R + r] = acc[j][i];
                    }
                }
            }
    }
}

template <int RT, int MODE = 0, int PT = 0, bool SPLIT = false>
__device__ void m2l_gemm_tile(const float *In, float *Out, int64_t R, int p_rt, int G, const float *T, int64_t r0,
                              float *sm, int Ga = 0, int band = 1 << 30) {
    if constexpr (SPLIT) {
        static_assert(PT == 8, "the split bfloat16 tile is built for p = 8");
        m2l_gemm_tile_split<RT, MODE>(In, Out, R, G, T, r0, sm, Ga, band);
        return;
    }
    // PT = 8: the term count is a compile-time 8, so the tile's index arithmetic
    // folds into constants and rows are read 16 bytes at a time; PT = 0: any p
    constexpr int NR = RT / 16;   // 16-wide column tiles per block
    constexpr int KC = 8;         // K steps (of 4) per operator chunk in registers
    const int p = PT ? PT : p_rt;
    const int U = G * p;
    const int UP = U + 1;
    float *sIn = sm;
    float *sT = sm + (size_t)RT * UP;
    const int nT = (2 * G - 1) * p * p;
    for (int e = threadIdx.x; e < nT; e += 256) sT[e] = T[e];
    const int pp = p * p;
    const int p3 = pp * p;
    if constexpr (PT == 8) {
        // U = 8 G: rows in 16-byte chunks, which never straddle a cell
        const int U4 = U / 4;
        if constexpr (MODE == 0) {
            for (int e = threadIdx.x; e < RT * U4; e += 256) {
                const int rr = e / U4, c4 = e - rr * U4;
                const int64_t r = r0 + rr;
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (r < R) v = *reinterpret_cast<const float4 *>(In + r * U + 4 * c4);
                float *d = sIn + rr * UP + 4 * c4;
                d[0] = v.x;
                d[1] = v.y;
                d[2] = v.z;
                d[3] = v.w;
            }
        } else {
            int64_t *rowbase = reinterpret_cast<int64_t *>(sT + nT + (nT & 1));
            for (int rr = threadIdx.x; rr < RT; rr += 256) {
                const int64_t r = r0 + rr;
                int64_t b = -1;
                if (r < R) {
                    if constexpr (MODE == 1) {
                        const int Uy = Ga * 8;
                        const int zq = (int)(r / Uy), yq = (int)(r % Uy);
                        b = ((int64_t)(zq >> 3) * Ga + (yq >> 3)) * G * 512 + ((zq & 7) * 8 + (yq & 7)) * 8;
                    } else {
                        const int c = (int)(r >> 6), rem = (int)(r & 63);
                        b = ((int64_t)((c / Ga) * 8 + (rem >> 3)) * Ga * 8 + (c % Ga) * 8 + (rem & 7)) * U;
                    }
                }
                rowbase[rr] = b;
            }
            __syncthreads();
            for (int e = threadIdx.x; e < RT * U4; e += 256) {
                const int rr = e / U4, c4 = e - rr * U4;
                const int64_t b = rowbase[rr];
                // MODE 1: column u = 4 c4 is (cell u / 8, term u % 8), 512 floats per cell
                const int64_t col = MODE == 1 ? (int64_t)(c4 >> 1) * 512 + (c4 & 1) * 4 : 4 * c4;
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (b >= 0) v = *reinterpret_cast<const float4 *>(In + b + col);
                float *d = sIn + rr * UP + 4 * c4;
                d[0] = v.x;
                d[1] = v.y;
                d[2] = v.z;
                d[3] = v.w;
            }
        }
    } else if constexpr (MODE == 0) {
        for (int e = threadIdx.x; e < RT * U; e += 256) {
            const int rr = e / U, u = e % U;
            const int64_t r = r0 + rr;
            sIn[rr * UP + u] = r < R ? In[r * U + u] : 0.f;
        }
    } else {
        // element (rr, u) of the tile sits at rowbase[rr] + colofs[u]
        int64_t *rowbase = reinterpret_cast<int64_t *>(sT + nT + (nT & 1));
        int *colofs = reinterpret_cast<int *>(rowbase + RT);
        for (int rr = threadIdx.x; rr < RT; rr += 256) {
            const int64_t r = r0 + rr;
            int64_t b = -1;
            if (r < R) {
                if constexpr (MODE == 1) {   // row r = (z', y') of the cell-major moments
                    const int Uy = Ga * p;
                    const int zq = (int)(r / Uy), yq = (int)(r % Uy);
                    b = ((int64_t)(zq / p) * Ga + yq / p) * G * (int64_t)p3 + ((zq % p) * p + yq % p) * p;
                } else {                     // row q = (ky, kx, ay, ax) in cell-column order
                    const int c = (int)(r / pp), rem = (int)(r % pp);
                    b = ((int64_t)((c / Ga) * p + rem / p) * Ga * p + (c % Ga) * p + rem % p) * U;
                }
            }
            rowbase[rr] = b;
        }
        for (int u = threadIdx.x; u < U; u += 256) colofs[u] = MODE == 1 ? (u / p) * p3 + u % p : u;
        __syncthreads();
        for (int e = threadIdx.x; e < RT * U; e += 256) {
            const int rr = e / U, u = e % U;
            const int64_t b = rowbase[rr];
            sIn[rr * UP + u] = b >= 0 ? In[b + colofs[u]] : 0.f;
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nk = (U + 3) / 4;
    const int nv = (U + 15) / 16;
    // the grid's y index picks a group of four 16-wide column blocks (one group
    // when the grid is one-dimensional)
    for (int vc = wave + 4 * (int)blockIdx.y; vc < nv; vc += 4 * (int)gridDim.y) {
        const int v = vc * 16 + (lane & 15);
        const int tv = v / p, b = v % p;
        f32x4 acc[NR];
#pragma unroll
        for (int j = 0; j < NR; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
        // K steps [kb, ke) that meet an operator block within `band` cells of this
        // column block's cells (the blocks beyond it are negligible and skipped)
        int kb = 0, ke = nk;
        if (band < G - 1) {
            const int vlast = vc * 16 + 15 < U ? vc * 16 + 15 : U - 1;
            const int c_lo = (vc * 16) / p - band, c_hi = vlast / p + band;
            kb = (c_lo > 0 ? c_lo : 0) * p / 4;
            const int u_end = (c_hi + 1 < G ? c_hi + 1 : G) * p;
            ke = (u_end + 3) / 4 < nk ? (u_end + 3) / 4 : nk;
        }
        const int u0 = 4 * kb + (lane >> 4);
        int s = u0 / p, ai = u0 % p;   // column u = 4 k + lane / 16 as (cell, term)
        // p = 8: entry of step k at base8 - 64 (k / 2) + 4 (k % 2)
        const int base8 = ((tv + G - 1) * 8 + b) * 8 + (lane >> 4);
        for (int k0 = kb; k0 < ke; k0 += KC) {
            // this lane's operator entries M[v][u] for KC steps
            float a[KC];
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                if constexpr (PT == 8) {
                    const int kk = k0 + k;
                    a[k] = (v < U && kk < ke) ? sT[base8 - 64 * (kk >> 1) + 4 * (kk & 1)] : 0.f;
                } else {
                    const int u = 4 * (k0 + k) + (lane >> 4);
                    a[k] = (v < U && u < U && k0 + k < ke) ? sT[((tv - s + G - 1) * p + b) * p + ai] : 0.f;
                    ai += 4;
                    while (ai >= p) {
                        ai -= p;
                        ++s;
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < NR; ++j) {
                const float *bcol = sIn + (16 * j + (lane & 15)) * UP + (lane >> 4);
#pragma unroll
                for (int k = 0; k < KC; ++k) {
                    float bv;
                    if constexpr (PT == 8) {
                        bv = k0 + k < ke ? bcol[4 * (k0 + k)] : 0.f;
                    } else {
                        const int u = 4 * (k0 + k) + (lane >> 4);
                        bv = (u < U && k0 + k < ke) ? bcol[4 * (k0 + k)] : 0.f;
                    }
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[k], bv, acc[j], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < NR; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int vo = vc * 16 + 4 * (lane >> 4) + i;
                const int64_t r = r0 + 16 * j + (lane & 15);
                if (vo < U && r < R) {
                    if constexpr (MODE == 2) {   // vo = z' = (kz, az); r = q in cell-column order
                        const int q = (int)r;
                        Out[(int64_t)(vo / p) * R * p + (vo % p) * pp + (int64_t)(q / pp) * p3 + q % pp] = acc[j][i];
                    } else {
                        Out[(int64_t)vo * R + r] = acc[j][i];
                    }
                }
            }
    }
}

template <int RT>
__global__ void __launch_bounds__(256) k_m2l_gemm(const float *In, float *Out, int64_t R, int p, int G,
                                                  const float *T, int band) {
    extern __shared__ float sm[];
    if (p == 8) m2l_gemm_tile<RT, 0, 8>(In, Out, R, p, G, T, (int64_t)blockIdx.x * RT, sm, 0, band);
    else m2l_gemm_tile<RT>(In, Out, R, p, G, T, (int64_t)blockIdx.x * RT, sm, 0, band);
}

// The whole-K tile with split bfloat16 products (p = 8).
template <int RT>
__global__ void __launch_bounds__(256) k_m2l_gemm_bf16x3(const float *In, float *Out, int64_t R, int G,
                                                         const float *T, int band) {
    extern __shared__ float sm[];
    m2l_gemm_tile<RT, 0, 8, true>(In, Out, R, 8, G, T, (int64_t)blockIdx.x * RT, sm, 0, band);
}

// The split bfloat16 pass for any p, 32 x 32 output tiles: each K step builds the
// operator tile from T and splits both operands in registers; a lane supplies
// eight consecutive k of its row of A and of its column of B (the same k for
// both).  Used where the whole-K tile does not apply (p != 8, or too little LDS).
__global__ void __launch_bounds__(64) k_m2l_pass_bf16x3(const float *In, float *Out, int64_t R, int p,
                                                        int G, const float *T) {
    __shared__ float sA[MT][MK2 + 1];   // operator rows v, columns u
    __shared__ float sB[MT][MK2 + 1];   // input rows r, columns u
    const int U = G * p;
    const int64_t r0 = (int64_t)blockIdx.x * MT;
    const int v0 = blockIdx.y * MT;
    const int lane = threadIdx.x;
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int u0 = 0; u0 < U; u0 += MK2) {
#pragma unroll
        for (int e = lane; e < MT * MK2; e += 64) {
            const int row = e / MK2, kk = e % MK2;
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
        const int k8 = 8 * (lane >> 4), rr = lane & 15;
        bf16x8 a0h, a0l, a1h, a1l, b0h, b0l, b1h, b1l;
        split_bf16(&sA[rr][k8], 1, a0h, a0l);
        split_bf16(&sA[16 + rr][k8], 1, a1h, a1l);
        split_bf16(&sB[rr][k8], 1, b0h, b0l);
        split_bf16(&sB[16 + rr][k8], 1, b1h, b1l);
#define MSP_BF16X3(ACC, AH, AL, BH, BL)                                              \
    ACC = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AL, BH, ACC, 0, 0, 0);             \
    ACC = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AH, BL, ACC, 0, 0, 0);             \
    ACC = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AH, BH, ACC, 0, 0, 0);
        MSP_BF16X3(acc[0][0], a0h, a0l, b0h, b0l)
        MSP_BF16X3(acc[0][1], a0h, a0l, b1h, b1l)
        MSP_BF16X3(acc[1][0], a1h, a1l, b0h, b0l)
        MSP_BF16X3(acc[1][1], a1h, a1l, b1h, b1l)
#undef MSP_BF16X3
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
// Taylor series of cell (kx, ky, kz) at its points [start, end) (block-wide).
// TGT: target flags given; SUB: the self term w_j is subtracted (both fixed per
// launch, so the gathers through the permutation issue without branches)
template <int P, bool TGT, bool SUB>
__device__ void l2p_cell_impl(const float4 *ps, const int32_t *perm, const uint8_t *is_target,
                              const float *w, int Gx, int Gy, double lox, double loy, double loz,
                              double cell, double inv_sigma, const float *C, float *u_out, int kx,
                              int ky, int kz, int64_t start, int64_t end) {
    constexpr int P3 = P * P * P;
    __shared__ float sC[P3];
    const int64_t Rx = (int64_t)Gx * P, Ry = (int64_t)Gy * P;
    for (int e = threadIdx.x; e < P3; e += kBlock) {
        const int ax = e % P, ay = (e / P) % P, az = e / (P * P);
        sC[e] = C[(((int64_t)kz * P + az) * Ry + (int64_t)ky * P + ay) * Rx + (int64_t)kx * P + ax];
    }
    __syncthreads();
    const double cx = lox + (kx + 0.5) * cell, cy = loy + (ky + 0.5) * cell, cz = loz + (kz + 0.5) * cell;
    // four points per thread and pass, so that every coefficient read from LDS serves
    // four Horner chains (with fewer, the LDS reads bound the loop)
    constexpr int NPT = 4;
    for (int64_t i0 = start + threadIdx.x; i0 < end; i0 += NPT * kBlock) {
        float X[NPT], Y[NPT], Z[NPT], ws[NPT];
        int32_t jo[NPT];
        bool has[NPT], tg[NPT];
#pragma unroll
        for (int u = 0; u < NPT; ++u) {
            const int64_t i = i0 + (int64_t)u * kBlock;
            has[u] = i < end;
            const float4 q = ps[has[u] ? i : i0];
            X[u] = (q.x - (float)cx) * (float)inv_sigma;
            Y[u] = (q.y - (float)cy) * (float)inv_sigma;
            Z[u] = (q.z - (float)cz) * (float)inv_sigma;
            jo[u] = perm[has[u] ? i : i0];
        }
        // the scattered reads of the output step are issued before the evaluation
#pragma unroll
        for (int u = 0; u < NPT; ++u) {
            tg[u] = TGT ? is_target[jo[u]] != 0 : true;
            ws[u] = SUB ? w[jo[u]] : 0.f;
        }
        float uz[NPT];
#pragma unroll
        for (int u = 0; u < NPT; ++u) uz[u] = 0.f;
        for (int az = P - 1; az >= 0; --az) {
            float uy[NPT];
#pragma unroll
            for (int u = 0; u < NPT; ++u) uy[u] = 0.f;
#pragma unroll
            for (int ay = P - 1; ay >= 0; --ay) {
                const float *c = sC + (az * P + ay) * P;
                float ux[NPT];
#pragma unroll
                for (int u = 0; u < NPT; ++u) ux[u] = c[P - 1];
#pragma unroll
                for (int ax = P - 2; ax >= 0; --ax) {
                    const float cv = c[ax];
#pragma unroll
                    for (int u = 0; u < NPT; ++u) ux[u] = fmaf(ux[u], X[u], cv);
                }
#pragma unroll
                for (int u = 0; u < NPT; ++u) uy[u] = fmaf(uy[u], Y[u], ux[u]);
            }
#pragma unroll
            for (int u = 0; u < NPT; ++u) uz[u] = fmaf(uz[u], Z[u], uy[u]);
        }
        // back to input order; non-targets get 0
#pragma unroll
        for (int u = 0; u < NPT; ++u)
            if (has[u]) u_out[jo[u]] = tg[u] ? uz[u] - ws[u] : 0.f;
    }
}

template <int P>
__device__ void l2p_cell(const float4 *ps, const int32_t *perm, const uint8_t *is_target, const float *w,
                         int subtract_self, int Gx, int Gy, double lox, double loy, double loz,
                         double cell, double inv_sigma, const float *C, float *u_out, int kx, int ky,
                         int kz, int64_t start, int64_t end) {
    if (is_target) {
        if (subtract_self)
            l2p_cell_impl<P, true, true>(ps, perm, is_target, w, Gx, Gy, lox, loy, loz, cell, inv_sigma, C,
                                         u_out, kx, ky, kz, start, end);
        else
            l2p_cell_impl<P, true, false>(ps, perm, is_target, w, Gx, Gy, lox, loy, loz, cell, inv_sigma, C,
                                          u_out, kx, ky, kz, start, end);
    } else {
        if (subtract_self)
            l2p_cell_impl<P, false, true>(ps, perm, is_target, w, Gx, Gy, lox, loy, loz, cell, inv_sigma, C,
                                          u_out, kx, ky, kz, start, end);
        else
            l2p_cell_impl<P, false, false>(ps, perm, is_target, w, Gx, Gy, lox, loy, loz, cell, inv_sigma,
                                           C, u_out, kx, ky, kz, start, end);
    }
}

template <int P>
__global__ void __launch_bounds__(kBlock) k_l2p(const uint64_t *keys, int64_t n, const float4 *ps,
                                                const int32_t *perm, const uint8_t *is_target,
                                                const float *w, int subtract_self, int level, int Gx,
                                                int Gy, int Gz, double lox, double loy, double loz,
                                                double cell, double inv_sigma, const float *C,
                                                float *u_out) {
    const int64_t g = blockIdx.x;
    const int kx = (int)(g % Gx), ky = (int)((g / Gx) % Gy), kz = (int)(g / ((int64_t)Gx * Gy));
    int64_t start, end;
    cell_range(keys, n, level, kx, ky, kz, start, end);
    if (start == end) return;
    l2p_cell<P>(ps, perm, is_target, w, subtract_self, Gx, Gy, lox, loy, loz, cell, inv_sigma, C, u_out,
                kx, ky, kz, start, end);
}

// ---------------------------------------------------------------------------------
// Two-level variant.  Moments are formed at the 4 x 4 x 4 sub-cells two levels
// below the expansion level with pf < p terms (P2M), shifted to the expansion
// cell with M2M, translated there (M2L), and shifted back to the sub-cells with
// L2L truncated to pf terms for L2P.  The sub-cells of a cell are contiguous in
// key order, and sub-cell s = (d1 << 3) | d2 (two octant digits) sits at offset
// (k - 1.5) h_f along each axis, k in 0..3, from the cell centre.  Both shifts are
// done as one separable contraction over the 64 sub-cells, axis by axis:
//   M2M  A[a] = sum_s sum_{g<=a, g<pf} a_s[g] prod_k d_k^(a_k-g_k)/(a_k-g_k)!
//   L2L  c_s[b] = sum_{g>=b} C[g] prod_k binom(g_k, b_k) d_k^(g_k-b_k),  b < pf
// ---------------------------------------------------------------------------------

// Orders LDS accesses among the lanes of one wavefront (the lanes run in lockstep;
// this keeps the compiler from moving LDS reads above the wave's writes and waits
// for them to land).
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int sub_coord(int s, int axis) {
    const int d1 = s >> 3, d2 = s & 7, sh = 2 - axis;
    return (((d1 >> sh) & 1) << 1) | ((d2 >> sh) & 1);
}

// Shift tables for the four sub-cell offsets along an axis: m2m[k][m] = d_k^m/m!,
// l2l[k][g][b] = binom(g, b) d_k^(g-b), d_k = (k - 1.5) * hf / sigma.
template <int P>
__device__ inline void shift_tables(double hf_over_sigma, float (*m2m)[P], float (*l2l)[P][P]) {
    for (int e = threadIdx.x; e < 4 * P; e += blockDim.x) {
        const int k = e / P, m = e % P;
        const double d = (k - 1.5) * hf_over_sigma;
        double v = 1.0;
        for (int q = 1; q <= m; ++q) v *= d / q;
        m2m[k][m] = (float)v;
    }
    for (int e = threadIdx.x; e < 4 * P * P; e += blockDim.x) {
        const int k = e / (P * P), g = (e / P) % P, b = e % P;
        const double d = (k - 1.5) * hf_over_sigma;
        double v = 0.0;
        if (g >= b) {
            double binom = 1.0;
            for (int q = 1; q <= b; ++q) binom = binom * (g - b + q) / q;
            v = binom;
            for (int q = 0; q < g - b; ++q) v *= d;
        }
        l2l[k][g][b] = (float)v;
    }
}

template <int P, int PF>
__global__ void __launch_bounds__(kBlock) k_p2m_2lvl(const uint64_t *keys, int64_t n, const float4 *ps,
                                                     const int32_t *perm, const float *w, int level,
                                                     int Gx, int Gy, int Gz, double lox, double loy,
                                                     double loz, double cell, double inv_sigma, float *A) {
    constexpr int P3 = P * P * P;
    constexpr int pf = PF, pf2 = PF * PF, pf3 = PF * PF * PF;
    constexpr int NG = 64 / pf2;                             // point groups per wave
    __shared__ float As[64 * pf3];                           // [s][gz][gy][gx]
    __shared__ float B1[16 * pf2 * P];                       // [sy][sz][gz][gy][ax]
    __shared__ float B2[4 * pf * P * P];                     // [sz][gz][ay][ax]
    __shared__ float sm2m[4][P];
    __shared__ float sl2l[4][P][P];
    __shared__ int64_t bnd[65];
    __shared__ float4 stage[kBlock / 64][64];
    const int64_t g = blockIdx.x;
    const int kx = (int)(g % Gx), ky = (int)((g / Gx) % Gy), kz = (int)(g / ((int64_t)Gx * Gy));
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const double hf = cell * 0.25;
    {
        const uint64_t prefix = morton3((uint32_t)kx, (uint32_t)ky, (uint32_t)kz);
        const int shf = 3 * (kDepth - level - 2);
        if (tid <= 64) {
            const uint64_t key = tid < 64 ? ((prefix << 6) | (uint64_t)tid) << shf
                                          : ((prefix + 1ull) << 6) << shf;
            bnd[tid] = lower_bound_u64(keys, 0, n, key);
        }
    }
    shift_tables<P>(hf * inv_sigma, sm2m, sl2l);
    __syncthreads();
    const double cx = lox + (kx + 0.5) * cell, cy = loy + (ky + 0.5) * cell, cz = loz + (kz + 0.5) * cell;
    // fine moments: wave w takes sub-cells w, w+4, ...  Each chunk of up to 64
    // points is first staged by the wave (one point per lane, so the weight
    // gathers are independent), then lane = (group, gy, gz) keeps the pf moments
    // along x and walks every NG-th staged point.
    const int grp = lane / pf2, pair = lane % pf2, gy = pair % pf, gz = pair / pf;
    const bool active = grp < NG;
    float4 *stg = stage[wid];
    for (int s0 = 0; s0 < 64; s0 += 4) {
        const int s = s0 + wid;
        const double sx = cx + (sub_coord(s, 0) - 1.5) * hf, sy = cy + (sub_coord(s, 1) - 1.5) * hf,
                     sz = cz + (sub_coord(s, 2) - 1.5) * hf;
        float acc[PF];
#pragma unroll
        for (int a = 0; a < PF; ++a) acc[a] = 0.f;
        for (int64_t c0 = bnd[s]; c0 < bnd[s + 1]; c0 += 64) {
            const int m = bnd[s + 1] - c0 < 64 ? (int)(bnd[s + 1] - c0) : 64;
            if (lane < m) {
                const float4 q = ps[c0 + lane];
                stg[lane] = make_float4(((q.x - (float)sx) * (float)inv_sigma),
                                        ((q.y - (float)sy) * (float)inv_sigma),
                                        ((q.z - (float)sz) * (float)inv_sigma), w ? w[perm[c0 + lane]] : q.w);
            }
            wave_sync();
            if (active) {
                for (int j = grp; j < m; j += NG) {
                    const float4 q = stg[j];
                    float f = q.w;
#pragma unroll
                    for (int k = 1; k < PF; ++k) {
                        f = k <= gy ? f * q.y : f;
                        f = k <= gz ? f * q.z : f;
                    }
#pragma unroll
                    for (int a = 0; a < PF; ++a) {
                        acc[a] += f;
                        f *= q.x;
                    }
                }
            }
            wave_sync();
        }
        // point groups in order (lanes pf2 apart), then 1/(gx! gy! gz!)
#pragma unroll
        for (int a = 0; a < PF; ++a) {
            float tot = 0.f;
            for (int q = 0; q < NG; ++q) tot += __shfl(acc[a], pair + q * pf2, 64);
            acc[a] = tot;
        }
        if (grp == 0) {
            float fy = 1.f, fz = 1.f;
            for (int k = 2; k <= gy; ++k) fy *= (float)k;
            for (int k = 2; k <= gz; ++k) fz *= (float)k;
            float fx = 1.f;
#pragma unroll
            for (int a = 0; a < PF; ++a) {
                if (a > 1) fx *= (float)a;
                As[s * pf3 + (gz * pf + gy) * pf + a] = acc[a] / (fx * fy * fz);
            }
        }
    }
    __syncthreads();
    // x: B1[sy][sz][gz][gy][ax] = sum_sx sum_{gx<=ax} As[s][gz][gy][gx] m2m[sx][ax-gx]
    for (int e = tid; e < 16 * pf2 * P; e += kBlock) {
        const int ax = e % P, gy = (e / P) % pf, zz = (e / (P * pf)) % pf, yzs = e / (P * pf2);
        const int syi = yzs >> 2, szi = yzs & 3;
        float acc = 0.f;
        for (int sxi = 0; sxi < 4; ++sxi) {
            // sub-cell index with coordinates (sxi, syi, szi)
            const int d1 = ((sxi >> 1) << 2) | ((syi >> 1) << 1) | (szi >> 1);
            const int d2 = ((sxi & 1) << 2) | ((syi & 1) << 1) | (szi & 1);
            const float *a_s = As + ((d1 << 3) | d2) * pf3 + (zz * pf + gy) * pf;
            for (int gx = 0; gx <= ax && gx < pf; ++gx) acc = fmaf(a_s[gx], sm2m[sxi][ax - gx], acc);
        }
        B1[e] = acc;
    }
    __syncthreads();
    // y: B2[sz][gz][ay][ax] = sum_sy sum_{gy<=ay} B1[sy][sz][gz][gy][ax] m2m[sy][ay-gy]
    for (int e = tid; e < 4 * pf * P * P; e += kBlock) {
        const int ax = e % P, ay = (e / P) % P, zz = (e / (P * P)) % pf, szi = e / (P * P * pf);
        float acc = 0.f;
        for (int syi = 0; syi < 4; ++syi) {
            const float *b1 = B1 + (((syi << 2) | szi) * pf + zz) * pf * P;
            for (int gy = 0; gy <= ay && gy < pf; ++gy) acc = fmaf(b1[gy * P + ax], sm2m[syi][ay - gy], acc);
        }
        B2[e] = acc;
    }
    __syncthreads();
    // z: A[az][ay][ax] = sum_sz sum_{gz<=az} B2[sz][gz][ay][ax] m2m[sz][az-gz]
    const int64_t Rx = (int64_t)Gx * P, Ry = (int64_t)Gy * P;
    for (int e = tid; e < P3; e += kBlock) {
        const int ax = e % P, ay = (e / P) % P, az = e / (P * P);
        float acc = 0.f;
        for (int szi = 0; szi < 4; ++szi)
            for (int zz = 0; zz <= az && zz < pf; ++zz)
                acc = fmaf(B2[((szi * pf + zz) * P + ay) * P + ax], sm2m[szi][az - zz], acc);
        A[(((int64_t)kz * P + az) * Ry + (int64_t)ky * P + ay) * Rx + (int64_t)kx * P + ax] = acc;
    }
}

template <int P, int PF>
__global__ void __launch_bounds__(kBlock) k_l2p_2lvl(const uint64_t *keys, int64_t n, const float4 *ps,
                                                     const int32_t *perm, const uint8_t *is_target,
                                                     const float *w, int subtract_self, int level,
                                                     int Gx, int Gy, int Gz, double lox, double loy,
                                                     double loz, double cell, double inv_sigma,
                                                     const float *C, float *u_out) {
    constexpr int P3 = P * P * P;
    constexpr int pf = PF, pf2 = PF * PF, pf3 = PF * PF * PF;
    __shared__ float sC[P3];                 // [az][ay][ax]
    __shared__ float D1[4 * pf * P * P];     // [sz][bz][ay][ax]
    __shared__ float D2[16 * pf2 * P];       // [sy][sz][bz][by][ax]
    __shared__ float cs[16 * pf3];           // [s - s_group][bz][by][bx]
    __shared__ float sm2m[4][P];
    __shared__ float sl2l[4][P][P];
    __shared__ int64_t bnd[65];
    const int64_t g = blockIdx.x;
    const int kx = (int)(g % Gx), ky = (int)((g / Gx) % Gy), kz = (int)(g / ((int64_t)Gx * Gy));
    const int tid = threadIdx.x;
    const double hf = cell * 0.25;
    {
        const uint64_t prefix = morton3((uint32_t)kx, (uint32_t)ky, (uint32_t)kz);
        const int shf = 3 * (kDepth - level - 2);
        if (tid <= 64) {
            const uint64_t key = tid < 64 ? ((prefix << 6) | (uint64_t)tid) << shf
                                          : ((prefix + 1ull) << 6) << shf;
            bnd[tid] = lower_bound_u64(keys, 0, n, key);
        }
    }
    shift_tables<P>(hf * inv_sigma, sm2m, sl2l);
    const int64_t Rx = (int64_t)Gx * P, Ry = (int64_t)Gy * P;
    for (int e = tid; e < P3; e += kBlock) {
        const int ax = e % P, ay = (e / P) % P, az = e / (P * P);
        sC[e] = C[(((int64_t)kz * P + az) * Ry + (int64_t)ky * P + ay) * Rx + (int64_t)kx * P + ax];
    }
    __syncthreads();
    if (bnd[0] == bnd[64]) return;
    // z: D1[sz][bz][ay][ax] = sum_{gz>=bz} C[gz][ay][ax] l2l[sz][gz][bz]
    for (int e = tid; e < 4 * pf * P * P; e += kBlock) {
        const int axy = e % (P * P), bz = (e / (P * P)) % pf, szi = e / (P * P * pf);
        float acc = 0.f;
        for (int gz = bz; gz < P; ++gz) acc = fmaf(sC[gz * P * P + axy], sl2l[szi][gz][bz], acc);
        D1[e] = acc;
    }
    __syncthreads();
    // y: D2[sy][sz][bz][by][ax] = sum_{gy>=by} D1[sz][bz][gy][ax] l2l[sy][gy][by]
    for (int e = tid; e < 16 * pf2 * P; e += kBlock) {
        const int ax = e % P, by = (e / P) % pf, bz = (e / (P * pf)) % pf, yzs = e / (P * pf2);
        const int syi = yzs >> 2, szi = yzs & 3;
        const float *d1 = D1 + (szi * pf + bz) * P * P;
        float acc = 0.f;
        for (int gy = by; gy < P; ++gy) acc = fmaf(d1[gy * P + ax], sl2l[syi][gy][by], acc);
        D2[e] = acc;
    }
    __syncthreads();
    // x stage and evaluation in four groups of 16 sub-cells:
    //   cs[s][bz][by][bx] = sum_{gx>=bx} D2[sy][sz][bz][by][gx] l2l[sx][gx][bx]
    // then wave w evaluates sub-cells w, w+4, ... of the group at their targets
    const int lane = tid & 63, wid = tid >> 6;
    const double cx = lox + (kx + 0.5) * cell, cy = loy + (ky + 0.5) * cell, cz = loz + (kz + 0.5) * cell;
    for (int sg = 0; sg < 64; sg += 16) {
        for (int e = tid; e < 16 * pf3; e += kBlock) {
            const int bx = e % pf, by = (e / pf) % pf, bz = (e / pf2) % pf, sidx = sg + e / pf3;
            const int sxi = sub_coord(sidx, 0), syi = sub_coord(sidx, 1), szi = sub_coord(sidx, 2);
            const float *d2 = D2 + ((((syi << 2) | szi) * pf + bz) * pf + by) * P;
            float acc = 0.f;
            for (int gx = bx; gx < P; ++gx) acc = fmaf(d2[gx], sl2l[sxi][gx][bx], acc);
            cs[e] = acc;
        }
        __syncthreads();
        for (int s0 = 0; s0 < 16; s0 += 4) {
            const int sidx = sg + s0 + wid;
            const double sx = cx + (sub_coord(sidx, 0) - 1.5) * hf, sy = cy + (sub_coord(sidx, 1) - 1.5) * hf,
                         sz = cz + (sub_coord(sidx, 2) - 1.5) * hf;
            const float *c = cs + (s0 + wid) * pf3;
            for (int64_t i = bnd[sidx] + lane; i < bnd[sidx + 1]; i += 64) {
                const float4 q = ps[i];
                const float X = ((q.x - (float)sx) * (float)inv_sigma);
                const float Y = ((q.y - (float)sy) * (float)inv_sigma);
                const float Z = ((q.z - (float)sz) * (float)inv_sigma);
                float uz = 0.f;
#pragma unroll
                for (int bz = pf - 1; bz >= 0; --bz) {
                    float uy = 0.f;
#pragma unroll
                    for (int by = pf - 1; by >= 0; --by) {
                        const float *row = c + (bz * pf + by) * pf;
                        float ux = row[pf - 1];
#pragma unroll
                        for (int bx = pf - 2; bx >= 0; --bx) ux = fmaf(ux, X, row[bx]);
                        uy = fmaf(uy, Y, ux);
                    }
                    uz = fmaf(uz, Z, uy);
                }
                const int32_t j = perm[i];
                const bool tg = !is_target || is_target[j];
                u_out[j] = tg ? (subtract_self ? uz - w[j] : uz) : 0.f;
            }
        }
        __syncthreads();
    }
}

// Value, gradient and (LAP) Laplacian of a cell's Taylor series (coefficients sC in
// the order [az][ay][ax]) at the offset (X, Y, Z) from its centre, in sigma;
// is = 1/sigma.  Nested Horner: along x the row polynomial r and r' (and r''); along
// y the row sums of r, r' (r'') and the first (two) y-derivatives of the sum of r;
// along z the same for the values of that level.
template <int P, bool LAP>
__device__ inline void l2p_grad_point_t(const float *sC, float X, float Y, float Z, float is, float *o) {
    // z level accumulators of: v0 (value), v1 (d/dx), v2 (d2/dx2), w1 (d/dy), w2 (d2/dy2)
    float z0 = 0.f, z1 = 0.f, z2 = 0.f, zy1 = 0.f, zy2 = 0.f, zd1 = 0.f, zd2 = 0.f;
    for (int az = P - 1; az >= 0; --az) {
        float y0 = 0.f, y1 = 0.f, y2 = 0.f, yd1 = 0.f, yd2 = 0.f;
#pragma unroll
        for (int ay = P - 1; ay >= 0; --ay) {
            const float *c = sC + (az * P + ay) * P;
            float r0 = c[P - 1], r1 = 0.f, r2 = 0.f;
#pragma unroll
            for (int ax = P - 2; ax >= 0; --ax) {
                if (LAP) r2 = fmaf(r2, X, r1);
                r1 = fmaf(r1, X, r0);
                r0 = fmaf(r0, X, c[ax]);
            }
            // Horner in Y for the sums of r0, r1, r2 and derivatives of the r0 sum
            if (LAP) yd2 = fmaf(yd2, Y, yd1);
            yd1 = fmaf(yd1, Y, y0);
            y0 = fmaf(y0, Y, r0);
            y1 = fmaf(y1, Y, r1);
            if (LAP) y2 = fmaf(y2, Y, r2);
        }
        if (LAP) zd2 = fmaf(zd2, Z, zd1);
        zd1 = fmaf(zd1, Z, z0);
        z0 = fmaf(z0, Z, y0);
        z1 = fmaf(z1, Z, y1);
        if (LAP) z2 = fmaf(z2, Z, 2.f * y2);
        zy1 = fmaf(zy1, Z, yd1);
        if (LAP) zy2 = fmaf(zy2, Z, 2.f * yd2);
    }
    o[0] = z0;   // value, gradient x y z, Laplacian
    o[1] = z1 * is;
    o[2] = zy1 * is;
    o[3] = zd1 * is;
    if (LAP) o[4] = (z2 + zy2 + 2.f * zd2) * is * is;
}

template <int P>
__device__ inline void l2p_grad_point(const float *sC, float X, float Y, float Z, float is, int want_lap, float *o) {
    if (want_lap) l2p_grad_point_t<P, true>(sC, X, Y, Z, is, o);
    else l2p_grad_point_t<P, false>(sC, X, Y, Z, is, o);
}

// L2P with derivatives at every point of each cell (in key order), one block per cell.
template <int P>
__global__ void __launch_bounds__(kBlock) k_l2p_grad(const uint64_t *keys, int64_t n, const float4 *ps,
                                                     int level, int Gx, int Gy, int Gz, double lox,
                                                     double loy, double loz, double cell,
                                                     double inv_sigma, const float *C, float *out,
                                                     int stride, int want_lap) {
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
    const float is = (float)inv_sigma;
    for (int64_t i = start + threadIdx.x; i < end; i += kBlock) {
        const float4 q = ps[i];
        const float X = ((q.x - (float)cx) * (float)inv_sigma);
        const float Y = ((q.y - (float)cy) * (float)inv_sigma);
        const float Z = ((q.z - (float)cz) * (float)inv_sigma);
        l2p_grad_point<P>(sC, X, Y, Z, is, want_lap, out + i * stride);
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
    const float *w;          // input order (self term)
    const float *w_gather;   // gathered by the P2M through the permutation; NULL: staged in ps.w
    const uint8_t *is_target;
    int subtract_self;
    float *u_out;
    bool stage;   // P2M writes the gathered weights into the sorted records (MSP_STAGE_WEIGHTS)
};

// Target flags and the self term applied in input order after an L2P that wrote
// every point's sum: reading the flags and weights here is coalesced, where the
// L2P would have gathered them through the permutation.
__global__ void k_finish_u(int64_t n, const uint8_t *is_target, const float *w, int subtract_self, float *u) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    const bool tg = !is_target || is_target[j];
    u[j] = tg ? (subtract_self ? u[j] - w[j] : u[j]) : 0.f;
}

// The same four points per thread with 16-byte loads and stores of u and w and a
// 4-byte load of the flags (u and w 16-byte aligned, the flags 4-byte aligned,
// checked by the caller); the last n % 4 points one by one.
__global__ void k_finish_u4(int64_t n, const uint8_t *is_target, const float *w, int subtract_self, float *u) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t j0 = 4 * q;
    if (j0 + 4 <= n) {
        float4 v = reinterpret_cast<float4 *>(u)[q];
        if (subtract_self) {
            const float4 s = reinterpret_cast<const float4 *>(w)[q];
            v.x -= s.x;
            v.y -= s.y;
            v.z -= s.z;
            v.w -= s.w;
        }
        if (is_target) {
            const uint32_t f = reinterpret_cast<const uint32_t *>(is_target)[q];
            v.x = (f & 0xffu) ? v.x : 0.f;
            v.y = (f & 0xff00u) ? v.y : 0.f;
            v.z = (f & 0xff0000u) ? v.z : 0.f;
            v.w = (f & 0xff000000u) ? v.w : 0.f;
        }
        reinterpret_cast<float4 *>(u)[q] = v;
    } else {
        for (int64_t j = j0; j < n; ++j) {
            const bool tg = !is_target || is_target[j];
            u[j] = tg ? (subtract_self ? u[j] - w[j] : u[j]) : 0.f;
        }
    }
}

template <int P, int PF>
int launch_2lvl(msp_tree *t, const FgtPlan &pl, double inv_sigma, bool l2p, const float *C, float *A,
                const GridArgs &ga, hipStream_t s) {
    const int64_t ncell = (int64_t)pl.G[0] * pl.G[1] * pl.G[2];
    if (!l2p)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_p2m_2lvl<P, PF>), dim3((unsigned)ncell), dim3(kBlock), 0, s,
                           t->keys.as<uint64_t>(), t->n, t->ps.as<float4>(), t->perm.as<int32_t>(), ga.w_gather,
                           pl.level, pl.G[0], pl.G[1], pl.G[2], t->geo.lo[0], t->geo.lo[1], t->geo.lo[2],
                           pl.cell, inv_sigma, A);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_l2p_2lvl<P, PF>), dim3((unsigned)ncell), dim3(kBlock), 0, s,
                           t->keys.as<uint64_t>(), t->n, t->ps.as<float4>(), t->perm.as<int32_t>(),
                           ga.is_target, ga.w, ga.subtract_self, pl.level, pl.G[0], pl.G[1], pl.G[2],
                           t->geo.lo[0], t->geo.lo[1], t->geo.lo[2], pl.cell, inv_sigma, C, ga.u_out);
    MSP_CHECK_LAUNCH();
    return MSP_OK;
}

template <int P>
int launch_p2m_l2p(msp_tree *t, const FgtPlan &pl, double inv_sigma, bool l2p, const float *C,
                   float *A, const GridArgs &ga, hipStream_t s) {
    const int64_t ncell = (int64_t)pl.G[0] * pl.G[1] * pl.G[2];
    if constexpr (P >= 6 && P <= 8) {
        if (pl.pf > 0) {
            switch (pl.pf) {
                case 3: return launch_2lvl<P, 3>(t, pl, inv_sigma, l2p, C, A, ga, s);
                case 4: return launch_2lvl<P, 4>(t, pl, inv_sigma, l2p, C, A, ga, s);
                case 5: return launch_2lvl<P, 5>(t, pl, inv_sigma, l2p, C, A, ga, s);
                default: return fail(MSP_EINVAL, "two-level terms %d not built", pl.pf);
            }
        }
    }
    if (!l2p && P == 8) {
        hipLaunchKernelGGL(k_p2m_mfma8, dim3((unsigned)ncell), dim3(kBlock), 0, s, t->keys.as<uint64_t>(), t->n,
                           t->ps.as<float4>(), t->perm.as<int32_t>(), ga.w_gather, pl.level, pl.G[0], pl.G[1], pl.G[2],
                           t->geo.lo[0], t->geo.lo[1], t->geo.lo[2], pl.cell, inv_sigma, A,
                           ga.stage ? t->ps.as<float4>() : nullptr);
    } else if (!l2p) {
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_p2m<P>), dim3((unsigned)ncell), dim3(kBlock), 0, s,
                           t->keys.as<uint64_t>(), t->n, t->ps.as<float4>(), t->perm.as<int32_t>(),
                           ga.w_gather, pl.level, pl.G[0], pl.G[1], pl.G[2], t->geo.lo[0], t->geo.lo[1],
                           t->geo.lo[2], pl.cell, inv_sigma, A, ga.stage ? t->ps.as<float4>() : nullptr);
    } else {
        // every point's sum straight to input order, flags and self term afterwards
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_l2p<P>), dim3((unsigned)ncell), dim3(kBlock), 0, s,
                           t->keys.as<uint64_t>(), t->n, t->ps.as<float4>(), t->perm.as<int32_t>(),
                           (const uint8_t *)nullptr, ga.w, 0, pl.level, pl.G[0], pl.G[1], pl.G[2],
                           t->geo.lo[0], t->geo.lo[1], t->geo.lo[2], pl.cell, inv_sigma, C, ga.u_out);
        // (the target flags and the self term follow in fgt_forward_grid)
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

namespace {
template <int P>
int launch_l2p_grad(msp_tree *t, const FgtPlan &pl, double inv_sigma, const float *C, float *out,
                    int stride, int want_lap, hipStream_t s) {
    const int64_t ncell = (int64_t)pl.G[0] * pl.G[1] * pl.G[2];
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_l2p_grad<P>), dim3((unsigned)ncell), dim3(kBlock), 0, s,
                       t->keys.as<uint64_t>(), t->n, t->ps.as<float4>(), pl.level, pl.G[0], pl.G[1],
                       pl.G[2], t->geo.lo[0], t->geo.lo[1], t->geo.lo[2], pl.cell, inv_sigma, C, out,
                       stride, want_lap);
    MSP_CHECK_LAUNCH();
    return MSP_OK;
}
}  // namespace

int fgt_field_grad(msp_tree *t, const FgtPlan &pl, const msp_fgt_params *prm, const float *w,
                   float *out, int stride, int want_lap, hipStream_t s) {
    // moments of w, all-pairs translation, then value/gradient/Laplacian at every point
    msp_fgt_params q = *prm;
    q.flags &= ~(uint32_t)MSP_TWO_LEVEL;
    FgtPlan p1 = pl;
    p1.pf = 0;
    MSP_TRY(fgt_forward_grid(t, p1, &q, w, nullptr, nullptr, s));
    const double inv_sigma = 1.0 / prm->sigma;
    const float *C = t->gridB.as<float>();
    PhaseScope ps(&t->timing, PH_L2P, s);
    switch (pl.p) {
#define CASE(P) case P: return launch_l2p_grad<P>(t, pl, inv_sigma, C, out, stride, want_lap, s);
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
        CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16)
#undef CASE
    }
    return fail(MSP_EINVAL, "p out of range");
}

// ---------------------------------------------------------------------------------
// Batches of expansion-route populations: one launch per pass covers all of them.
// Work units are (population, operator), (population, grid float), (population,
// node) and (population, M2L tile), located by binary search in prefix sums.
// P2M and L2P run over "ranges": the nodes at the expansion level and the leaves
// above it, each holding whole cells of that level (split by key prefix).
namespace {

__device__ inline int find_pop(const int64_t *off, int npop, int64_t x) {
    int lo = 0, hi = npop;   // off[lo] <= x < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ void k_bops(FgtBatchPlan bp) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= bp.n_ops) return;
    const int k = find_pop(bp.ops_off, bp.npop, g);
    const FgtPop &f = bp.pops[k];
    m2l_ops_one(bp.p, f.G[0], f.G[1], f.G[2], f.step, f.opsx, f.opsy, f.opsz, (int)(g - bp.ops_off[k]));
}

// zero moment grids (cells without points are never written by the P2M), clear
// the cell counters and the timestamps.  Each population's grid is cleared
// in 16-byte stores by all threads (grids start at allocation boundaries).
__global__ void k_bclear(FgtBatchPlan bp) {
    const int64_t g0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    if (g0 == 0) {
        bp.ncells[0] = 0;
        bp.ncells[1] = 0;
    }
    if (g0 < bp.npop) {
        bp.stamps[2 * bp.pops[g0].pop] = ~0ull;
        bp.stamps[2 * bp.pops[g0].pop + 1] = 0ull;
    }
    for (int k = 0; k < bp.npop; ++k) {
        float *A = bp.pops[k].A;
        const int64_t n = bp.grid_off[k + 1] - bp.grid_off[k];
        const int64_t n4 = n / 4;
        float4 *A4 = reinterpret_cast<float4 *>(A);
        for (int64_t g = g0; g < n4; g += nth) A4[g] = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int64_t g = 4 * n4 + g0; g < n; g += nth) A[g] = 0.f;
    }
}

// Occupied cells of every population.  A window is 64 consecutive points (key
// order) of one population, one point per lane: a lane whose point starts a cell
// (its level prefix differs from the previous point's) ends it at the next lane that
// starts a cell or lies past the population; the cell that runs past the window is
// followed 64 keys at a time.  Cells of at most cmax points go to the front of the
// list, larger ones to the back, as (population, first point, points, cell index).
// A wavefront takes kCellWin consecutive windows and makes one atomic addition per
// list for all of them (additions on one address are serialised by the memory
// system).
constexpr int kCellWin = 16;
__global__ void __launch_bounds__(256) k_bcells(FgtBatchPlan bp, int cmax) {
    const int lane = threadIdx.x & 63;
    const int64_t w0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * kCellWin;
    if (w0 >= bp.n_pw) return;   // whole wavefronts
    int4 cw[kCellWin];
    uint64_t msw[kCellWin], mbw[kCellWin];
    int ns = 0, nb = 0;
#pragma unroll
    for (int q = 0; q < kCellWin; ++q) {
        const int64_t wv = w0 + q;
        bool emit = false, small = false;
        cw[q] = make_int4(0, 0, 0, 0);
        if (wv < bp.n_pw) {
            const int k = find_pop(bp.pw_off, bp.npop, wv);
            const FgtPop &f = bp.pops[k];
            const int sh = 3 * (kDepth - f.level);
            const int64_t base = (wv - bp.pw_off[k]) * 64, i = base + lane;
            const bool in = i < f.n;
            const uint64_t pre = in ? f.keys[i] >> sh : 0ull;
            uint64_t prev = __shfl_up(pre, 1, 64);
            if (lane == 0) prev = base > 0 ? f.keys[base - 1] >> sh : ~0ull;
            const bool start = in && (i == 0 || prev != pre);
            const uint64_t bound = __ballot(start || !in);
            const uint64_t starts = __ballot(start);
            if (starts) {
                // end of the cell of the last starting lane, when it runs past the window
                const int last = 63 - __clzll(starts);
                const uint64_t after = last < 63 ? (bound >> (last + 1)) : 0ull;
                int64_t tail = -1;
                if (after == 0ull) {
                    const uint64_t lp = __shfl(pre, last, 64);
                    int64_t e0 = base + 64;
                    for (;;) {
                        const int64_t j = e0 + lane;
                        const uint64_t m = __ballot(j >= f.n || (f.keys[j] >> sh) != lp);
                        if (m) {
                            tail = e0 + __ffsll((unsigned long long)m) - 1;
                            break;
                        }
                        e0 += 64;
                    }
                }
                if (start) {
                    const uint64_t nxb = lane < 63 ? (bound >> (lane + 1)) : 0ull;
                    const int64_t e = nxb ? i + __ffsll((unsigned long long)nxb) : tail;
                    const int kx = (int)compact3(pre >> 2), ky = (int)compact3(pre >> 1), kz = (int)compact3(pre);
                    cw[q] = make_int4(k, (int)i, (int)(e - i), (kz * f.G[1] + ky) * f.G[0] + kx);
                    emit = true;
                    small = e - i <= cmax;
                }
            }
        }
        msw[q] = __ballot(emit && small);
        mbw[q] = __ballot(emit && !small);
        ns += (int)__popcll(msw[q]);
        nb += (int)__popcll(mbw[q]);
    }
    int bs = 0, bb = 0;
    if (lane == 0) {
        if (ns) bs = atomicAdd(&bp.ncells[0], ns);
        if (nb) bb = atomicAdd(&bp.ncells[1], nb);
    }
    bs = __shfl(bs, 0, 64);
    bb = __shfl(bb, 0, 64);
    const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll
    for (int q = 0; q < kCellWin; ++q) {
        if ((msw[q] >> lane) & 1ull) bp.cells[bs + __popcll(msw[q] & below)] = cw[q];
        if ((mbw[q] >> lane) & 1ull) bp.cells[bp.cap - 1 - (bb + __popcll(mbw[q] & below))] = cw[q];
        bs += (int)__popcll(msw[q]);
        bb += (int)__popcll(mbw[q]);
    }
}

__device__ inline void cell_coords(const FgtPop &f, int cidx, int &kx, int &ky, int &kz) {
    kx = cidx % f.G[0];
    ky = (cidx / f.G[0]) % f.G[1];
    kz = cidx / (f.G[0] * f.G[1]);
}

// index of coefficient (ax, ay, az) of cell (kx, ky, kz): cell-major or interleaved
template <int P>
__device__ inline int64_t grid_index(const FgtPop &f, int cm, int kx, int ky, int kz, int ax, int ay, int az) {
    if (cm) return ((((int64_t)kz * f.G[1] + ky) * f.G[0] + kx) * P + az) * (P * P) + ay * P + ax;
    const int64_t Rx = (int64_t)f.G[0] * P, Ry = (int64_t)f.G[1] * P;
    return (((int64_t)kz * P + az) * Ry + (int64_t)ky * P + ay) * Rx + (int64_t)kx * P + ax;
}

// Moments of the points [s0, e) of one cell by one wavefront, written into the
// grid (normalisation as p2m_cell; cell-major layout when cm is set, else
// interleaved).  Points pass through LDS 64 at a
// time.  For p = 1, 2, 4, 8 a lane (point group, ay half, az) accumulates its (ay, ax)
// block over every NG-th point and the groups are added by butterfly shuffles;
// otherwise a lane owns whole (ay, az) rows and visits every point.
template <int P>
__device__ void p2m_cell_wave(const float4 *ps, const int32_t *perm, const float *w, int Gx, int Gy,
                              const double *lo, double cell, double inv_sigma, float *A, int cm, int kx, int ky,
                              int kz, int64_t s0, int64_t e, float4 *stage) {
    constexpr bool ILP = P == 1 || P == 2 || P == 4 || P == 8;
    const int lane = threadIdx.x & 63;
    const double cx = lo[0] + (kx + 0.5) * cell, cy = lo[1] + (ky + 0.5) * cell, cz = lo[2] + (kz + 0.5) * cell;
    const int64_t Rx = (int64_t)Gx * P, Ry = (int64_t)Gy * P;
    const int64_t cbase = (((int64_t)kz * Gy + ky) * Gx + kx) * (P * P * P);
    auto out = [&](int ax, int ay, int az, float v) {
        if (cm) A[cbase + (az * P + ay) * P + ax] = v;
        else A[(((int64_t)kz * P + az) * Ry + (int64_t)ky * P + ay) * Rx + (int64_t)kx * P + ax] = v;
    };
    auto stage_chunk = [&](int64_t c0) {
        const int64_t j = c0 + lane;
        float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
        if (j < e) {
            const float4 t = ps[j];
            q = make_float4(((t.x - (float)cx) * (float)inv_sigma), ((t.y - (float)cy) * (float)inv_sigma),
                            ((t.z - (float)cz) * (float)inv_sigma), w[perm[j]]);
        }
        return q;
    };
    if constexpr (ILP) {
        constexpr int H = P == 8 ? 2 : 1;
        constexpr int AY = P / H;
        constexpr int NG = 64 / (P * H);
        const int az = lane % P, ah = (lane / P) % H, grp = lane / (P * H);
        float a2[AY][P];
#pragma unroll
        for (int i = 0; i < AY; ++i)
#pragma unroll
            for (int ax = 0; ax < P; ++ax) a2[i][ax] = 0.f;
        float4 nxt = stage_chunk(s0);
        for (int64_t c0 = s0; c0 < e; c0 += 64) {
            wave_sync();
            stage[lane] = nxt;
            wave_sync();
            if (c0 + 64 < e) nxt = stage_chunk(c0 + 64);
            const int m = e - c0 < 64 ? (int)(e - c0) : 64;
            for (int jj = grp; jj < m; jj += NG) {
                const float4 q = stage[jj];
                float wz = q.w;
                for (int k = 0; k < az; ++k) wz *= q.z;
                for (int k = 0; k < ah * AY; ++k) wz *= q.y;
                float yp[AY], xp[P];
                yp[0] = wz;
                xp[0] = 1.f;
#pragma unroll
                for (int k = 1; k < AY; ++k) yp[k] = yp[k - 1] * q.y;
#pragma unroll
                for (int k = 1; k < P; ++k) xp[k] = xp[k - 1] * q.x;
#pragma unroll
                for (int i = 0; i < AY; ++i)
#pragma unroll
                    for (int ax = 0; ax < P; ++ax) a2[i][ax] = fmaf(yp[i], xp[ax], a2[i][ax]);
            }
        }
#pragma unroll
        for (int o = P * H; o < 64; o <<= 1)
#pragma unroll
            for (int i = 0; i < AY; ++i)
#pragma unroll
                for (int ax = 0; ax < P; ++ax) a2[i][ax] += __shfl_xor(a2[i][ax], o, 64);
        if (grp == 0) {
            float fz = 1.f;
            for (int k = 2; k <= az; ++k) fz *= (float)k;
            float fy = 1.f;
            for (int k = 2; k <= ah * AY - 1; ++k) fy *= (float)k;
#pragma unroll
            for (int i = 0; i < AY; ++i) {
                const int ay = ah * AY + i;
                if (ay > 1) fy *= (float)ay;
                float fx = 1.f;
#pragma unroll
                for (int ax = 0; ax < P; ++ax) {
                    if (ax > 1) fx *= (float)ax;
                    a2[i][ax] = a2[i][ax] / (fx * fy * fz);
                }
            }
            if (P == 8 && cm) {   // this lane's (ay, ax) block is 32 consecutive floats
                float4 *o = reinterpret_cast<float4 *>(A + cbase + az * 64 + ah * 32);
#pragma unroll
                for (int i = 0; i < AY; ++i)
#pragma unroll
                    for (int h = 0; h < P / 4; ++h)
                        o[i * (P / 4) + h] = make_float4(a2[i][4 * h], a2[i][4 * h + 1], a2[i][4 * h + 2], a2[i][4 * h + 3]);
            } else {
#pragma unroll
                for (int i = 0; i < AY; ++i)
#pragma unroll
                    for (int ax = 0; ax < P; ++ax) out(ax, ah * AY + i, az, a2[i][ax]);
            }
        }
    } else {
        constexpr int P2 = P * P;
        constexpr int RP = (P2 + 63) / 64;
        float acc[RP][P];
#pragma unroll
        for (int rr = 0; rr < RP; ++rr)
#pragma unroll
            for (int ax = 0; ax < P; ++ax) acc[rr][ax] = 0.f;
        float4 nxt = stage_chunk(s0);
        for (int64_t c0 = s0; c0 < e; c0 += 64) {
            wave_sync();
            stage[lane] = nxt;
            wave_sync();
            if (c0 + 64 < e) nxt = stage_chunk(c0 + 64);
            const int m = e - c0 < 64 ? (int)(e - c0) : 64;
            for (int jj = 0; jj < m; ++jj) {
                const float4 q = stage[jj];
                float xp[P];
                xp[0] = 1.f;
#pragma unroll
                for (int k = 1; k < P; ++k) xp[k] = xp[k - 1] * q.x;
#pragma unroll
                for (int rr = 0; rr < RP; ++rr) {
                    const int row = lane + 64 * rr;
                    if (row >= P2) continue;
                    float f = q.w;
                    for (int k = 0; k < row % P; ++k) f *= q.y;
                    for (int k = 0; k < row / P; ++k) f *= q.z;
#pragma unroll
                    for (int ax = 0; ax < P; ++ax) acc[rr][ax] = fmaf(f, xp[ax], acc[rr][ax]);
                }
            }
        }
#pragma unroll
        for (int rr = 0; rr < RP; ++rr) {
            const int row = lane + 64 * rr;
            if (row >= P2) continue;
            const int ay = row % P, az = row / P;
            float fyz = 1.f;
            for (int k = 2; k <= ay; ++k) fyz *= (float)k;
            for (int k = 2; k <= az; ++k) fyz *= (float)k;
            float fx = 1.f;
#pragma unroll
            for (int ax = 0; ax < P; ++ax) {
                if (ax > 1) fx *= (float)ax;
                out(ax, ay, az, acc[rr][ax] / (fx * fyz));
            }
        }
    }
}

// Small cells, eight per wavefront: lane group grp = lane / 8 takes cell r0 + grp,
// whose points pass through LDS eight at a time (zero weight past the end of the
// cell, which adds exact zeros; the next eight are loaded while the current ones
// are used), and each of its eight lanes accumulates a share of the p^3 moments over
// the cell's points in order.  For p = 8 the share of lane sub is the set of 16-byte
// chunks k * 8 + sub (k = 0 .. 15) of the cell-major coefficient block (az = k / 2,
// ay = 4 (k % 2) + sub / 2, ax = 4 (sub % 2) + e), so that every store of the group
// covers one whole 128-byte line; otherwise lane sub takes slice az = sub.  P <= 8.
template <int P>
__device__ void p2m_cells_group(const FgtBatchPlan &bp, int64_t r0, int64_t nsmall, float4 *stage) {
    const int lane = threadIdx.x & 63, grp = lane >> 3, sub = lane & 7;
    const int64_t r = r0 + grp;
    const bool has = r < nsmall;
    const int4 c = has ? bp.cells[r] : make_int4(0, 0, 0, 0);
    const FgtPop &f = bp.pops[c.x];
    if (has && sub == 0 && c.y == 0) atomicMin(&bp.stamps[2 * f.pop], (unsigned long long)wall_clock64());
    int kx = 0, ky = 0, kz = 0;
    if (has) cell_coords(f, c.w, kx, ky, kz);
    const double cx = f.lo[0] + (kx + 0.5) * f.cell, cy = f.lo[1] + (ky + 0.5) * f.cell,
                 cz = f.lo[2] + (kz + 0.5) * f.cell;
    const int cnt = has ? c.z : 0;
    int mx = cnt;
    for (int o = 8; o < 64; o <<= 1) {
        const int t = __shfl_xor(mx, o, 64);
        mx = t > mx ? t : mx;
    }
    auto fetch = [&](int c0) {
        const int j = c0 + sub;
        float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
        if (j < cnt) {
            const float4 t = f.ps[c.y + j];
            q = make_float4(((t.x - (float)cx) * (float)f.inv_sigma), ((t.y - (float)cy) * (float)f.inv_sigma),
                            ((t.z - (float)cz) * (float)f.inv_sigma), f.w[f.perm[c.y + j]]);
        }
        return q;
    };
    constexpr bool CH = P == 8;
    constexpr int NA = CH ? 16 : P, NB = CH ? 4 : P;
    float acc[NA][NB];
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = 0.f;
    const int ya = sub >> 1, xodd = sub & 1;
    float4 nxt = fetch(0);
    for (int c0 = 0; c0 < mx; c0 += 8) {
        wave_sync();
        stage[lane] = nxt;
        wave_sync();
        if (c0 + 8 < mx) nxt = fetch(c0 + 8);
#pragma unroll 2
        for (int t = 0; t < 8; ++t) {
            const float4 q = stage[grp * 8 + t];
            if constexpr (CH) {
                const float x2 = q.x * q.x, y2 = q.y * q.y;
                const float x0 = xodd ? x2 * x2 : 1.f;
                float y0 = 1.f;
                for (int k = 0; k < ya; ++k) y0 *= q.y;
                const float y1 = y0 * (y2 * y2);
                const float xp[4] = {x0, x0 * q.x, x0 * x2, x0 * x2 * q.x};
                float zp = q.w;
#pragma unroll
                for (int az = 0; az < 8; ++az) {
                    const float f0 = zp * y0, f1 = zp * y1;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        acc[2 * az][e] = fmaf(f0, xp[e], acc[2 * az][e]);
                        acc[2 * az + 1][e] = fmaf(f1, xp[e], acc[2 * az + 1][e]);
                    }
                    zp *= q.z;
                }
            } else {
                float wz = q.w;
                for (int k = 0; k < sub; ++k) wz *= q.z;
                float yp[P], xp[P];
                yp[0] = wz;
                xp[0] = 1.f;
#pragma unroll
                for (int k = 1; k < P; ++k) {
                    yp[k] = yp[k - 1] * q.y;
                    xp[k] = xp[k - 1] * q.x;
                }
#pragma unroll
                for (int ay = 0; ay < P; ++ay)
#pragma unroll
                    for (int ax = 0; ax < P; ++ax) acc[ay][ax] = fmaf(yp[ay], xp[ax], acc[ay][ax]);
            }
        }
    }
    if (!has) return;
    auto fact = [](int m) {
        float v = 1.f;
        for (int k = 2; k <= m; ++k) v *= (float)k;
        return v;
    };
    if constexpr (CH) {
        const float fx[4] = {fact(4 * xodd), fact(4 * xodd + 1), fact(4 * xodd + 2), fact(4 * xodd + 3)};
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int az = k >> 1, ay = 4 * (k & 1) + ya;
            const float fyz = fact(ay) * fact(az);
            float v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = acc[k][e] / (fx[e] * fyz);
            if (bp.gemm) {
                *reinterpret_cast<float4 *>(f.A + (int64_t)c.w * 512 + (k * 8 + sub) * 4) =
                    make_float4(v[0], v[1], v[2], v[3]);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) f.A[grid_index<P>(f, 0, kx, ky, kz, 4 * xodd + e, ay, az)] = v[e];
            }
        }
    } else {
        if (sub >= P) return;
        const float fz = fact(sub);
#pragma unroll
        for (int ay = 0; ay < P; ++ay)
#pragma unroll
            for (int ax = 0; ax < P; ++ax)
                f.A[grid_index<P>(f, bp.gemm, kx, ky, kz, ax, ay, sub)] = acc[ay][ax] / (fact(ax) * fact(ay) * fz);
    }
}

// P2M over the cell list: large cells one per wavefront, then small cells eight per
// wavefront (four wavefronts per block, each on its own cells).
template <int P>
__global__ void __launch_bounds__(256) k_bp2m(FgtBatchPlan bp) {
    __shared__ float4 stage[4][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * 4 + wave, nw = (int64_t)gridDim.x * 4;
    const int64_t nsmall = bp.ncells[0], nbig = bp.ncells[1];
    for (int64_t r = wid; r < nbig; r += nw) {
        const int4 c = bp.cells[bp.cap - 1 - r];
        const FgtPop &f = bp.pops[c.x];
        if (lane == 0 && c.y == 0) atomicMin(&bp.stamps[2 * f.pop], (unsigned long long)wall_clock64());
        int kx, ky, kz;
        cell_coords(f, c.w, kx, ky, kz);
        p2m_cell_wave<P>(f.ps, f.perm, f.w, f.G[0], f.G[1], f.lo, f.cell, f.inv_sigma, f.A, bp.gemm, kx, ky, kz,
                         c.y, (int64_t)c.y + c.z, stage[wave]);
        wave_sync();
    }
    if constexpr (P <= 8) {
        for (int64_t r0 = wid * 8; r0 < nsmall; r0 += nw * 8) p2m_cells_group<P>(bp, r0, nsmall, stage[wave]);
    }
}

__global__ void __launch_bounds__(64) k_bm2l(FgtBatchPlan bp, int pass) {
    const int64_t g = blockIdx.x;
    const int k = find_pop(bp.tile_off[pass], bp.npop, g);
    const FgtPop &f = bp.pops[k];
    const int p = bp.p;
    const int64_t Ux = (int64_t)f.G[0] * p, Uy = (int64_t)f.G[1] * p, Uz = (int64_t)f.G[2] * p;
    const float *In = pass == 0 ? f.A : (pass == 1 ? f.B : f.Tmp);
    float *Out = pass == 1 ? f.Tmp : f.B;
    const int64_t R = pass == 0 ? Uz * Uy : (pass == 1 ? Ux * Uz : Uy * Ux);
    const int G = f.G[pass];
    const float *T = pass == 0 ? f.opsx : (pass == 1 ? f.opsy : f.opsz);
    const int64_t nr = (R + MT - 1) / MT;
    const int64_t t = g - bp.tile_off[pass][k];
    m2l_tile_mfma(In, Out, R, p, G, T, (t % nr) * MT, (int)(t / nr) * MT);
}

// x pass from the cell-major moments, z pass into the cell-major Taylor grid
template <int PASS>
__global__ void __launch_bounds__(256) k_bm2l_gemm(FgtBatchPlan bp) {
    extern __shared__ float sm[];
    const int64_t g = blockIdx.x;
    const int k = find_pop(bp.tile_off[PASS], bp.npop, g);
    const FgtPop &f = bp.pops[k];
    const int p = bp.p;
    const int64_t Ux = (int64_t)f.G[0] * p, Uy = (int64_t)f.G[1] * p, Uz = (int64_t)f.G[2] * p;
    const int64_t r0 = (g - bp.tile_off[PASS][k]) * 32;
    if (p == 8 && bp.split) {
        if constexpr (PASS == 0)
            m2l_gemm_tile<32, 1, 8, true>(f.A, f.B, Uz * Uy, p, f.G[0], f.opsx, r0, sm, f.G[1], f.band[0]);
        else if constexpr (PASS == 1)
            m2l_gemm_tile<32, 0, 8, true>(f.B, f.Tmp, Ux * Uz, p, f.G[1], f.opsy, r0, sm, 0, f.band[1]);
        else
            m2l_gemm_tile<32, 2, 8, true>(f.Tmp, f.B, Uy * Ux, p, f.G[2], f.opsz, r0, sm, f.G[0], f.band[2]);
    } else if (p == 8) {
        if constexpr (PASS == 0)
            m2l_gemm_tile<32, 1, 8>(f.A, f.B, Uz * Uy, p, f.G[0], f.opsx, r0, sm, f.G[1], f.band[0]);
        else if constexpr (PASS == 1)
            m2l_gemm_tile<32, 0, 8>(f.B, f.Tmp, Ux * Uz, p, f.G[1], f.opsy, r0, sm, 0, f.band[1]);
        else
            m2l_gemm_tile<32, 2, 8>(f.Tmp, f.B, Uy * Ux, p, f.G[2], f.opsz, r0, sm, f.G[0], f.band[2]);
    } else {
        if constexpr (PASS == 0)
            m2l_gemm_tile<32, 1>(f.A, f.B, Uz * Uy, p, f.G[0], f.opsx, r0, sm, f.G[1], f.band[0]);
        else if constexpr (PASS == 1)
            m2l_gemm_tile<32, 0>(f.B, f.Tmp, Ux * Uz, p, f.G[1], f.opsy, r0, sm, 0, f.band[1]);
        else
            m2l_gemm_tile<32, 2>(f.Tmp, f.B, Uy * Ux, p, f.G[2], f.opsz, r0, sm, f.G[0], f.band[2]);
    }
}

// Taylor series of cell (kx, ky, kz) at its points [s0, e) by one wavefront (grid
// cell-major when cm is set, else interleaved).  The cell's p^3 coefficients are
// staged in LDS (az slices padded by 4 floats so that
// the slices a lane group reads fall in different banks).  A pass takes up to 64
// targets; when it has fewer, L = 64 / (targets rounded up to a power of 2) lanes
// (at most the largest power of 2 <= P) share one target: lane `sub` evaluates the
// az slices sub, sub + L, ... (Horner in x, then y, then in z^L over its slices),
// scales by z^sub, and the L partial values are added by butterfly shuffles.
template <int P>
__device__ void l2p_cell_wave(const FgtPop &f, int cm, int kx, int ky, int kz, int64_t s0, int64_t e, float *sC) {
    constexpr int SZ = P * P + 4;
    constexpr int LMAX = P >= 16 ? 16 : (P >= 8 ? 8 : (P >= 4 ? 4 : (P >= 2 ? 2 : 1)));
    const int lane = threadIdx.x & 63;
    const int64_t Rx = (int64_t)f.G[0] * P, Ry = (int64_t)f.G[1] * P;
    const int64_t cbase = (((int64_t)kz * f.G[1] + ky) * f.G[0] + kx) * (P * P * P);
    for (int q = lane; q < P * P * P; q += 64) {
        const int ax = q % P, ay = (q / P) % P, az = q / (P * P);
        sC[az * SZ + ay * P + ax] = cm ? f.B[cbase + q]
                                       : f.B[(((int64_t)kz * P + az) * Ry + (int64_t)ky * P + ay) * Rx + (int64_t)kx * P + ax];
    }
    wave_sync();
    const double cx = f.lo[0] + (kx + 0.5) * f.cell, cy = f.lo[1] + (ky + 0.5) * f.cell,
                 cz = f.lo[2] + (kz + 0.5) * f.cell;
    for (int64_t c0 = s0; c0 < e; ) {
        const int64_t left = e - c0;
        int tp = 1;
        while (tp < left && tp < 64) tp <<= 1;
        const int L = 64 / tp < LMAX ? 64 / tp : LMAX;
        const int slots = 64 / L;
        const int a = lane / L, sub = lane % L;
        const int64_t i = c0 + a;
        const bool live = a < left;
        const float4 q = live ? f.ps[i] : make_float4(0.f, 0.f, 0.f, 0.f);
        const int32_t j = live ? f.perm[i] : 0;
        const bool tgt = live && (!f.is_target || f.is_target[j]);
        const float wself = (live && f.subtract_self) ? f.w[j] : 0.f;
        const float X = ((q.x - (float)cx) * (float)f.inv_sigma);
        const float Y = ((q.y - (float)cy) * (float)f.inv_sigma);
        const float Z = ((q.z - (float)cz) * (float)f.inv_sigma);
        float zl = 1.f, zs = 1.f;
        for (int k = 0; k < L; ++k) {
            if (k == sub) zs = zl;
            zl *= Z;
        }
        int top = sub;
        while (top + L < P) top += L;
        float uz = 0.f;
        for (int az = top; az >= 0; az -= L) {
            const float *cz_ = sC + az * SZ;
            float uy = 0.f;
#pragma unroll
            for (int ay = P - 1; ay >= 0; --ay) {
                const float *c = cz_ + ay * P;
                float ux = c[P - 1];
#pragma unroll
                for (int ax = P - 2; ax >= 0; --ax) ux = fmaf(ux, X, c[ax]);
                uy = fmaf(uy, Y, ux);
            }
            uz = fmaf(uz, zl, uy);
        }
        float u = uz * zs;
        for (int o = 1; o < L; o <<= 1) u += __shfl_xor(u, o, 64);
        if (live && sub == 0) f.u_out[j] = tgt ? u - wself : 0.f;
        c0 += slots;
    }
}

// Small cells, eight per wavefront: lane group grp = lane / 8 takes cell r0 + grp;
// its eight lanes hold shares of the cell's Taylor coefficients in registers (the
// same shares as the grouped P2M: for p = 8 the 16-byte chunks k * 8 + sub, read
// one 128-byte line per group and load; otherwise slice az = sub), each evaluates
// its share at every target of the cell (Horner in x within a chunk, then over az
// in z), and the eight values are added by butterfly shuffles.  Targets pass
// through LDS eight per group at a time; the lane that loaded a target also holds
// its output index, flag and self weight and writes its value.  P <= 8.
template <int P>
__device__ void l2p_cells_group(const FgtBatchPlan &bp, int64_t r0, int64_t nsmall, float4 *stage) {
    const int lane = threadIdx.x & 63, grp = lane >> 3, sub = lane & 7;
    const int64_t r = r0 + grp;
    const bool has = r < nsmall;
    const int4 c = has ? bp.cells[r] : make_int4(0, 0, 0, 0);
    const FgtPop &f = bp.pops[c.x];
    int kx = 0, ky = 0, kz = 0;
    if (has) cell_coords(f, c.w, kx, ky, kz);
    constexpr bool CH = P == 8;
    constexpr int NA = CH ? 16 : P, NB = CH ? 4 : P;
    const int ya = sub >> 1, xodd = sub & 1;
    float cf[NA][NB];
    if constexpr (CH) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (has && bp.gemm) {
                v = *reinterpret_cast<const float4 *>(f.B + (int64_t)c.w * 512 + (k * 8 + sub) * 4);
            } else if (has) {
                const int az = k >> 1, ay = 4 * (k & 1) + ya;
                v = make_float4(f.B[grid_index<P>(f, 0, kx, ky, kz, 4 * xodd, ay, az)],
                                f.B[grid_index<P>(f, 0, kx, ky, kz, 4 * xodd + 1, ay, az)],
                                f.B[grid_index<P>(f, 0, kx, ky, kz, 4 * xodd + 2, ay, az)],
                                f.B[grid_index<P>(f, 0, kx, ky, kz, 4 * xodd + 3, ay, az)]);
            }
            cf[k][0] = v.x;
            cf[k][1] = v.y;
            cf[k][2] = v.z;
            cf[k][3] = v.w;
        }
    } else {
#pragma unroll
        for (int ay = 0; ay < P; ++ay)
#pragma unroll
            for (int ax = 0; ax < P; ++ax)
                cf[ay][ax] = (has && sub < P) ? f.B[grid_index<P>(f, bp.gemm, kx, ky, kz, ax, ay, sub)] : 0.f;
    }
    const double cx = f.lo[0] + (kx + 0.5) * f.cell, cy = f.lo[1] + (ky + 0.5) * f.cell,
                 cz = f.lo[2] + (kz + 0.5) * f.cell;
    const int cnt = has ? c.z : 0;
    int mx = cnt;
    for (int o = 8; o < 64; o <<= 1) {
        const int t = __shfl_xor(mx, o, 64);
        mx = t > mx ? t : mx;
    }
    // this lane's target of a chunk: position (in sigma, from the centre), output
    // index (-1: none), flag and self weight
    struct Tgt {
        float4 q;
        int32_t j;
        bool t;
        float ws;
    };
    auto fetch = [&](int c0) {
        Tgt g{make_float4(0.f, 0.f, 0.f, 0.f), -1, false, 0.f};
        const int jj = c0 + sub;
        if (jj < cnt) {
            const float4 t = f.ps[c.y + jj];
            g.q = make_float4(((t.x - (float)cx) * (float)f.inv_sigma), ((t.y - (float)cy) * (float)f.inv_sigma),
                              ((t.z - (float)cz) * (float)f.inv_sigma), 0.f);
            g.j = f.perm[c.y + jj];
            g.t = !f.is_target || f.is_target[g.j];
            g.ws = f.subtract_self ? f.w[g.j] : 0.f;
        }
        return g;
    };
    Tgt cur, nxt = fetch(0);
    for (int c0 = 0; c0 < mx; c0 += 8) {
        cur = nxt;
        wave_sync();
        stage[lane] = cur.q;
        wave_sync();
        if (c0 + 8 < mx) nxt = fetch(c0 + 8);
#pragma unroll 2
        for (int t = 0; t < 8; ++t) {
            const float4 q = stage[grp * 8 + t];
            float v;
            if constexpr (CH) {
                const float x2 = q.x * q.x, y2 = q.y * q.y;
                const float y4 = y2 * y2;
                float s = 0.f;
#pragma unroll
                for (int az = 7; az >= 0; --az) {
                    const float *c0p = cf[2 * az], *c1p = cf[2 * az + 1];
                    const float h0 = fmaf(fmaf(fmaf(c0p[3], q.x, c0p[2]), q.x, c0p[1]), q.x, c0p[0]);
                    const float h1 = fmaf(fmaf(fmaf(c1p[3], q.x, c1p[2]), q.x, c1p[1]), q.x, c1p[0]);
                    s = fmaf(s, q.z, fmaf(y4, h1, h0));
                }
                float hy = 1.f;
                for (int k = 0; k < ya; ++k) hy *= q.y;
                v = s * hy * (xodd ? x2 * x2 : 1.f);
            } else {
                float uy = 0.f;
#pragma unroll
                for (int ay = P - 1; ay >= 0; --ay) {
                    float ux = cf[ay][P - 1];
#pragma unroll
                    for (int ax = P - 2; ax >= 0; --ax) ux = fmaf(ux, q.x, cf[ay][ax]);
                    uy = fmaf(uy, q.y, ux);
                }
                float zs = 1.f;
                for (int k = 0; k < sub; ++k) zs *= q.z;
                v = uy * zs;
            }
            v += __shfl_xor(v, 1, 64);
            v += __shfl_xor(v, 2, 64);
            v += __shfl_xor(v, 4, 64);
            if (sub == t && cur.j >= 0) f.u_out[cur.j] = cur.t ? v - cur.ws : 0.f;
        }
    }
    // end stamp once per run of consecutive groups of one population
    const int prev_pop = __shfl(has ? f.pop : -1, lane - 8 < 0 ? lane : lane - 8, 64);
    if (has && sub == 0 && (grp == 0 || prev_pop != f.pop))
        atomicMax(&bp.stamps[2 * f.pop + 1], (unsigned long long)wall_clock64());
}

// L2P over the cell list: large cells one per wavefront, then small cells eight per
// wavefront (four wavefronts per block, each on its own cells).
template <int P>
__global__ void __launch_bounds__(256) k_bl2p(FgtBatchPlan bp) {
    constexpr int SC = P * (P * P + 4) > 256 ? P * (P * P + 4) : 256;   // slice buffer, or 64 float4
    __shared__ __align__(16) float sC[4][SC];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * 4 + wave, nw = (int64_t)gridDim.x * 4;
    const int64_t nsmall = bp.ncells[0], nbig = bp.ncells[1];
    for (int64_t r = wid; r < nbig; r += nw) {
        const int4 c = bp.cells[bp.cap - 1 - r];
        const FgtPop &f = bp.pops[c.x];
        int kx, ky, kz;
        cell_coords(f, c.w, kx, ky, kz);
        l2p_cell_wave<P>(f, bp.gemm, kx, ky, kz, c.y, (int64_t)c.y + c.z, sC[wave]);
        wave_sync();
        if (lane == 0) atomicMax(&bp.stamps[2 * f.pop + 1], (unsigned long long)wall_clock64());
    }
    if constexpr (P <= 8) {
        float4 *stage = reinterpret_cast<float4 *>(sC[wave]);
        for (int64_t r0 = wid * 8; r0 < nsmall; r0 += nw * 8) l2p_cells_group<P>(bp, r0, nsmall, stage);
    }
}

// L2P with derivatives over the cell list (one wavefront per cell): value,
// gradient and (want_lap) Laplacian at every point of the cell, into the
// population's records f.rec + i * stride + slot (key order i).
template <int P>
__global__ void __launch_bounds__(64) k_bl2p_grad(FgtBatchPlan bp, int stride, int slot, int want_lap) {
    constexpr int P3 = P * P * P;
    __shared__ float sC[P3];
    const int lane = threadIdx.x;
    const int64_t nsmall = bp.ncells[0], nbig = bp.ncells[1];
    for (int64_t r = blockIdx.x; r < nsmall + nbig; r += gridDim.x) {
        const int4 c = r < nbig ? bp.cells[bp.cap - 1 - r] : bp.cells[r - nbig];
        const FgtPop &f = bp.pops[c.x];
        int kx, ky, kz;
        cell_coords(f, c.w, kx, ky, kz);
        wave_sync();   // the previous cell's coefficients are no longer read
        for (int q = lane; q < P3; q += 64) {
            const int ax = q % P, ay = (q / P) % P, az = q / (P * P);
            sC[q] = f.B[grid_index<P>(f, bp.gemm, kx, ky, kz, ax, ay, az)];
        }
        wave_sync();
        const double cx = f.lo[0] + (kx + 0.5) * f.cell, cy = f.lo[1] + (ky + 0.5) * f.cell,
                     cz = f.lo[2] + (kz + 0.5) * f.cell;
        const float is = (float)f.inv_sigma;
        for (int64_t i = (int64_t)c.y + lane; i < (int64_t)c.y + c.z; i += 64) {
            const float4 q = f.ps[i];
            const float X = ((q.x - (float)cx) * (float)f.inv_sigma);
            const float Y = ((q.y - (float)cy) * (float)f.inv_sigma);
            const float Z = ((q.z - (float)cz) * (float)f.inv_sigma);
            l2p_grad_point<P>(sC, X, Y, Z, is, want_lap, f.rec + i * stride + slot);
        }
    }
}

template <int P>
int batch_p2m_l2p(const FgtBatchPlan &bp, bool l2p, hipStream_t s) {
    const unsigned grid = (unsigned)(bp.cus * 8);
    if (!l2p) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_bp2m<P>), dim3(grid), dim3(256), 0, s, bp);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_bl2p<P>), dim3(grid), dim3(256), 0, s, bp);
    MSP_CHECK_LAUNCH();
    return MSP_OK;
}

int batch_p2m_l2p_p(const FgtBatchPlan &bp, bool l2p, hipStream_t s) {
    switch (bp.p) {
#define CASE(P) case P: return batch_p2m_l2p<P>(bp, l2p, s);
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
        CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16)
#undef CASE
    }
    return fail(MSP_EINVAL, "p out of range");
}

}  // namespace

namespace {
// operator tables, cleared grids, the cell list, P2M and the three M2L passes
int fgt_batch_expand(const FgtBatchPlan &bp, hipStream_t s) {
    hipLaunchKernelGGL(k_bops, dim3(grid_for(bp.n_ops, 64)), dim3(64), 0, s, bp);
    MSP_CHECK_LAUNCH();
    const int64_t fill_threads = bp.n_grid / 4 < (int64_t)bp.cus * 2048 ? bp.n_grid / 4 + 1 : (int64_t)bp.cus * 2048;
    hipLaunchKernelGGL(k_bclear, dim3(grid_for(fill_threads > bp.npop ? fill_threads : bp.npop, kBlock)),
                       dim3(kBlock), 0, s, bp);
    MSP_CHECK_LAUNCH();
    const int64_t cell_waves = (bp.n_pw + kCellWin - 1) / kCellWin;
    hipLaunchKernelGGL(k_bcells, dim3((unsigned)((cell_waves + 3) / 4)), dim3(256), 0, s, bp,
                       bp.p <= 8 ? kSmallCell : 0);
    MSP_CHECK_LAUNCH();
    MSP_TRY(batch_p2m_l2p_p(bp, false, s));
    for (int pass = 0; pass < 3; ++pass) {
        if (bp.n_tiles[pass] == 0) continue;
        if (bp.gemm) {
            const dim3 grid((unsigned)bp.n_tiles[pass]);
            if (pass == 0) hipLaunchKernelGGL(k_bm2l_gemm<0>, grid, dim3(256), bp.gemm_lds, s, bp);
            else if (pass == 1) hipLaunchKernelGGL(k_bm2l_gemm<1>, grid, dim3(256), bp.gemm_lds, s, bp);
            else hipLaunchKernelGGL(k_bm2l_gemm<2>, grid, dim3(256), bp.gemm_lds, s, bp);
        } else
            hipLaunchKernelGGL(k_bm2l, dim3((unsigned)bp.n_tiles[pass]), dim3(64), 0, s, bp, pass);
        MSP_CHECK_LAUNCH();
    }
    return MSP_OK;
}

template <int P>
int launch_bl2p_grad(const FgtBatchPlan &bp, int stride, int slot, int want_lap, hipStream_t s) {
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_bl2p_grad<P>), dim3((unsigned)(bp.cus * 16)), dim3(64), 0, s, bp,
                       stride, slot, want_lap);
    MSP_CHECK_LAUNCH();
    return MSP_OK;
}
}  // namespace

int fgt_batch_forward(const FgtBatchPlan &bp, hipStream_t s) {
    if (bp.npop == 0) return MSP_OK;
    MSP_TRY(fgt_batch_expand(bp, s));
    return batch_p2m_l2p_p(bp, true, s);
}

int fgt_batch_field_grad(const FgtBatchPlan &bp, int stride, int slot, int want_lap, hipStream_t s) {
    if (bp.npop == 0) return MSP_OK;
    MSP_TRY(fgt_batch_expand(bp, s));
    switch (bp.p) {
#define CASE(P) case P: return launch_bl2p_grad<P>(bp, stride, slot, want_lap, s);
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
        CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16)
#undef CASE
    }
    return fail(MSP_EINVAL, "p out of range");
}

void fgt_grid_bytes(const FgtPlan &pl, size_t *grid, size_t *ops) {
    const size_t p = (size_t)pl.p;
    const size_t ncell = (size_t)pl.G[0] * pl.G[1] * pl.G[2];
    *grid = ncell * p * p * p * 4;
    // a third grid, then the per-axis operator tables
    *ops = *grid + (size_t)(2 * (pl.G[0] + pl.G[1] + pl.G[2])) * p * p * 4;
}

int fgt_pop_prepare(msp_tree *t, const FgtPlan &pl, const msp_fgt_params *prm, FgtPop *f) {
    const int p = pl.p;
    const int64_t ncell = (int64_t)pl.G[0] * pl.G[1] * pl.G[2];
    size_t gbytes = 0, obytes = 0;
    fgt_grid_bytes(pl, &gbytes, &obytes);
    MSP_TRY(t->gridA.ensure(gbytes));
    MSP_TRY(t->gridB.ensure(gbytes));
    MSP_TRY(t->ops.ensure(obytes));
    t->ops_valid = false;   // the batched pass writes the tables itself
    t->grid_bytes_valid = (int64_t)gbytes;
    f->keys = t->keys.as<uint64_t>();
    f->ps = t->ps.as<float4>();
    f->perm = t->perm.as<int32_t>();
    f->n = t->n;
    f->nlevel = t->nlevel.as<int32_t>();
    f->nfirst = t->nfirst.as<int32_t>();
    f->ncount = t->ncount.as<int32_t>();
    f->nnchild = t->nnchild.as<int32_t>();
    f->n_nodes = t->n_nodes;
    f->subtract_self = (prm->flags & MSP_EXCLUDE_SELF) ? 1 : 0;
    f->rec = nullptr;
    f->A = t->gridA.as<float>();
    f->B = t->gridB.as<float>();
    f->Tmp = t->ops.as<float>();
    f->opsx = f->Tmp + (size_t)ncell * p * p * p;
    f->opsy = f->opsx + (size_t)(2 * pl.G[0] - 1) * p * p;
    f->opsz = f->opsy + (size_t)(2 * pl.G[1] - 1) * p * p;
    f->level = pl.level;
    for (int k = 0; k < 3; ++k) {
        f->G[k] = pl.G[k];
        f->lo[k] = t->geo.lo[k];
    }
    f->cell = pl.cell;
    f->inv_sigma = 1.0 / prm->sigma;
    f->step = pl.cell / prm->sigma;
    for (int k = 0; k < 3; ++k) f->band[k] = m2l_band(p, f->step, pl.G[k]);
    return MSP_OK;
}

int64_t fgt_pop_tiles(const FgtPop &f, int p, int pass, bool gemm) {
    const int64_t U[3] = {(int64_t)f.G[0] * p, (int64_t)f.G[1] * p, (int64_t)f.G[2] * p};
    const int64_t R = pass == 0 ? U[2] * U[1] : (pass == 1 ? U[0] * U[2] : U[1] * U[0]);
    if (gemm) return (R + 31) / 32;
    return ((R + MT - 1) / MT) * ((U[pass] + MT - 1) / MT);
}

size_t fgt_pop_gemm_lds(const FgtPop &f, int p, bool split) {
    size_t m = 0;
    for (int k = 0; k < 3; ++k) {
        const size_t l = split ? m2l_gemm_lds_split(f.G[k] * p, f.G[k], 32) : m2l_gemm_lds(f.G[k] * p, f.G[k], p, 32);
        m = l > m ? l : m;
    }
    return m;
}

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
    // two-level variant (on request): cells must hold many points for the shorter
    // sub-cell series to pay for the shifts; p 6..8 (LDS budget of the fused kernels)
    pl->pf = 0;
    if ((prm->flags & MSP_TWO_LEVEL) && p >= 6 && p <= 8 && level + 2 <= kDepth) {
        const int pf = fine_terms(p, pl->rho * 0.25);
        const double per_cell = n / (ncell > 0 ? ncell : 1.0);
        if (pf >= 3 && pf <= 5 && pf <= p - 2 && per_cell >= 512.0 && two_level_lds(p, pf) <= 60 * 1024)
            pl->pf = pf;
    }
    return MSP_OK;
}

int stage_inputs(msp_tree *t, const float *w, const uint8_t *is_target, hipStream_t s) {
    const int64_t n = t->n, nb = n > 0 ? n : 1;
    MSP_TRY(t->tflag.ensure(nb));
    MSP_TRY(t->usort.ensure(nb * 4));
    if (n == 0) return MSP_OK;
    ++t->ps_gen;
    PhaseScope ps(&t->timing, PH_STAGE, s);
    hipLaunchKernelGGL(k_stage, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, w, is_target,
                       t->perm.as<int32_t>(), n, t->ps.as<float4>(), t->tflag.as<uint8_t>());
    MSP_CHECK_LAUNCH();
    return MSP_OK;
}

int fgt_forward_grid(msp_tree *t, const FgtPlan &pl, const msp_fgt_params *prm, const float *w,
                     const uint8_t *is_target, float *u_out, hipStream_t s) {
    const bool staged = (prm->flags & MSP_WEIGHTS_STAGED) != 0;
    const GridArgs ga{w, staged ? nullptr : w, is_target, (prm->flags & MSP_EXCLUDE_SELF) ? 1 : 0, u_out,
                      !staged && (prm->flags & MSP_STAGE_WEIGHTS) != 0};
    if (ga.stage) ++t->ps_gen;   // its P2M rewrites the weights of the records
    const int p = pl.p;
    const int64_t ncell = (int64_t)pl.G[0] * pl.G[1] * pl.G[2];
    size_t gbytes = 0, obytes = 0;
    fgt_grid_bytes(pl, &gbytes, &obytes);
    MSP_TRY(t->gridA.ensure(gbytes));
    MSP_TRY(t->gridB.ensure(gbytes));
    const size_t ops_bytes_before = t->ops.bytes;
    MSP_TRY(t->ops.ensure(obytes));
    if (t->ops.bytes != ops_bytes_before) t->ops_valid = false;   // reallocated
    t->grid_bytes_valid = (int64_t)gbytes;
    if (t->n == 0) return MSP_OK;
    float *A = t->gridA.as<float>();
    float *B = t->gridB.as<float>();
    float *Tmp = t->ops.as<float>();                     // second intermediate grid
    float *opsx = Tmp + (size_t)ncell * p * p * p;
    float *opsy = opsx + (size_t)(2 * pl.G[0] - 1) * p * p;
    float *opsz = opsy + (size_t)(2 * pl.G[1] - 1) * p * p;
    const double step = pl.cell / prm->sigma;
    // the operator tables depend on (p, grid, cell / sigma) only: kept from the last
    // call when those are unchanged
    uint64_t sig[5] = {(uint64_t)p, (uint64_t)pl.G[0], (uint64_t)pl.G[1], (uint64_t)pl.G[2], 0};
    std::memcpy(&sig[4], &step, sizeof(double));
    if (!t->ops_valid || !std::equal(sig, sig + 5, t->ops_sig)) {
        PhaseScope ps(&t->timing, PH_OPS, s);
        const int nops = 2 * (pl.G[0] + pl.G[1] + pl.G[2]) - 3;
        hipLaunchKernelGGL(k_m2l_ops, dim3(grid_for(nops, 64)), dim3(64), 0, s, p, pl.G[0], pl.G[1],
                           pl.G[2], step, opsx, opsy, opsz);
        MSP_CHECK_LAUNCH();
        std::copy(sig, sig + 5, t->ops_sig);
        t->ops_valid = true;
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
    const bool bf16x3 = (prm->flags & MSP_M2L_BF16X3) != 0;
    for (int k = 0; k < 3; ++k) {
        const Pass &ps = passes[k];
        PhaseScope sc(&t->timing, PH_M2L_X + k, s);
        if (valu) {
            dim3 grid((unsigned)((ps.R + TR - 1) / TR), (unsigned)((ps.U + TV - 1) / TV));
            hipLaunchKernelGGL(k_m2l_pass, grid, dim3(kBlock), 0, s, ps.in, ps.out, ps.R, p, ps.G, ps.T);
        } else if (bf16x3) {
            // rows per block: enough blocks to fill the chip, at most 64, and fewer
            // when the tile would not fit in LDS
            int RT = 64;
            while (RT > 16 && ((ps.R + RT - 1) / RT < 1024 || m2l_gemm_lds_split((int)ps.U, ps.G, RT) > 64 * 1024))
                RT >>= 1;
            const size_t lds = m2l_gemm_lds_split((int)ps.U, ps.G, RT);
            if (p == 8 && lds <= 64 * 1024) {
                const dim3 grid((unsigned)((ps.R + RT - 1) / RT));
                const int band = m2l_band(p, step, ps.G);
                if (RT == 64)
                    hipLaunchKernelGGL(k_m2l_gemm_bf16x3<64>, grid, dim3(256), lds, s, ps.in, ps.out, ps.R, ps.G, ps.T, band);
                else if (RT == 32)
                    hipLaunchKernelGGL(k_m2l_gemm_bf16x3<32>, grid, dim3(256), lds, s, ps.in, ps.out, ps.R, ps.G, ps.T, band);
                else
                    hipLaunchKernelGGL(k_m2l_gemm_bf16x3<16>, grid, dim3(256), lds, s, ps.in, ps.out, ps.R, ps.G, ps.T, band);
            } else {
                dim3 grid((unsigned)((ps.R + MT - 1) / MT), (unsigned)((ps.U + MT - 1) / MT));
                hipLaunchKernelGGL(k_m2l_pass_bf16x3, grid, dim3(64), 0, s, ps.in, ps.out, ps.R, p, ps.G, ps.T);
            }
        } else {
            // rows per block: enough blocks to fill the chip, at most 64, and fewer
            // when the tile would not fit in LDS
            int RT = 64;
            while (RT > 16 && ((ps.R + RT - 1) / RT < 1024 || m2l_gemm_lds((int)ps.U, ps.G, p, RT) > 64 * 1024))
                RT >>= 1;
            const size_t lds = m2l_gemm_lds((int)ps.U, ps.G, p, RT);
            if (lds <= 64 * 1024) {
                // column groups of four 16-wide blocks, one per wavefront, as the grid's y,
                // only while the row tiles alone make fewer than 1024 blocks (every group
                // stages the whole input rows)
                const int64_t rows = (ps.R + RT - 1) / RT;
                const int ngroup = ((int)(ps.U + 15) / 16 + 3) / 4;
                const int64_t want = (1024 + rows - 1) / rows;
                const int cg = want < ngroup ? (int)want : ngroup;
                const dim3 grid((unsigned)rows, (unsigned)cg);
                const int band = m2l_band(p, step, ps.G);
                if (RT == 64)
                    hipLaunchKernelGGL(k_m2l_gemm<64>, grid, dim3(256), lds, s, ps.in, ps.out, ps.R, p, ps.G, ps.T, band);
                else if (RT == 32)
                    hipLaunchKernelGGL(k_m2l_gemm<32>, grid, dim3(256), lds, s, ps.in, ps.out, ps.R, p, ps.G, ps.T, band);
                else
                    hipLaunchKernelGGL(k_m2l_gemm<16>, grid, dim3(256), lds, s, ps.in, ps.out, ps.R, p, ps.G, ps.T, band);
            } else {
                dim3 grid((unsigned)((ps.R + MT - 1) / MT), (unsigned)((ps.U + MT - 1) / MT));
                hipLaunchKernelGGL(k_m2l_pass_mfma, grid, dim3(64), 0, s, ps.in, ps.out, ps.R, p, ps.G, ps.T);
            }
        }
        MSP_CHECK_LAUNCH();
    }
    if (!u_out) return MSP_OK;   // callers that evaluate the Taylor grid themselves
    {
        PhaseScope ps(&t->timing, PH_L2P, s);
        MSP_TRY(dispatch_p2m_l2p(t, pl, inv_sigma, true, B, nullptr, ga, s));
    }
    // the single-level L2P writes every point's sum: target flags and self term in
    // input order afterwards (the two-level L2P applies them itself)
    if (pl.pf == 0 && (ga.is_target || ga.subtract_self)) {
        PhaseScope ps(&t->timing, PH_SCATTER, s);
        const bool vec = (uintptr_t)ga.u_out % 16 == 0 && (!ga.subtract_self || (uintptr_t)ga.w % 16 == 0) &&
                         (!ga.is_target || (uintptr_t)ga.is_target % 4 == 0);
        if (vec)
            hipLaunchKernelGGL(k_finish_u4, dim3(grid_for((t->n + 3) / 4, kBlock)), dim3(kBlock), 0, s, t->n,
                               ga.is_target, ga.w, ga.subtract_self, ga.u_out);
        else
            hipLaunchKernelGGL(k_finish_u, dim3(grid_for(t->n, kBlock)), dim3(kBlock), 0, s, t->n, ga.is_target,
                               ga.w, ga.subtract_self, ga.u_out);
        MSP_CHECK_LAUNCH();
    }
    return MSP_OK;
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
