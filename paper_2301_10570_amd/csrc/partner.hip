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
#include <type_traits>

namespace msp {

double rho_max_for_p(int p);

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kBlock = 256;
constexpr int kC1 = 70;                    // Algorithm 2's element threshold
constexpr int kLaneLeaf = 128;               // leaves up to this size are summed by one lane
constexpr int kSmallNode = 512;              // nodes up to this size: eight lanes per query sum them
constexpr int kDirectPoints = 16384;         // nodes up to this size are summed directly (no walk)
constexpr double kAdmitTol = 1e-5;   // M2P error vs the node's own smallest contribution
constexpr double kRunTol = 1e-7;     // M2P error vs the running total of the query
constexpr double kSkipTol = 1e-12;   // dropped node's largest contribution vs the running total
// direct sums in float32 when every term of the node lies within exp(-kSpan32) of
// its largest possible one (float32 holds down to about exp(-87))
constexpr double kSpan32 = 60.0;
// work counters (when counting is on): queries and pairs of the eight-lane and the
// wavefront passes; queries, nodes visited, expansions, pairs and stack rounds of
// the walk
enum WorkSlot : int { W_DIRECT_Q = 0, W_DIRECT_PAIRS, W_WAVE_Q, W_WAVE_PAIRS, W_WALK_Q, W_WALK_NODES, W_WALK_M2P,
                      W_WALK_PAIRS, W_WALK_STEPS };

// Sources (staged weight != 0) below every node, from an exclusive prefix count
// S over the points in key order: nsrc(v) = S[first + count] - S[first].
// Tiles of kSrcTile points, point k * 256 + t of a tile to thread t.
constexpr int kSrcItems = 16;
constexpr int kSrcTile = 256 * kSrcItems;

__device__ inline int32_t block_sum_256(int32_t v, int32_t *lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    return lds[0] + lds[1] + lds[2] + lds[3];
}

__global__ void __launch_bounds__(256) k_src_tiles(int64_t n, const float4 *ps, int32_t *tile_sum) {
    __shared__ int32_t lds[4];
    const int64_t base = (int64_t)blockIdx.x * kSrcTile;
    int32_t c = 0;
#pragma unroll
    for (int k = 0; k < kSrcItems; ++k) {
        const int64_t i = base + k * 256 + threadIdx.x;
        if (i < n) c += ps[i].w != 0.f ? 1 : 0;
    }
    const int32_t tot = block_sum_256(c, lds);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

// exclusive scan of the tile sums in place (one block, chunks of 1024)
__global__ void __launch_bounds__(1024) k_src_tile_scan(int64_t nt, int32_t *tile) {
    __shared__ int32_t part[1024];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nt; c0 += 1024) {
        const int64_t g = c0 + threadIdx.x;
        const int32_t v = g < nt ? tile[g] : 0;
        part[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int32_t t = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0;
            __syncthreads();
            part[threadIdx.x] += t;
            __syncthreads();
        }
        if (g < nt) tile[g] = carry + part[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 0) carry += part[1023];
        __syncthreads();
    }
}

// S[i] for the points of one tile (S[n] = total from the tile holding point n - 1)
__global__ void __launch_bounds__(256) k_src_prefix(int64_t n, const float4 *ps, const int32_t *tile_off,
                                                    int32_t *S) {
    __shared__ int32_t wsum[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * kSrcTile;
    int32_t run = tile_off[blockIdx.x];
    const uint64_t below = (1ull << lane) - 1ull;
    for (int k = 0; k < kSrcItems; ++k) {
        const int64_t i = base + k * 256 + threadIdx.x;
        const bool f = i < n && ps[i].w != 0.f;
        const uint64_t m = __ballot(f);
        __syncthreads();
        if (lane == 0) wsum[wave] = (int32_t)__popcll(m);
        __syncthreads();
        int32_t before = run;
        for (int q = 0; q < wave; ++q) before += wsum[q];
        before += (int32_t)__popcll(m & below);
        if (i < n) S[i] = before;
        if (i == n - 1) S[n] = before + (f ? 1 : 0);
        run += wsum[0] + wsum[1] + wsum[2] + wsum[3];
    }
}

// sources per node; the moment flags start cleared (the moment kernels set those
// of the levels they visit)
__global__ void k_nsrc_nodes(int64_t nn, const int32_t *nfirst, const int32_t *ncount, const int32_t *S,
                             int32_t *nsrc, uint8_t *hasA) {
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= nn) return;
    const int32_t f = nfirst[v];
    nsrc[v] = S[f + ncount[v]] - S[f];
    hasA[v] = 0;
}

// Key-order position of each query's target: its Morton key (as the tree build
// computes it) is searched among the sorted keys, then the run of equal keys is
// scanned for the point itself.  -1 for an index out of range.
// tally (or NULL): per-level counters of the walk's order, cleared here for the
// k_order_place that follows on the stream
__global__ void k_query_pos(int64_t nq, const int32_t *target_idx, int64_t n, const float4 *pin,
                            const uint64_t *keys, const int32_t *perm, double lx, double ly, double lz,
                            double scale, int32_t *qpos, int32_t *tally) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (tally && q < kMaxLevels) tally[q] = 0;
    if (q >= nq) return;
    const int32_t t = target_idx[q];
    int32_t pos = -1;
    if (t >= 0 && t < n) {
        const float4 a = pin[t];
        const uint64_t key = morton3(quantise(a.x, lx, scale), quantise(a.y, ly, scale), quantise(a.z, lz, scale));
        for (int64_t p = lower_bound_u64(keys, 0, n, key); p < n && keys[p] == key; ++p)
            if (perm[p] == t) {
                pos = (int32_t)p;
                break;
            }
    }
    qpos[q] = pos;
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

// Rigorous bound, relative to the node's total weight, on the Hermite terms a
// p-term tensor expansion leaves out: with |A_a| <= W prod rho^a_k / a_k! (every
// source within rho sigma of the centre per axis) and Cramer's inequality
// |h_n(x)| <= K 2^(n/2) sqrt(n!) exp(-x^2/2), each term is at most
// W prod_k a(alpha_k) with a(n) = K (sqrt2 rho)^n / sqrt(n!), so the omitted
// part is at most W (F^3 - F_p^3), F = sum_n a(n), F_p = sum_{n<p} a(n).
__device__ inline double trunc_bound(double rho, int p) {
    const double K = 1.086435, x = 1.4142135623730951 * rho;
    double a = K, fp = 0.0, tail = 0.0;
    for (int k = 0; k < 400; ++k) {
        if (k < p) fp += a;
        else tail += a;
        a *= x / sqrt((double)(k + 1));
        if (k >= p && a < 1e-17 * (fp + tail)) break;
    }
    const double f = fp + tail;
    return tail * (f * f + f * fp + fp * fp);
}

// h_0..h_{P-1} at y: h_0 = exp(-y^2), h_{k+1} = 2y h_k - 2k h_{k-1}.
template <int P>
__device__ inline void hermite_row(float y, float (&h)[P]) {
    h[0] = expf(-y * y);
    if constexpr (P > 1) h[1] = 2.f * y * h[0];
#pragma unroll
    for (int k = 1; k + 1 < P; ++k) h[k + 1] = 2.f * y * h[k] - 2.f * (float)k * h[k - 1];
}

__device__ inline float hermite_at(float y, int k) {
    float h0 = expf(-y * y);
    if (k == 0) return h0;
    float h1 = 2.f * y * h0;
    for (int m = 1; m < k; ++m) {
        const float hn = 2.f * y * h1 - 2.f * (float)m * h0;
        h0 = h1;
        h1 = hn;
    }
    return h1;
}

// One row of Eq. (7): sum_ax A[ax] h_ax.
template <int P>
__device__ inline float m2p_row(const float *__restrict__ row, const float (&hx)[P]) {
    float sx = 0.f;
    if constexpr (P % 4 == 0) {
        const float4 *r4 = reinterpret_cast<const float4 *>(row);
#pragma unroll
        for (int k = 0; k < P / 4; ++k) {
            const float4 v = r4[k];
            sx = fmaf(v.x, hx[4 * k], sx);
            sx = fmaf(v.y, hx[4 * k + 1], sx);
            sx = fmaf(v.z, hx[4 * k + 2], sx);
            sx = fmaf(v.w, hx[4 * k + 3], sx);
        }
    } else {
#pragma unroll
        for (int ax = 0; ax < P; ++ax) sx = fmaf(row[ax], hx[ax], sx);
    }
    return sx;
}

// Eq. (7) evaluated at y = (t - c)/sigma by one lane: sum_a A_a h_ax h_ay h_az.
template <int P>
__device__ inline float m2p_lane(const float *__restrict__ A, float yx, float yy, float yz) {
    float hx[P], hy[P], hz[P];
    hermite_row<P>(yx, hx);
    hermite_row<P>(yy, hy);
    hermite_row<P>(yz, hz);
    float acc = 0.f;
#pragma unroll 1
    for (int az = 0; az < P; ++az) {
        float sy = 0.f;
#pragma unroll
        for (int ay = 0; ay < P; ++ay) sy = fmaf(m2p_row<P>(A + (az * P + ay) * P, hx), hy[ay], sy);
        acc = fmaf(sy, hz[az], acc);
    }
    return acc;
}

// The same sum with its rows spread over the lanes; every lane gets the total.
template <int P>
__device__ inline double m2p_wave(const float *__restrict__ A, float yx, float yy, float yz, int lane) {
    float hx[P];
    hermite_row<P>(yx, hx);
    float part = 0.f;
    for (int r = lane; r < P * P; r += 64) {
        const float sx = m2p_row<P>(A + r * P, hx);
        part = fmaf(sx, hermite_at(yy, r % P) * hermite_at(yz, r / P), part);
    }
    return wave_sum((double)part);
}

__device__ inline int wave_incl_scan(int v, int lane) {
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// One wavefront per node, striding over the nodes v0 .. v1 of one level.
// Levels must be processed from the deepest upward.  The children's records are
// read once, one lane per child; the points of the children that carry no
// moments (of the node itself for a leaf) are flattened into one list staged 64
// at a time; the moment blocks of the others are shifted (M2M) G at a time in LDS.
// M2M = false: no child of the level can carry moments (the children are leaves
// of at most leaf_max <= 70 points), so no shift buffers are needed.
template <int P, bool M2M>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4)))
k_node_moments(int64_t v0, int64_t v1, int level, const int32_t *nfirst, const int32_t *ncount,
               const int32_t *nfchild, const int32_t *nnchild, const int32_t *nix,
               const int32_t *niy, const int32_t *niz, const int32_t *ndigit, double lox,
               double loy, double loz, double side, const float4 *ps, double inv_sigma,
               const int32_t *nsrc, uint8_t *hasA, float *nodeA, int64_t slot0) {
    constexpr int P2 = P * P, P3 = P2 * P;
    constexpr int RP = (P2 + 63) / 64;                  // (ay, az) rows per lane
    constexpr bool MX = P == 8;                         // P2M on the matrix cores
    constexpr bool ILP = P == 1 || P == 2 || P == 4;
    constexpr int STR = MX ? 24 : ILP ? 4 : 3 * P + 1;  // staged floats per point
    constexpr int PR = P + 1;                           // padded row of a child block
    // about 4.5 KB of shift buffers, so that the wave's LDS stays near 8 KB and four
    // waves fit on each SIMD
    constexpr int G0 = 4608 / (P2 * PR * 4);
    constexpr int G = !M2M ? 1 : (G0 < 1 ? 1 : (G0 > 8 ? 8 : G0));   // child blocks shifted together
    // P <= 8: the eight child octants are shifted as a reduction tree (x-shifted
    // pairs summed, then y, then z), with four blocks in LDS; larger P: G child
    // blocks at a time, each shifted along x, y and z
    constexpr bool TREE = P <= 8;
    // the staged points and the shift buffers are used one after the other
    constexpr int NPTS = 64 * STR, NCB = !M2M ? 1 : TREE ? 4 * P2 * PR : G * P2 * PR;
    __shared__ __align__(16) float pts[NPTS > NCB ? NPTS : NCB];
    __shared__ float tot[P3];
    float *cbuf = pts;
    __shared__ float shift[2][P];                       // d^k / k! for the two child offsets
    __shared__ int32_t part_first[64], part_end[64];
    __shared__ int32_t och[8];                          // child of each octant digit with moments
    const int lane = threadIdx.x;
    const double h = side / (double)(1ll << level);
    if (lane < 2 * P) {
        const int bit = lane / P, k = lane % P;
        const double d = (bit - 0.5) * 0.5 * h * inv_sigma;   // child centre - node centre, in sigma
        double val = 1.0;
        for (int m = 1; m <= k; ++m) val *= d / m;
        shift[bit][k] = (float)val;
    }
    __syncthreads();
    for (int64_t v = v0 + blockIdx.x; v < v1; v += gridDim.x) {
        // the node's fields in one round of loads
        const int32_t ns = nsrc[v], nc = nnchild[v], nf = nfirst[v], ncnt = ncount[v], fch = nfchild[v];
        const int32_t ix = nix[v], iy = niy[v], iz = niz[v];
        const bool want = ns > kC1;
        if (lane == 0) hasA[v] = want ? 1 : 0;
        if (!want) continue;
        const double cx = lox + (ix + 0.5) * h, cy = loy + (iy + 0.5) * h, cz = loz + (iz + 0.5) * h;
        // parts: the children (lanes 0..nc-1), or the node itself when it is a leaf
        // or when no child can carry moments (then the children's points are the
        // node's own range and their records need not be read)
        int32_t cf = 0, cn = 0, cdig = 0, cid = -1;
        bool chas = false;
        if (nc == 0 || !M2M) {
            if (lane == 0) {
                cf = nf;
                cn = ncnt;
            }
        } else if (lane < nc) {
            cid = fch + lane;
            chas = hasA[cid] != 0;
            cf = nfirst[cid];
            cn = ncount[cid];
            cdig = ndigit[cid];
        }
        const int take = chas ? 0 : cn;
        const int incl = wave_incl_scan(take, lane);
        const int total = __shfl(incl, 63, 64);
        part_first[lane] = cf - (incl - take);
        part_end[lane] = take > 0 ? incl : -1;
        float acc[RP][P];
#pragma unroll
        for (int rr = 0; rr < RP; ++rr)
#pragma unroll
            for (int k = 0; k < P; ++k) acc[rr][k] = 0.f;

        // P2M (Eq. (7)) over the flattened points
        if constexpr (MX) {
            // with ay = 2 ay_hi + ay_lo the moments are the 16 x 32 product
            //   M[(ax, ay_lo)][(ay_hi, az)] = sum_j X_j^ax Y_j^ay_lo * w_j Y_j^(2 ay_hi) Z_j^az,
            // four points per v_mfma_f32_16x16x4f32 (two 16-column tiles); the points
            // pass through LDS 64 at a time as their powers X^k, Y^k and w Z^k (k < 8),
            // the next chunk held in registers
            const int mr = lane & 15, kq = lane >> 4;
            const int ax = mr >> 1, aylo = mr & 1, azc = mr & 7, ayh = mr >> 3;
            f32x4 d0 = {0.f, 0.f, 0.f, 0.f}, d1 = {0.f, 0.f, 0.f, 0.f};
            int owner = 0;
            float4 nxt = make_float4(0.f, 0.f, 0.f, 0.f);
            auto fetch = [&](int32_t c0) {
                const int32_t j = c0 + lane;
                nxt = make_float4(0.f, 0.f, 0.f, 0.f);   // past the list: weight 0
                if (j < total) {
                    while (part_end[owner] <= j) ++owner;
                    const float4 q = ps[part_first[owner] + j];
                    nxt = make_float4(((q.x - (float)cx) * (float)inv_sigma), ((q.y - (float)cy) * (float)inv_sigma),
                                      ((q.z - (float)cz) * (float)inv_sigma), q.w);
                }
            };
            __syncthreads();   // part_first / part_end written above
            fetch(0);
            for (int32_t c0 = 0; c0 < total; c0 += 64) {
                __syncthreads();
                {
                    float *r = pts + lane * STR;
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
                __syncthreads();
                if (c0 + 64 < total) fetch(c0 + 64);
                // rows past the list weigh 0, so the steps go in groups of eight (a
                // wave-uniform count): all operands of a group are read from LDS
                // before its products
                const int m = __builtin_amdgcn_readfirstlane(total - c0 < 64 ? total - c0 : 64);
                for (int s0 = 0; s0 < (m + 3) / 4; s0 += 8) {
                    float av[8], b0v[8], b1v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const float *r = pts + (4 * (s0 + u) + kq) * STR;
                        const float wzv = r[16 + azc];
                        av[u] = r[ax] * r[8 + aylo];
                        b0v[u] = r[8 + 2 * ayh] * wzv;
                        b1v[u] = r[8 + 2 * ayh + 4] * wzv;
                    }
                    __builtin_amdgcn_sched_barrier(0);   // keep the reads ahead of the products
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u], b0v[u], d0, 0, 0, 0);
                        d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u], b1v[u], d1, 0, 0, 0);
                    }
                }
            }
            // D[4 kq + i][n] of the two tiles, times 1 / (ax! ay! az!)
            float fz = 1.f;
            for (int k = 2; k <= azc; ++k) fz *= (float)k;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int mm = 4 * kq + i, axo = mm >> 1, ay0 = 2 * ayh + (mm & 1), ay1 = ay0 + 4;
                float fx = 1.f, f0 = 1.f, f1 = 1.f;
                for (int k = 2; k <= axo; ++k) fx *= (float)k;
                for (int k = 2; k <= ay0; ++k) f0 *= (float)k;
                for (int k = 2; k <= ay1; ++k) f1 *= (float)k;
                tot[(azc * 8 + ay0) * 8 + axo] = d0[i] / (fx * f0 * fz);
                tot[(azc * 8 + ay1) * 8 + axo] = d1[i] / (fx * f1 * fz);
            }
        } else if constexpr (ILP) {
            // lane = (point group, ay half, az): each lane accumulates the (ay, ax) block
            // of its az and half of the ay range over every NG-th staged point; the
            // groups are added by butterfly shuffles
            constexpr int H = 1;                  // ay halves per lane group
            constexpr int AY = P / H;
            constexpr int NG = 64 / (P * H);
            const int az = lane % P, ah = (lane / P) % H, grp = lane / (P * H);
            float a2[AY][P];
#pragma unroll
            for (int ay = 0; ay < AY; ++ay)
#pragma unroll
                for (int ax = 0; ax < P; ++ax) a2[ay][ax] = 0.f;
            float4 *pt4 = reinterpret_cast<float4 *>(pts);
            int owner = 0;
            // each lane holds the point of the next chunk while the current one is used
            float4 nxt = make_float4(0.f, 0.f, 0.f, 0.f);
            auto fetch = [&](int32_t c0) {
                const int32_t j = c0 + lane;
                if (j < total) {
                    while (part_end[owner] <= j) ++owner;
                    nxt = ps[part_first[owner] + j];
                }
            };
            __syncthreads();   // part_first / part_end written above
            fetch(0);
            for (int32_t c0 = 0; c0 < total; c0 += 64) {
                __syncthreads();
                if (c0 + lane < total)
                    pt4[lane] = make_float4(((nxt.x - (float)cx) * (float)inv_sigma),
                                            ((nxt.y - (float)cy) * (float)inv_sigma),
                                            ((nxt.z - (float)cz) * (float)inv_sigma), nxt.w);
                __syncthreads();
                if (c0 + 64 < total) fetch(c0 + 64);
                const int m = total - c0 < 64 ? total - c0 : 64;
                for (int jj = grp; jj < m; jj += NG) {
                    const float4 q = pt4[jj];
                    float wz = q.w;
                    for (int k = 0; k < az; ++k) wz *= q.z;
                    for (int k = 0; k < ah * AY; ++k) wz *= q.y;   // y^(first ay of the half)
                    float yp[AY], xp[P];
                    yp[0] = wz;
                    xp[0] = 1.f;
#pragma unroll
                    for (int k = 1; k < AY; ++k) yp[k] = yp[k - 1] * q.y;
#pragma unroll
                    for (int k = 1; k < P; ++k) xp[k] = xp[k - 1] * q.x;
#pragma unroll
                    for (int ay = 0; ay < AY; ++ay)
#pragma unroll
                        for (int ax = 0; ax < P; ++ax) a2[ay][ax] = fmaf(yp[ay], xp[ax], a2[ay][ax]);
                }
            }
#pragma unroll
            for (int o = P * H; o < 64; o <<= 1)
#pragma unroll
                for (int ay = 0; ay < AY; ++ay)
#pragma unroll
                    for (int ax = 0; ax < P; ++ax) a2[ay][ax] += __shfl_xor(a2[ay][ax], o, 64);
            if (grp == 0) {
                float fz = 1.f;
                for (int k = 2; k <= az; ++k) fz *= (float)k;
                float fy = 1.f;
                for (int k = 2; k <= ah * AY - 1; ++k) fy *= (float)k;   // (first ay - 1)!
#pragma unroll
                for (int i = 0; i < AY; ++i) {
                    const int ay = ah * AY + i;
                    if (ay > 1) fy *= (float)ay;
                    float fx = 1.f;
#pragma unroll
                    for (int ax = 0; ax < P; ++ax) {
                        if (ax > 1) fx *= (float)ax;
                        tot[(az * P + ay) * P + ax] = a2[i][ax] / (fx * fy * fz);
                    }
                }
            }
        } else {
            int owner = 0;
            for (int32_t c0 = 0; c0 < total; c0 += 64) {
                __syncthreads();
                const int32_t j = c0 + lane;
                if (j < total) {
                    while (part_end[owner] <= j) ++owner;
                    const float4 qp = ps[part_first[owner] + j];
                    const float X = ((qp.x - (float)cx) * (float)inv_sigma);
                    const float Y = ((qp.y - (float)cy) * (float)inv_sigma);
                    const float Z = ((qp.z - (float)cz) * (float)inv_sigma);
                    float *r = pts + lane * STR;
                    float px = qp.w, py = 1.f, pz = 1.f;
    #pragma unroll
                    for (int k = 0; k < P; ++k) {
                        r[k] = px;
                        r[P + k] = py;
                        r[2 * P + k] = pz;
                        px *= X;
                        py *= Y;
                        pz *= Z;
                    }
                }
                __syncthreads();
                const int m = total - c0 < 64 ? total - c0 : 64;
                for (int jj = 0; jj < m; ++jj) {
                    const float *r = pts + jj * STR;
    #pragma unroll
                    for (int rr = 0; rr < RP; ++rr) {
                        const int row = lane + 64 * rr;
                        if (row >= P2) continue;
                        const float fyz = r[P + row % P] * r[2 * P + row / P];
    #pragma unroll
                        for (int k = 0; k < P; ++k) acc[rr][k] = fmaf(fyz, r[k], acc[rr][k]);
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
                for (int k = 0; k < P; ++k) {
                    if (k > 1) fx *= (float)k;
                    tot[row * P + k] = acc[rr][k] / (fx * fyz);
                }
            }
        }

        // M2M of the children that carry moments:
        // A'_a = sum_{g<=a} A_g d^(a-g)/(a-g)! along x, then y, then z
        uint64_t todo = M2M ? __ballot(chas) : 0ull;
        if constexpr (M2M && TREE) {
            if (todo) {
                // octant digit 4 bx + 2 by + bz; pairs q = 2 by + bz
                if (lane < 8) och[lane] = -1;
                __syncthreads();
                if (chas) och[cdig] = cid;
                __syncthreads();
                // x: row (az, ay) of the two children of each pair, shifted and summed
                for (int r = lane; r < P2; r += 64) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        float o[P];
#pragma unroll
                        for (int k = 0; k < P; ++k) o[k] = 0.f;
#pragma unroll
                        for (int bx = 0; bx < 2; ++bx) {
                            const int32_t c = och[4 * bx + q];
                            if (c < 0) continue;
                            const float *row = nodeA + (int64_t)(c - slot0) * P3 + r * P;
                            float a[P];
#pragma unroll
                            for (int k = 0; k < P; ++k) a[k] = row[k];
#pragma unroll
                            for (int k = 0; k < P; ++k)
#pragma unroll
                                for (int m = 0; m <= k; ++m) o[k] = fmaf(a[m], shift[bx][k - m], o[k]);
                        }
                        float *dst = cbuf + (q * P2 + r) * PR;
#pragma unroll
                        for (int k = 0; k < P; ++k) dst[k] = o[k];
                    }
                }
                __syncthreads();
                // y: column (az, ax) of the pairs by = 0, 1 of each bz, into the by = 0 block
                for (int i = lane; i < 2 * P2; i += 64) {
                    const int bz = i / P2, az = (i % P2) / P, ax = i % P;
                    float o[P];
#pragma unroll
                    for (int k = 0; k < P; ++k) o[k] = 0.f;
#pragma unroll
                    for (int by = 0; by < 2; ++by) {
                        const float *col = cbuf + ((2 * by + bz) * P2 + az * P) * PR + ax;
                        float a[P];
#pragma unroll
                        for (int k = 0; k < P; ++k) a[k] = col[k * PR];
#pragma unroll
                        for (int k = 0; k < P; ++k)
#pragma unroll
                            for (int m = 0; m <= k; ++m) o[k] = fmaf(a[m], shift[by][k - m], o[k]);
                    }
                    float *col0 = cbuf + (bz * P2 + az * P) * PR + ax;
#pragma unroll
                    for (int k = 0; k < P; ++k) col0[k * PR] = o[k];
                }
                __syncthreads();
                // z: column (ay, ax) of the blocks bz = 0, 1, added to the node's moments
                for (int i = lane; i < P2; i += 64) {
                    const int ay = i / P, ax = i % P;
                    float o[P];
#pragma unroll
                    for (int k = 0; k < P; ++k) o[k] = 0.f;
#pragma unroll
                    for (int bz = 0; bz < 2; ++bz) {
                        const float *col = cbuf + (bz * P2 + ay) * PR + ax;
                        float a[P];
#pragma unroll
                        for (int k = 0; k < P; ++k) a[k] = col[k * P * PR];
#pragma unroll
                        for (int k = 0; k < P; ++k)
#pragma unroll
                            for (int m = 0; m <= k; ++m) o[k] = fmaf(a[m], shift[bz][k - m], o[k]);
                    }
#pragma unroll
                    for (int k = 0; k < P; ++k) tot[(k * P + ay) * P + ax] += o[k];
                }
            }
            todo = 0;
        }
        while (M2M && !TREE && todo) {
            int32_t gid[G];
            int gdig[G];
            int ng = 0;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                gid[g] = -1;
                gdig[g] = 0;
                if (todo) {
                    const int q = __builtin_ctzll(todo);
                    todo &= todo - 1;
                    gid[g] = __shfl(cid, q, 64);
                    gdig[g] = __shfl(cdig, q, 64);
                    ng = g + 1;
                }
            }
            __syncthreads();
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if (g >= ng) continue;
                const float *Ac = nodeA + (int64_t)(gid[g] - slot0) * P3;
                for (int e = lane; e < P3; e += 64) cbuf[g * P2 * PR + (e / P) * PR + e % P] = Ac[e];
            }
            __syncthreads();
            // x: rows (g, az, ay)
            for (int i = lane; i < ng * P2; i += 64) {
                const int g = i / P2;
                int bx = 0;
#pragma unroll
                for (int gg = 0; gg < G; ++gg)
                    if (gg == g) bx = (gdig[gg] >> 2) & 1;
                float *row = cbuf + g * P2 * PR + (i % P2) * PR;
                float a[P];
#pragma unroll
                for (int k = 0; k < P; ++k) a[k] = row[k];
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    float s = 0.f;
#pragma unroll
                    for (int m = 0; m <= k; ++m) s = fmaf(a[m], shift[bx][k - m], s);
                    row[k] = s;
                }
            }
            __syncthreads();
            // y: columns (g, az, ax)
            for (int i = lane; i < ng * P2; i += 64) {
                const int g = i / P2, az = (i % P2) / P, ax = i % P;
                int by = 0;
#pragma unroll
                for (int gg = 0; gg < G; ++gg)
                    if (gg == g) by = (gdig[gg] >> 1) & 1;
                float *col = cbuf + g * P2 * PR + az * P * PR + ax;
                float a[P];
#pragma unroll
                for (int k = 0; k < P; ++k) a[k] = col[k * PR];
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    float s = 0.f;
#pragma unroll
                    for (int m = 0; m <= k; ++m) s = fmaf(a[m], shift[by][k - m], s);
                    col[k * PR] = s;
                }
            }
            __syncthreads();
            // z: columns (g, ay, ax)
            for (int i = lane; i < ng * P2; i += 64) {
                const int g = i / P2, ay = (i % P2) / P, ax = i % P;
                int bz = 0;
#pragma unroll
                for (int gg = 0; gg < G; ++gg)
                    if (gg == g) bz = gdig[gg] & 1;
                float *col = cbuf + g * P2 * PR + ay * PR + ax;
                float a[P];
#pragma unroll
                for (int k = 0; k < P; ++k) a[k] = col[k * P * PR];
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    float s = 0.f;
#pragma unroll
                    for (int m = 0; m <= k; ++m) s = fmaf(a[m], shift[bz][k - m], s);
                    col[k * P * PR] = s;
                }
            }
            __syncthreads();
            for (int e = lane; e < P3; e += 64) {
                float s = tot[e];
                const int off = (e / P) * PR + e % P;
#pragma unroll
                for (int g = 0; g < G; ++g)
                    if (g < ng) s += cbuf[g * P2 * PR + off];
                tot[e] = s;
            }
        }
        __syncthreads();
        float *dst = nodeA + (v - slot0) * P3;
        for (int e = lane; e < P3; e += 64) dst[e] = tot[e];
        __syncthreads();
    }
}


// Queries whose node X holds at most kSmallNode points: the sums over its
// children straight from the points (direct sums), eight queries per wavefront,
// lane c of a query's eight summing the points of child c (contiguous in key
// order).  With a cutoff, children beyond the reach of the query are left out as
// in the walk.  Queries without children to choose from (a leaf node, an invalid
// target or node) get zeros and choice -1 here.
__global__ void __launch_bounds__(256)
k_partner_direct(int64_t nq, const int64_t *nq_dev, const int32_t *target_idx, const int32_t *node_id,
                 const float *uniforms,
                 int64_t n, int64_t n_nodes, const int32_t *qpos, const int32_t *nlevel,
                 const int32_t *nfirst, const int32_t *ncount, const int32_t *nfchild,
                 const int32_t *nnchild, const int32_t *nix, const int32_t *niy, const int32_t *niz,
                 double lox, double loy, double loz, double side, const float4 *ps, double sigma,
                 float cutoff2, int unlimited, int exclude_self, float *probs, int32_t *choice,
                 double *raw, unsigned long long *work) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t q = g >> 3;
    const int c = (int)(g & 7);
    const int lane = threadIdx.x & 63, gbase = lane & ~7;
    if (q >= (nq_dev ? *nq_dev : nq)) return;   // (the eight lanes of a query leave together)
    int32_t ti = target_idx[q], X = node_id[q], nc = 0, fc = 0;
    bool ok = ti >= 0 && ti < n && X >= 0 && X < n_nodes && qpos[q] >= 0;
    if (ok) {
        nc = nnchild[X];
        fc = nfchild[X];
        ok = nc > 0 && fc > X && fc + nc <= n_nodes;
    }
    if (!ok) {
        probs[q * 8 + c] = 0.f;
        if (raw) raw[q * 8 + c] = 0.0;
        if (c == 0 && choice) choice[q] = -1;
        return;
    }
    if (ncount[X] > kSmallNode) return;   // the wavefront pass or the walk
    const int32_t child = c < nc ? fc + c : -1;
    const int32_t si = qpos[q];
    const float4 qt = ps[si];
    const double tx = qt.x, ty = qt.y, tz = qt.z;
    const double kexp = 1.4426950408889634 / (sigma * sigma);
    auto box_d2 = [&](int32_t u) {
        const double h = side / (double)(1ll << nlevel[u]);
        const double half = 0.5 * h;
        const double gx = fmax(fabs(tx - (lox + (nix[u] + 0.5) * h)) - half, 0.0);
        const double gy = fmax(fabs(ty - (loy + (niy[u] + 0.5) * h)) - half, 0.0);
        const double gz = fmax(fabs(tz - (loz + (niz[u] + 0.5) * h)) - half, 0.0);
        return gx * gx + gy * gy + gz * gz;
    };
    auto box_d2_far = [&](int32_t u, double &far2) {
        const double h = side / (double)(1ll << nlevel[u]);
        const double half = 0.5 * h;
        const double ax = fabs(tx - (lox + (nix[u] + 0.5) * h)), ay = fabs(ty - (loy + (niy[u] + 0.5) * h)),
                     az = fabs(tz - (loz + (niz[u] + 0.5) * h));
        far2 = (ax + half) * (ax + half) + (ay + half) * (ay + half) + (az + half) * (az + half);
        const double gx = fmax(ax - half, 0.0), gy = fmax(ay - half, 0.0), gz = fmax(az - half, 0.0);
        return gx * gx + gy * gy + gz * gz;
    };
    int dg = -1, in = 0;
    int32_t uend = 0;
    if (child >= 0) {
        const int sh = nlevel[child] - nlevel[X] - 1;
        dg = (((nix[child] >> sh) & 1) << 2) | (((niy[child] >> sh) & 1) << 1) | ((niz[child] >> sh) & 1);
        in = 1;
        if (!unlimited) {
            const double reach = sqrt(box_d2(X)) + sqrt((double)cutoff2);
            in = box_d2(child) <= reach * reach;
        }
        uend = nfirst[child] + ncount[child];
    }
    // lane c sums the points of child c (a contiguous range in key order), eight
    // records in flight.  Each term in float32 relative to the node's closest
    // approach g0 to the target, exp(-(d^2 - g0^2) / sigma^2) <= 1 (scaled by
    // exp(-g0^2 / sigma^2) at the end, and moved to float64 every 32 terms), when
    // the node's farthest corner keeps every term above exp(-kSpan32) (far from
    // float32's underflow); wider nodes sum in float64.
    double far2;
    const double g0 = box_d2_far(X, far2);
    const bool narrow = (far2 - g0) * kexp <= kSpan32 * 1.4426950408889634;
    const float g0f = (float)g0, ksf = (float)kexp, txf = qt.x, tyf = qt.y, tzf = qt.z;
    double mysum = 0.0;
    if (child >= 0 && in) {
        const int32_t cf = nfirst[child], cend = uend;
        if (narrow) {
            float run = 0.f;
            int nrun = 0;
            for (int32_t j0 = cf; j0 < cend; j0 += 8) {
                float4 qv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) qv[u] = j0 + u < cend ? ps[j0 + u] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int32_t j = j0 + u;
                    const float4 qj = qv[u];
                    if (j >= cend || qj.w == 0.f || (exclude_self && j == si)) continue;
                    const float ex = txf - qj.x, ey = tyf - qj.y, ez = tzf - qj.z;
                    run = fmaf(qj.w, __builtin_amdgcn_exp2f((g0f - (ex * ex + ey * ey + ez * ez)) * ksf), run);
                }
                if (++nrun == 4) {
                    mysum += (double)run;
                    run = 0.f;
                    nrun = 0;
                }
            }
            mysum += (double)run;
            mysum *= exp2_neg(g0 * kexp);
        } else {
            for (int32_t j = cf; j < cend; ++j) {
                const float4 qj = ps[j];
                if (qj.w == 0.f || (exclude_self && j == si)) continue;
                const double ex = tx - qj.x, ey = ty - qj.y, ez = tz - qj.z;
                mysum += (double)qj.w * exp2_neg((ex * ex + ey * ey + ez * ez) * kexp);
            }
        }
    }
    // the group's sums and child ids by octant (lane k holds child k)
    double S[8];
    int32_t cid[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        S[d] = 0.0;
        cid[d] = -1;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const double sk = __shfl(mysum, gbase + k, 64);
        const int dk = __shfl(dg, gbase + k, 64);
        const int32_t ck = __shfl(child, gbase + k, 64);
#pragma unroll
        for (int d = 0; d < 8; ++d)
            if (d == dk && ck >= 0) {
                S[d] = sk;
                cid[d] = ck;
            }
    }
    double total = 0.0;
#pragma unroll
    for (int d = 0; d < 8; ++d) total += S[d];
    double mine = 0.0;
#pragma unroll
    for (int d = 0; d < 8; ++d)
        if (d == c) mine = S[d];
    probs[q * 8 + c] = total > 0.0 ? (float)(mine / total) : 0.f;
    if (raw) raw[q * 8 + c] = mine;
    if (c == 0 && work) {
        atomicAdd(&work[W_DIRECT_Q], 1ull);
        atomicAdd(&work[W_DIRECT_PAIRS], (unsigned long long)ncount[X]);
    }
    if (c == 0) {
        if (choice) {
            int32_t pick = -1;
            if (total > 0.0 && uniforms) {
                const double target = (double)uniforms[q] * total;
                double accp = 0.0;
                int32_t last = -1;
#pragma unroll
                for (int d = 0; d < 8; ++d) {
                    if (pick >= 0) continue;
                    if (S[d] > 0.0) last = cid[d];
                    accp += S[d];
                    if (accp > target && S[d] > 0.0) pick = cid[d];
                }
                if (pick < 0) pick = last;
            }
            choice[q] = pick;
        }
    }
}

// Queries whose node holds more than kSmallNode and at most kDirectPoints
// points: one wavefront per query sums the node's points directly, lane group g
// (eight lanes) the points of child g.  Other queries return at once.
__global__ void __launch_bounds__(256)
k_partner_wave(int64_t nq, const int64_t *nq_dev, const int32_t *target_idx, const int32_t *node_id,
               const float *uniforms,
               int64_t n, int64_t n_nodes, const int32_t *qpos, const int32_t *nlevel,
               const int32_t *nfirst, const int32_t *ncount, const int32_t *nfchild,
               const int32_t *nnchild, const int32_t *nix, const int32_t *niy, const int32_t *niz,
               double lox, double loy, double loz, double side, const float4 *ps, double sigma,
               float cutoff2, int unlimited, int exclude_self, float *probs, int32_t *choice,
               double *raw, unsigned long long *work) {
    const int64_t q = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (q >= (nq_dev ? *nq_dev : nq)) return;
    const int32_t ti = target_idx[q], X = node_id[q];
    if (!(ti >= 0 && ti < n && X >= 0 && X < n_nodes && qpos[q] >= 0)) return;
    const int nc = nnchild[X];
    const int32_t fc = nfchild[X];
    if (!(nc > 0 && fc > X && fc + nc <= n_nodes)) return;
    const int32_t cnt = ncount[X];
    if (cnt <= kSmallNode || cnt > kDirectPoints) return;
    const int32_t si = qpos[q];
    const float4 qt = ps[si];
    const double tx = qt.x, ty = qt.y, tz = qt.z;
    const double kexp = 1.4426950408889634 / (sigma * sigma);
    const int lx = nlevel[X];
    auto box_d2 = [&](int32_t u) {
        const double h = side / (double)(1ll << nlevel[u]);
        const double half = 0.5 * h;
        const double gx = fmax(fabs(tx - (lox + (nix[u] + 0.5) * h)) - half, 0.0);
        const double gy = fmax(fabs(ty - (loy + (niy[u] + 0.5) * h)) - half, 0.0);
        const double gz = fmax(fabs(tz - (loz + (niz[u] + 0.5) * h)) - half, 0.0);
        return gx * gx + gy * gy + gz * gz;
    };
    // child k of lane k: point range end, octant, within reach, node id
    int32_t uend = 0, cid = -1;
    int dg = 0, in = 0;
    if (lane < nc) {
        cid = fc + lane;
        uend = nfirst[cid] + ncount[cid];
        const int shf = nlevel[cid] - lx - 1;
        dg = (((nix[cid] >> shf) & 1) << 2) | (((niy[cid] >> shf) & 1) << 1) | ((niz[cid] >> shf) & 1);
        in = 1;
        if (!unlimited) {
            const double reach = sqrt(box_d2(X)) + sqrt((double)cutoff2);
            in = box_d2(cid) <= reach * reach;
        }
    }
    // the lane group g (lanes 8 g .. 8 g + 7) sums the points of child g, lane s of
    // the group taking every eighth one with eight records in flight (the group
    // reads whole lines); float32 terms relative to the node's closest approach
    // when the node is narrow enough (as in the eight-lane pass), float64 otherwise
    double g0, far2;
    {
        const double h = side / (double)(1ll << lx), half = 0.5 * h;
        const double ax = fabs(tx - (lox + (nix[X] + 0.5) * h)), ay = fabs(ty - (loy + (niy[X] + 0.5) * h)),
                     az = fabs(tz - (loz + (niz[X] + 0.5) * h));
        far2 = (ax + half) * (ax + half) + (ay + half) * (ay + half) + (az + half) * (az + half);
        const double gx = fmax(ax - half, 0.0), gy = fmax(ay - half, 0.0), gz = fmax(az - half, 0.0);
        g0 = gx * gx + gy * gy + gz * gz;
    }
    const bool narrow = (far2 - g0) * kexp <= kSpan32 * 1.4426950408889634;
    const float g0f = (float)g0, ksf = (float)kexp, txf = qt.x, tyf = qt.y, tzf = qt.z;
    const int grp = lane >> 3, sl = lane & 7;
    const int32_t gend = __shfl(uend, grp, 64), gcid = __shfl(cid, grp, 64);
    const int gin = __shfl(in, grp, 64);
    double mysum = 0.0;
    if (gcid >= 0 && gin) {
        const int32_t cf = nfirst[gcid];
        if (narrow) {
            float run = 0.f;
            int nrun = 0;
            for (int32_t j0 = cf + sl; j0 < gend; j0 += 64) {
                float4 qv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) qv[u] = j0 + 8 * u < gend ? ps[j0 + 8 * u] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int32_t j = j0 + 8 * u;
                    const float4 qj = qv[u];
                    if (j >= gend || qj.w == 0.f || (exclude_self && j == si)) continue;
                    const float ex = txf - qj.x, ey = tyf - qj.y, ez = tzf - qj.z;
                    run = fmaf(qj.w, __builtin_amdgcn_exp2f((g0f - (ex * ex + ey * ey + ez * ez)) * ksf), run);
                }
                if (++nrun == 4) {
                    mysum += (double)run;
                    run = 0.f;
                    nrun = 0;
                }
            }
            mysum += (double)run;
            mysum *= exp2_neg(g0 * kexp);
        } else {
            for (int32_t j = cf + sl; j < gend; j += 8) {
                const float4 qj = ps[j];
                if (qj.w == 0.f || (exclude_self && j == si)) continue;
                const double ex = tx - qj.x, ey = ty - qj.y, ez = tz - qj.z;
                mysum += (double)qj.w * exp2_neg((ex * ex + ey * ey + ez * ez) * kexp);
            }
        }
    }
    mysum += __shfl_xor(mysum, 1, 64);
    mysum += __shfl_xor(mysum, 2, 64);
    mysum += __shfl_xor(mysum, 4, 64);
    // per octant: child k's sum sits in lane 8 k
    double S[8], total = 0.0;
    int32_t cids[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        S[d] = 0.0;
        cids[d] = -1;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const double sk = __shfl(mysum, 8 * k, 64);
        const int dk = __shfl(dg, k, 64);
        const int32_t ck = __shfl(cid, k, 64);
#pragma unroll
        for (int d = 0; d < 8; ++d)
            if (ck >= 0 && d == dk) {
                S[d] = sk;
                cids[d] = ck;
            }
    }
#pragma unroll
    for (int d = 0; d < 8; ++d) total += S[d];
    if (lane < 8) {
        double mine = 0.0;
#pragma unroll
        for (int d = 0; d < 8; ++d)
            if (d == lane) mine = S[d];
        probs[q * 8 + lane] = total > 0.0 ? (float)(mine / total) : 0.f;
        if (raw) raw[q * 8 + lane] = mine;
    }
    if (lane == 0 && work) {
        atomicAdd(&work[W_WAVE_Q], 1ull);
        atomicAdd(&work[W_WAVE_PAIRS], (unsigned long long)cnt);
    }
    if (lane == 0 && choice) {
        int32_t pick = -1;
        if (total > 0.0 && uniforms) {
            const double target = (double)uniforms[q] * total;
            double accp = 0.0;
            int32_t last = -1;
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                if (pick >= 0) continue;
                if (S[d] > 0.0) last = cids[d];
                accp += S[d];
                if (accp > target && S[d] > 0.0) pick = cids[d];
            }
            if (pick < 0) pick = last;
        }
        choice[q] = pick;
    }
}

// The queries whose node holds more than kDirectPoints points.  The sums over
// the children of X come from a walk below X by the kWalkWaves
// wavefronts of a block, sharing one stack: each step takes up to 64 kWalkWaves
// nodes from the top of the stack, one per lane, and every node's children are
// pushed so that the nearest ends on top.  Decisions compare against
// R = max(lower bound, total summed so far), which never exceeds the final total;
// the lower bound comes first, from the chain of nearest nodes below X (the
// first node of the chain within reach carrying moments gives its M2P value
// minus the rigorous truncation bound, a leaf at the end of the chain its exact
// sum).  For a node carrying moments:
//   - dropped if all of its weight at its nearest point stays below kSkipTol R;
//   - M2P if the calibrated error model is below kAdmitTol of the node's own
//     smallest term, or below kRunTol R;
// otherwise its children are pushed, and a leaf is summed directly (by its
// lane, or by the whole wave when it holds more than kLaneLeaf points).
// Every decision and every sum is taken in a fixed order (nodes go to waves by
// their place on the stack, and the waves' partial sums are added in wave
// order), so the result is the same from run to run.
constexpr int kWalkWaves = 4;
constexpr int kStack = 4096;   // stack entries of a query

struct WalkShared {
    int32_t stk[kStack];
    int32_t c_first[kWalkWaves][64], c_end[kWalkWaves][64];
    int32_t m2p_order[kWalkWaves][64];   // lanes whose node is evaluated by expansion, in lane order
    float m2p_res[kWalkWaves][64];
    double part[kWalkWaves][8];          // per-wave partial sums of a step
    int32_t wpush[kWalkWaves];
    int32_t any_has[kWalkWaves];
    double lbv;
    int8_t c_digit[kWalkWaves][64];
};

// the idx-th query of the walk's order (coarsest query nodes first), or nq
__device__ inline int64_t walk_query_at(const int32_t *qorder, int64_t nq, int64_t idx) {
    const int32_t *tally = qorder + (size_t)kMaxLevels * nq;
    for (int l = 0; l < kMaxLevels; ++l) {
        if (idx < tally[l]) return qorder[(size_t)l * nq + idx];
        idx -= tally[l];
    }
    return nq;
}

struct WalkArgs {
    int64_t nq;
    const int32_t *target_idx, *node_id;
    const float *uniforms;
    int64_t n, n_nodes;
    const int32_t *qpos, *nlevel, *nfirst, *ncount, *nfchild, *nnchild, *nix, *niy, *niz;
    double lox, loy, loz, side;
    const float4 *ps;
    const uint8_t *hasA;
    const float *nodeA;
    int64_t slot0;
    double sigma;
    float cutoff2;
    int unlimited;
    double rho_ref;
    int exclude_self;
    float *probs;
    int32_t *choice;
    double *raw;
    const int32_t *qorder;
    unsigned long long *work;   // work counters (W_*), or NULL
};

// One query.  SHARED: walked by all kWalkWaves wavefronts of the block (this is
// wave wv), with the block's whole stack; otherwise wavefront wv walks it alone
// with its own quarter of the stack space.
template <int P, bool SHARED>
__device__ void walk_query(const WalkArgs &a, int64_t q, WalkShared &sh, int wv) {
    constexpr int P3 = P * P * P;
    constexpr int NW = SHARED ? kWalkWaves : 1;
    constexpr int cap = SHARED ? kStack : kStack / kWalkWaves;
    int32_t *stk = SHARED ? sh.stk : sh.stk + wv * (kStack / kWalkWaves);
    auto sync = [&]() {
        if constexpr (SHARED) __syncthreads();
        else wave_sync();
    };
    const int lane = threadIdx.x & 63;
    const bool lead = !SHARED || wv == 0;   // the wave that writes the query's outputs
    const int32_t ti = a.target_idx[q], X = a.node_id[q];
    const bool ok = ti >= 0 && ti < a.n && X >= 0 && X < a.n_nodes && a.qpos[q] >= 0;
    const int nc = ok ? a.nnchild[X] : 0;
    const int32_t fc = ok ? a.nfchild[X] : 0;
    if (nc == 0 || fc <= X || fc + nc > a.n_nodes) {
        if (lead) {
            if (lane < 8) a.probs[q * 8 + lane] = 0.f;
            if (lane < 8 && a.raw) a.raw[q * 8 + lane] = 0.0;
            if (lane == 0 && a.choice) a.choice[q] = -1;
        }
        return;
    }
    const int32_t si = a.qpos[q];
    const float4 qt = a.ps[si];
    const double tx = qt.x, ty = qt.y, tz = qt.z;
    const double inv_sigma = 1.0 / a.sigma;
    const double inv_s2 = inv_sigma * inv_sigma;
    const double kexp = 1.4426950408889634 * inv_s2;
    const int lx = a.nlevel[X];
    const int32_t *nlevel = a.nlevel, *nix = a.nix, *niy = a.niy, *niz = a.niz;
    const int32_t *nfirst = a.nfirst, *ncount = a.ncount, *nnchild = a.nnchild, *nfchild = a.nfchild;
    const float4 *ps = a.ps;
    const int64_t n_nodes = a.n_nodes, slot0 = a.slot0;
    const int unlimited = a.unlimited, exclude_self = a.exclude_self;
    auto centre = [&](int32_t u, double &cx, double &cy, double &cz, double &half) {
        const double h = a.side / (double)(1ll << nlevel[u]);
        cx = a.lox + (nix[u] + 0.5) * h;
        cy = a.loy + (niy[u] + 0.5) * h;
        cz = a.loz + (niz[u] + 0.5) * h;
        half = 0.5 * h;
    };
    // squared distance from the target to the box (near) and to its farthest corner (far)
    auto box_d2 = [&](int32_t u, double &far2) {
        double cx, cy, cz, half;
        centre(u, cx, cy, cz, half);
        const double ax = fabs(tx - cx), ay = fabs(ty - cy), az = fabs(tz - cz);
        const double gx = fmax(ax - half, 0.0), gy = fmax(ay - half, 0.0), gz = fmax(az - half, 0.0);
        far2 = (ax + half) * (ax + half) + (ay + half) * (ay + half) + (az + half) * (az + half);
        return gx * gx + gy * gy + gz * gz;
    };
    double far0;
    const double d0sq = box_d2(X, far0);
    const double reach = unlimited ? 0.0 : sqrt(d0sq) + sqrt((double)a.cutoff2);
    const double reach2 = reach * reach;
    // direct sum over one node's points by the whole wave
    auto wave_direct = [&](int32_t uf, int32_t un) {
        double part = 0.0;
        for (int32_t j = uf + lane; j < uf + un; j += 64) {
            const float4 qj = ps[j];
            if (qj.w == 0.f || (exclude_self && j == si)) continue;
            const double ex = tx - qj.x, ey = ty - qj.y, ez = tz - qj.z;
            part += (double)qj.w * exp2_neg((ex * ex + ey * ey + ez * ez) * kexp);
        }
        return wave_sum(part);
    };

    // lower bound of the total from the chain of nearest nodes (wave-uniform
    // call); a node reaching beyond the cutoff counts sources the walk drops, so
    // only the nodes of the chain that lie within reach contribute.  The first of
    // those carrying moments ends the chain: the nodes below it hold subsets of
    // its sources, so their sums cannot raise the bound beyond its own error.
    // this wave's work (wave-uniform): nodes visited, expansions evaluated, pairs summed
    unsigned long long w_nodes = 0, w_m2p = 0, w_pairs = 0, w_steps = 0;
    auto lower_bound = [&]() {
        double lb = 0.0;
        int32_t u = X;
        for (int guard = 0; guard <= kMaxLevels; ++guard) {
            double far2;
            (void)box_d2(u, far2);
            const bool inside = unlimited || far2 <= reach2;
            const int32_t uf = nfirst[u], un = ncount[u], unc = nnchild[u];
            if (inside && a.hasA[u]) {
                const float *A = a.nodeA + (int64_t)(u - slot0) * P3;
                double cx, cy, cz, half;
                centre(u, cx, cy, cz, half);
                double m = m2p_wave<P>(A, (float)((tx - cx) * inv_sigma), (float)((ty - cy) * inv_sigma),
                                       (float)((tz - cz) * inv_sigma), lane);
                ++w_m2p;
                if (exclude_self && si >= uf && si < uf + un) m -= (double)qt.w;
                lb = fmax(lb, m - trunc_bound(half * inv_sigma, P) * fabs((double)A[0]));
                break;
            }
            if (unc == 0) {
                if (inside) {
                    lb = fmax(lb, wave_direct(uf, un));
                    w_pairs += (unsigned long long)un;
                }
                break;
            }
            const int32_t f = nfchild[u];
            if (f <= u || f + unc > n_nodes) break;
            double bd = 1e300;
            int bl = 64;
            if (lane < unc) {
                double dummy;
                bd = box_d2(f + lane, dummy);
                bl = lane;
            }
            for (int o = 32; o > 0; o >>= 1) {
                const double od = __shfl_xor(bd, o, 64);
                const int ol = __shfl_xor(bl, o, 64);
                if (od < bd || (od == bd && ol < bl)) { bd = od; bl = ol; }
            }
            u = f + bl;
        }
        return lb;
    };

    // children of X, farthest at the bottom of the stack
    if (lead) {
        double dummy, dl = 0.0;
        if (lane < nc) dl = box_d2(fc + lane, dummy);
        int rank = 0;   // children farther away; ties: the larger index counts as farther
        for (int k = 0; k < nc; ++k) {
            const double dk = __shfl(dl, k, 64);
            rank += (dk > dl) || (dk == dl && k > lane);
        }
        if (lane < nc) stk[rank] = fc + lane;
    }
    int sp = nc;
    double S[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) S[d] = 0.0;
    double acc = 0.0, lb = 0.0;
    bool have_lb = false;
    int32_t *c_first = sh.c_first[wv], *c_end = sh.c_end[wv];
    int8_t *c_digit = sh.c_digit[wv];
    const double log_admit = log(kAdmitTol), log_runtol = log(kRunTol), log_skip = log(kSkipTol);
    const double log_model0 = log(2e-5);
    sync();
    while (sp > 0) {
        int B = sp < 64 * NW ? sp : 64 * NW;
        const int room = (cap - sp) / 7;   // pops B, pushes at most 8 B
        if (B > room) B = room > 1 ? room : 1;
        const int base = sp - B;
        const int slot = (SHARED ? wv * 64 : 0) + lane;   // this lane's place in the popped batch
        const int32_t u = slot < B ? stk[base + slot] : -1;
        const bool u_has = u >= 0 && a.hasA[u];
        if (a.work) {
            w_nodes += (unsigned long long)__popcll(__ballot(u >= 0));
            ++w_steps;
        }
        // the bound is needed only once a node carrying moments comes up
        if (!have_lb) {
            bool any = __ballot(u_has) != 0;
            if constexpr (SHARED) {
                if (lane == 0) sh.any_has[wv] = any ? 1 : 0;
                __syncthreads();
                any = false;
#pragma unroll
                for (int w = 0; w < NW; ++w) any = any || sh.any_has[w] != 0;
            }
            if (any) {
                if constexpr (SHARED) {
                    if (wv == 0) {
                        const double v = lower_bound();
                        if (lane == 0) sh.lbv = v;
                    }
                    __syncthreads();
                    lb = sh.lbv;
                } else {
                    lb = lower_bound();
                }
                have_lb = true;
            }
        }
        sync();   // every popped entry is read before pushes overwrite them
        const double run = fmax(lb, acc);
        const double lrun = run > 0.0 ? log(run) : -1e300;
        double val = 0.0;
        int digit = 0, npush = 0, nleaf = 0;
        bool big = false, do_m2p = false;
        float3 my = make_float3(0.f, 0.f, 0.f);
        int32_t uf = 0, un = 0, f = 0;
        if (u >= 0) {
            double cx, cy, cz, half;
            centre(u, cx, cy, cz, half);
            const int lu = nlevel[u];
            const int shf = lu - lx - 1;
            digit = (((nix[u] >> shf) & 1) << 2) | (((niy[u] >> shf) & 1) << 1) | ((niz[u] >> shf) & 1);
            double far2;
            const double g2 = box_d2(u, far2);
            uf = nfirst[u];
            un = ncount[u];
            const int32_t unc = nnchild[u];
            f = unc > 0 ? nfchild[u] : 0;
            if (unlimited || g2 <= reach2) {
                bool descend = unc > 0, direct = unc == 0;
                if (u_has) {
                    const float *A = a.nodeA + (int64_t)(u - slot0) * P3;
                    const double lw = log(fmax(fabs((double)A[0]), 1e-300));
                    if (lw - g2 * inv_s2 <= log_skip + lrun) {
                        descend = direct = false;
                    } else {
                        const double dx = tx - cx, dy = ty - cy, dz = tz - cz;
                        const double rho = half * inv_sigma;
                        const double r = sqrt(dx * dx + dy * dy + dz * dz) * inv_sigma;
                        // calibrated error model 2e-5 (rho / rho_max(p))^p of the expansion level
                        const double lm = log_model0 + P * log(rho / a.rho_ref);
                        const bool adm = lm + 0.5 * r * r + 2.0 * 1.7320508075688772 * rho * r + 3.0 * rho * rho <= log_admit ||
                                         lm + lw - 0.5 * r * r <= log_runtol + lrun;
                        if (adm) {
                            my = make_float3((float)(dx * inv_sigma), (float)(dy * inv_sigma),
                                             (float)(dz * inv_sigma));
                            if constexpr (P == 8) {
                                do_m2p = true;   // evaluated below by a lane group
                            } else {
                                val = (double)m2p_lane<P>(A, my.x, my.y, my.z);
                                do_m2p = true;   // (counted below; already evaluated)
                                if (exclude_self && si >= uf && si < uf + un) val -= (double)qt.w;
                            }
                            descend = direct = false;
                        }
                    }
                }
                if (direct) {
                    if (un <= kLaneLeaf) nleaf = un;
                    else big = true;
                }
                if (descend) {
                    if (f > u && f + unc <= n_nodes) npush = unc;
                    else big = true;   // malformed links: sum the node's points instead
                }
            }
        }
        if (a.work) w_m2p += (unsigned long long)__popcll(__ballot(do_m2p));
        if constexpr (P == 8) {
            // Eq. (7) for the nodes taken by expansion, eight nodes at a time: the
            // 8-lane group g evaluates one node, lane s of the group holding the
            // 16-byte pieces 8k + s (k < 16) of its 2 KB moment block, so that every
            // load of the group covers one whole 128-byte line
            const uint64_t mm = __ballot(do_m2p);
            if (mm) {
                int32_t *order = sh.m2p_order[wv];
                float *res = sh.m2p_res[wv];
                const int nm = __popcll(mm);
                const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
                if (do_m2p) order[__popcll(mm & below)] = lane;
                wave_sync();
                const int g = lane >> 3, sl = lane & 7;
                const int h = sl & 1, ayb = sl >> 1;
                for (int r0 = 0; r0 < nm; r0 += 8) {
                    const int k = r0 + g;
                    const int src = k < nm ? order[k] : lane;
                    const int32_t su = __shfl(u, src, 64);
                    const float yx = __shfl(my.x, src, 64), yy = __shfl(my.y, src, 64),
                                yz = __shfl(my.z, src, 64);
                    float part = 0.f;
                    if (k < nm) {
                        const float4 *blk = reinterpret_cast<const float4 *>(a.nodeA + (int64_t)(su - slot0) * P3);
                        float4 av[16];
#pragma unroll
                        for (int kk = 0; kk < 16; ++kk) av[kk] = blk[8 * kk + sl];
                        float hx[8], hy[8], hz[8];
                        hermite_row<8>(yx, hx);
                        hermite_row<8>(yy, hy);
                        hermite_row<8>(yz, hz);
#pragma unroll
                        for (int kk = 0; kk < 16; ++kk) {
                            // piece 8 kk + sl: az = kk / 2, ay = 4 (kk % 2) + sl / 2, ax = 4 (sl % 2) ..
                            const float4 v = av[kk];
                            float sx = v.x * hx[4 * h];
                            sx = fmaf(v.y, hx[4 * h + 1], sx);
                            sx = fmaf(v.z, hx[4 * h + 2], sx);
                            sx = fmaf(v.w, hx[4 * h + 3], sx);
                            part = fmaf(sx, hy[4 * (kk & 1) + ayb] * hz[kk >> 1], part);
                        }
                    }
                    part += __shfl_xor(part, 1, 64);
                    part += __shfl_xor(part, 2, 64);
                    part += __shfl_xor(part, 4, 64);
                    if (k < nm && sl == 0) res[src] = part;
                }
                wave_sync();
                if (do_m2p) {
                    val = (double)res[lane];
                    if (exclude_self && si >= uf && si < uf + un) val -= (double)qt.w;
                }
            }
        }
        // a single node taken with a nearly full stack (B = 1 is the only case
        // where the pushes can overflow): its points are summed instead
        if (B == 1 && npush > 0 && base + npush > cap) {
            big = true;
            npush = 0;
        }
        // pushes: this wave's lanes in lane order, the waves in wave order
        int incl = wave_incl_scan(npush, lane);
        int woff = 0, pushed = __shfl(incl, 63, 64);
        if constexpr (SHARED) {
            if (lane == 63) sh.wpush[wv] = incl;
            __syncthreads();
            pushed = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                if (w < wv) woff += sh.wpush[w];
                pushed += sh.wpush[w];
            }
        }
        if (npush > 0) {
            double cd[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                double fr;
                cd[k] = k < npush ? box_d2(f + k, fr) : 0.0;
            }
            const int pos0 = base + woff + incl - npush;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (k >= npush) continue;
                int rank = 0;
#pragma unroll
                for (int k2 = 0; k2 < 8; ++k2)
                    rank += k2 < npush && ((cd[k2] > cd[k]) || (cd[k2] == cd[k] && k2 > k));
                stk[pos0 + rank] = f + k;
            }
        }
        sp = base + pushed;
        // this wave's sums of the step, per octant: into the shared partials when
        // the block walks, into S (and acc) directly when the wave walks alone
        if constexpr (SHARED) {
            if (lane < 8) sh.part[wv][lane] = 0.0;
        }
        auto add_step = [&](int d, double v) {   // wave-uniform d and v
            if constexpr (SHARED) {
                if (lane == 0) sh.part[wv][d] += v;
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    if (e == d) S[e] += v;
                acc += v;
            }
        };
        // nodes summed by the whole wave
        uint64_t bigmask = __ballot(big);
        while (bigmask) {
            const int bl = __builtin_ctzll(bigmask);
            bigmask &= bigmask - 1;
            const int32_t bf = __shfl(uf, bl, 64), bn = __shfl(un, bl, 64);
            const int bd = __shfl(digit, bl, 64);
            add_step(bd, wave_direct(bf, bn));
            w_pairs += (unsigned long long)bn;
        }
        // the small leaves of the batch, their points spread over the lanes
        double pd[8];
#pragma unroll
        for (int d = 0; d < 8; ++d) pd[d] = (digit == d) ? val : 0.0;
        const int lincl = wave_incl_scan(nleaf, lane);
        const int ltotal = __shfl(lincl, 63, 64);
        w_pairs += (unsigned long long)ltotal;
        if (ltotal > 0) {
            c_first[lane] = uf - (lincl - nleaf);   // point index = c_first + flattened index
            c_end[lane] = nleaf > 0 ? lincl : -1;
            c_digit[lane] = (int8_t)digit;
            wave_sync();
            int owner = 0;
            for (int j = lane; j < ltotal; j += 64) {
                while (c_end[owner] <= j) ++owner;   // lanes in order, flattened indices increase
                const int32_t pj = c_first[owner] + j;
                const float4 qj = ps[pj];
                if (qj.w == 0.f || (exclude_self && pj == si)) continue;
                const double ex = tx - qj.x, ey = ty - qj.y, ez = tz - qj.z;
                const double e = (double)qj.w * exp2_neg((ex * ex + ey * ey + ez * ez) * kexp);
                const int dg = c_digit[owner];
#pragma unroll
                for (int d = 0; d < 8; ++d)
                    if (d == dg) pd[d] += e;
            }
        }
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            if (__ballot(pd[d] != 0.0) == 0) continue;
            add_step(d, wave_sum(pd[d]));
        }
        if constexpr (SHARED) {
            __syncthreads();
            // every wave adds the waves' sums in wave order: identical totals
#pragma unroll
            for (int w = 0; w < NW; ++w)
#pragma unroll
                for (int d = 0; d < 8; ++d) {
                    S[d] += sh.part[w][d];
                    acc += sh.part[w][d];
                }
        }
        sync();
    }
    if (a.work && lane == 0) {
        atomicAdd(&a.work[W_WALK_NODES], w_nodes);
        atomicAdd(&a.work[W_WALK_M2P], w_m2p);
        atomicAdd(&a.work[W_WALK_PAIRS], w_pairs);
        if (lead) {
            atomicAdd(&a.work[W_WALK_Q], 1ull);
            atomicAdd(&a.work[W_WALK_STEPS], w_steps);
        }
    }
    if (!lead) return;
    double total = 0.0;
#pragma unroll
    for (int d = 0; d < 8; ++d) total += S[d];
    // child node id per octant (absent children: -1)
    int32_t cid_l = -1;
    if (lane < 8) {
        for (int k = 0; k < nc; ++k) {
            const int32_t c = fc + k;
            const int shf = nlevel[c] - lx - 1;
            const int dg = (((nix[c] >> shf) & 1) << 2) | (((niy[c] >> shf) & 1) << 1) | ((niz[c] >> shf) & 1);
            if (dg == lane) cid_l = c;
        }
        double sl = 0.0;
#pragma unroll
        for (int d = 0; d < 8; ++d)
            if (d == lane) sl = S[d];
        a.probs[q * 8 + lane] = total > 0.0 ? (float)(sl / total) : 0.f;
        if (a.raw) a.raw[q * 8 + lane] = sl;
    }
    int32_t cids[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) cids[d] = __shfl(cid_l, d, 64);
    if (lane == 0 && a.choice) {
        int32_t pick = -1;
        if (total > 0.0 && a.uniforms) {
            const double target = (double)a.uniforms[q] * total;
            double accp = 0.0;
            int32_t last = -1;
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                if (pick >= 0) continue;
                if (S[d] > 0.0) last = cids[d];
                accp += S[d];
                if (accp > target && S[d] > 0.0) pick = cids[d];
            }
            if (pick < 0) pick = last;
        }
        a.choice[q] = pick;
    }
}

// Blocks take the queries of the walk, coarsest query nodes first (their walks
// are the longest, so they start early).  With at most four walks per block,
// each walk takes a whole block; otherwise every wavefront walks queries on its
// own: wavefront i the queries i, i + waves, ...
template <int P>
__global__ void __launch_bounds__(64 * kWalkWaves) k_partner(WalkArgs a) {
    __shared__ WalkShared sh;
    const int32_t *tally = a.qorder + (size_t)kMaxLevels * a.nq;
    int64_t nwalk = 0;
    for (int l = 0; l < kMaxLevels; ++l) nwalk += tally[l];
    const int wv = threadIdx.x >> 6;
    if (nwalk <= 4 * (int64_t)gridDim.x) {
        // few walks: each takes a whole block, block b the queries b, b + blocks, ...
        for (int64_t b = blockIdx.x; b < nwalk; b += gridDim.x) {
            __syncthreads();   // the previous query's shared state is no longer read
            walk_query<P, true>(a, walk_query_at(a.qorder, a.nq, b), sh, wv);
        }
        return;
    }
    // many walks: one wavefront each, every wavefront going on to its next query alone
    const int64_t stride = (int64_t)gridDim.x * kWalkWaves;
    for (int64_t i = (int64_t)blockIdx.x * kWalkWaves + wv; i < nwalk; i += stride)
        walk_query<P, false>(a, walk_query_at(a.qorder, a.nq, i), sh, wv);
}

// The walk's queries (valid ones whose node has children and more than
// kDirectPoints points; the direct passes take the others), coarsest query node
// first, without contention on a few counters: a block tallies its queries per
// level in LDS, reserves room for
// each level with one atomic addition, and places them in that level's segment
// order[l * nq ...]; the per-level tallies (after the segments) give the walk its
// mapping from block to query.  The order inside a level does not matter: every
// query writes only its own outputs.
__global__ void k_order_clear(int32_t *tally) {
    if (threadIdx.x < kMaxLevels) tally[threadIdx.x] = 0;
}

__global__ void __launch_bounds__(256) k_order_place(int64_t nq, const int64_t *nq_dev, const int32_t *target_idx,
                                                     const int32_t *node_id, int64_t n, int64_t n_nodes,
                                                     const int32_t *qpos, const int32_t *nlevel,
                                                     const int32_t *ncount, const int32_t *nfchild,
                                                     const int32_t *nnchild, int32_t *order) {
    __shared__ int32_t cnt[kMaxLevels], base[kMaxLevels];
    int32_t *tally = order + (size_t)kMaxLevels * nq;
    if (threadIdx.x < kMaxLevels) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int l = -1, slot = 0;
    if (q < (nq_dev ? *nq_dev : nq)) {
        const int32_t ti = target_idx[q], X = node_id[q];
        bool walk = ti >= 0 && ti < n && X >= 0 && X < n_nodes && qpos[q] >= 0;
        if (walk) {
            const int nc = nnchild[X];
            const int32_t fc = nfchild[X];
            walk = nc > 0 && fc > X && fc + nc <= n_nodes && ncount[X] > kDirectPoints;
        }
        if (walk) {
            l = nlevel[X];
            l = l < kMaxLevels ? l : kMaxLevels - 1;
            slot = atomicAdd(&cnt[l], 1);
        }
    }
    __syncthreads();
    if (threadIdx.x < kMaxLevels && cnt[threadIdx.x] > 0)
        base[threadIdx.x] = atomicAdd(&tally[threadIdx.x], cnt[threadIdx.x]);
    __syncthreads();
    if (l >= 0) order[(size_t)l * nq + base[l] + slot] = (int32_t)q;
}

}  // namespace

int source_prefix(msp_tree *t, hipStream_t s) {
    const int64_t n = t->n;
    const int64_t ntile = (n + kSrcTile - 1) / kSrcTile;
    MSP_TRY(t->src_prefix.ensure((size_t)(n + 1 + ntile) * 4));
    if (n == 0) return MSP_OK;
    int32_t *S = t->src_prefix.as<int32_t>();
    int32_t *tile = S + n + 1;
    hipLaunchKernelGGL(k_src_tiles, dim3((unsigned)ntile), dim3(256), 0, s, n, t->ps.as<float4>(), tile);
    MSP_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_src_tile_scan, dim3(1), dim3(1024), 0, s, ntile, tile);
    MSP_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_src_prefix, dim3((unsigned)ntile), dim3(256), 0, s, n, t->ps.as<float4>(), tile, S);
    MSP_CHECK_LAUNCH();
    t->src_prefix_gen = t->ps_gen;
    return MSP_OK;
}

namespace {

// coarsest level whose half-side is within rho_max(p) sigma: the moment level
int moment_level(const msp_tree *t, double sigma, int p) {
    const double rmax = rho_max_for_p(p);
    for (int l = 0; l <= kDepth; ++l)
        if (t->geo.side / std::ldexp(1.0, l + 1) / sigma <= rmax) return l;
    return kDepth;
}

// node moment pyramid (Eq. (7) and M2M) of the staged weights, from the deepest
// level up to the moment level
template <int P>
int partner_moments(msp_tree *t, const msp_fgt_params *prm, hipStream_t s) {
    const double sigma = prm->sigma;
    const int lh = moment_level(t, sigma, P);
    const int64_t nn = t->n_nodes;
    const int64_t slot0 = t->level_off[lh < kMaxLevels ? lh : kDepth + 1];
    const int64_t nslots = nn - slot0;
    MSP_TRY(t->node_hasA.ensure(nn));
    MSP_TRY(t->node_nsrc.ensure(nn * 4));
    MSP_TRY(t->nodeA.ensure((size_t)(nslots > 0 ? nslots : 1) * P * P * P * 4));
    {
        PhaseScope ps(&t->timing, PH_NODE_MOMENTS, s);
        {
            PhaseScope ps_counts(&t->timing, PH_NODE_COUNTS, s);
            if (t->n == 0) return fail(MSP_EINVAL, "node moments of an empty tree");
            // the prefix may come from the weighted build that staged these weights
            if (t->src_prefix_gen != t->ps_gen) MSP_TRY(source_prefix(t, s));
            hipLaunchKernelGGL(k_nsrc_nodes, dim3(grid_for(nn, kBlock)), dim3(kBlock), 0, s, nn,
                               t->nfirst.as<int32_t>(), t->ncount.as<int32_t>(), t->src_prefix.as<int32_t>(),
                               t->node_nsrc.as<int32_t>(), t->node_hasA.as<uint8_t>());
            MSP_CHECK_LAUNCH();
        }
        for (int l = t->depth; l >= 0; --l) {
            const int64_t a = t->level_off[l], b = t->level_off[l + 1];
            if (b <= a) continue;
            if (l < lh) break;
            // the deepest level holds only leaves, which never exceed leaf_max points
            if (l == t->depth && t->leaf_max <= kC1 && l < t->max_depth) continue;
            const int64_t nb = b - a < 65536 ? b - a : 65536;   // one node per block where it fits
            // children at the deepest level are leaves of at most leaf_max points: no moments
            const bool leaf_children = l + 1 == t->depth && t->leaf_max <= kC1 && l + 1 < t->max_depth;
            auto kern = leaf_children ? k_node_moments<P, false> : k_node_moments<P, true>;
            hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(64), 0, s, a, b,
                               l, t->nfirst.as<int32_t>(), t->ncount.as<int32_t>(), t->nfchild.as<int32_t>(),
                               t->nnchild.as<int32_t>(), t->nix.as<int32_t>(), t->niy.as<int32_t>(),
                               t->niz.as<int32_t>(), t->ndigit.as<int32_t>(), t->geo.lo[0], t->geo.lo[1],
                               t->geo.lo[2], t->geo.side, t->ps.as<float4>(), 1.0 / sigma,
                               t->node_nsrc.as<int32_t>(), t->node_hasA.as<uint8_t>(), t->nodeA.as<float>(),
                               slot0);
            MSP_CHECK_LAUNCH();
        }
    }
    t->node_moments_level = lh;
    t->node_moments_p = P;
    t->node_moments_bytes = (int64_t)(nslots > 0 ? nslots : 0) * P * P * P * 4;
    return MSP_OK;
}

// What the query kernels share: the queries' key-order positions, the walk's
// order (coarsest query node first) and the call's parameters.  Needs the node
// table only, not the node moments.
struct QuerySet {
    int64_t nq;
    const int64_t *nq_dev;
    const int32_t *target_idx, *node_id, *qpos;
    const float *uniforms;
    float *probs;
    int32_t *choice;
    double *raw;
    int32_t *order;
    double sigma, rmax;
    float R2;
    int unlimited, exclude_self;
    unsigned long long *work;
};

template <int P>
int queries_prepare(msp_tree *t, const msp_fgt_params *prm, const int32_t *target_idx,
                    const int32_t *node_id, int64_t nq, const float *uniforms, float *probs,
                    int32_t *choice, double *raw, const int32_t *qpos, hipStream_t s,
                    const int64_t *nq_dev, QuerySet *q) {
    // the walk's queries, coarsest first: per-level segments and their counters
    MSP_TRY(t->partner_order.ensure((size_t)((int64_t)kMaxLevels * nq + kMaxLevels) * 4));
    int32_t *order = t->partner_order.as<int32_t>();
    int32_t *tally = order + (size_t)kMaxLevels * nq;
    if (!qpos) {   // key-order positions of the targets (and the counters cleared)
        MSP_TRY(t->partner_qpos.ensure((size_t)nq * 4));
        const int64_t nthreads = nq > kMaxLevels ? nq : kMaxLevels;
        hipLaunchKernelGGL(k_query_pos, dim3(grid_for(nthreads, kBlock)), dim3(kBlock), 0, s, nq, target_idx, t->n,
                           t->pin.as<float4>(), t->keys.as<uint64_t>(), t->perm.as<int32_t>(), t->geo.lo[0],
                           t->geo.lo[1], t->geo.lo[2], t->geo.scale, t->partner_qpos.as<int32_t>(), tally);
        MSP_CHECK_LAUNCH();
        qpos = t->partner_qpos.as<int32_t>();
    } else {
        hipLaunchKernelGGL(k_order_clear, dim3(1), dim3(64), 0, s, tally);
        MSP_CHECK_LAUNCH();
    }
    const bool unlimited = !(prm->cutoff_sigmas > 0.f);
    const float R = unlimited ? 0.f : (float)(prm->cutoff_sigmas * prm->sigma);
    hipLaunchKernelGGL(k_order_place, dim3(grid_for(nq, kBlock)), dim3(kBlock), 0, s, nq, nq_dev, target_idx, node_id,
                       t->n, t->n_nodes, qpos, t->nlevel.as<int32_t>(), t->ncount.as<int32_t>(),
                       t->nfchild.as<int32_t>(), t->nnchild.as<int32_t>(), order);
    MSP_CHECK_LAUNCH();
    *q = QuerySet{nq, nq_dev, target_idx, node_id, qpos, uniforms, probs, choice, raw, order, prm->sigma,
                  rho_max_for_p(P), R * R, unlimited ? 1 : 0, (prm->flags & MSP_EXCLUDE_SELF) ? 1 : 0,
                  t->counting ? t->work.as<unsigned long long>() : nullptr};
    return MSP_OK;
}

// the walk (the queries whose node holds more than the wavefront pass takes),
// against the node moments of the last partner_moments call
template <int P>
int launch_walk(msp_tree *t, const QuerySet &q, hipStream_t s) {
    PhaseScope ps(&t->timing, PH_PARTNER, s);
    const int lh = moment_level(t, q.sigma, P);
    const int64_t nn = t->n_nodes;
    const int64_t slot0 = t->level_off[lh < kMaxLevels ? lh : kDepth + 1];
    WalkArgs wa{q.nq, q.target_idx, q.node_id, q.uniforms, t->n, nn, q.qpos, t->nlevel.as<int32_t>(),
                t->nfirst.as<int32_t>(), t->ncount.as<int32_t>(), t->nfchild.as<int32_t>(),
                t->nnchild.as<int32_t>(), t->nix.as<int32_t>(), t->niy.as<int32_t>(), t->niz.as<int32_t>(),
                t->geo.lo[0], t->geo.lo[1], t->geo.lo[2], t->geo.side, t->ps.as<float4>(),
                t->node_hasA.as<uint8_t>(), t->nodeA.as<float>(), slot0, q.sigma, q.R2, q.unlimited,
                q.rmax, q.exclude_self, q.probs, q.choice, q.raw, q.order, q.work};
    // as many blocks as the device holds at once (at most one per query)
    static int resident = 0;
    if (resident == 0) {
        int per_cu = 0, cus = 0, dev = 0;
        MSP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(k_partner<P>), 64 * kWalkWaves, 0));
        MSP_HIP(hipGetDevice(&dev));
        MSP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        resident = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
    }
    const int64_t nblocks = q.nq < resident ? q.nq : resident;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_partner<P>), dim3((unsigned)nblocks), dim3(64 * kWalkWaves), 0, s, wa);
    MSP_CHECK_LAUNCH();
    return MSP_OK;
}

// the eight-lane and wavefront passes (nodes of at most kDirectPoints points):
// point sums only, no node moments
int launch_direct(msp_tree *t, const QuerySet &q, hipStream_t s) {
    {
        PhaseScope pl(&t->timing, PH_PARTNER_DIRECT, s);
        hipLaunchKernelGGL(k_partner_direct, dim3(grid_for(q.nq * 8, 256)), dim3(256), 0, s, q.nq, q.nq_dev,
                           q.target_idx, q.node_id, q.uniforms, t->n, t->n_nodes, q.qpos, t->nlevel.as<int32_t>(),
                           t->nfirst.as<int32_t>(), t->ncount.as<int32_t>(), t->nfchild.as<int32_t>(),
                           t->nnchild.as<int32_t>(), t->nix.as<int32_t>(), t->niy.as<int32_t>(),
                           t->niz.as<int32_t>(), t->geo.lo[0], t->geo.lo[1], t->geo.lo[2], t->geo.side,
                           t->ps.as<float4>(), q.sigma, q.R2, q.unlimited, q.exclude_self, q.probs, q.choice,
                           q.raw, q.work);
        MSP_CHECK_LAUNCH();
    }
    {
        PhaseScope pw(&t->timing, PH_PARTNER_WAVE, s);
        hipLaunchKernelGGL(k_partner_wave, dim3(grid_for(q.nq, 4)), dim3(256), 0, s, q.nq, q.nq_dev, q.target_idx,
                           q.node_id, q.uniforms, t->n, t->n_nodes, q.qpos, t->nlevel.as<int32_t>(),
                           t->nfirst.as<int32_t>(), t->ncount.as<int32_t>(), t->nfchild.as<int32_t>(),
                           t->nnchild.as<int32_t>(), t->nix.as<int32_t>(), t->niy.as<int32_t>(),
                           t->niz.as<int32_t>(), t->geo.lo[0], t->geo.lo[1], t->geo.lo[2], t->geo.side,
                           t->ps.as<float4>(), q.sigma, q.R2, q.unlimited, q.exclude_self, q.probs, q.choice,
                           q.raw, q.work);
        MSP_CHECK_LAUNCH();
    }
    return MSP_OK;
}

// queries against the node moments of the last partner_moments call; raw (or
// NULL): the unnormalised per-octant sums.  The walk (few, long queries) runs on
// a side stream beside the direct passes (many short ones) on the caller's stream.
template <int P>
int partner_queries(msp_tree *t, const msp_fgt_params *prm, const int32_t *target_idx,
                    const int32_t *node_id, int64_t nq, const float *uniforms, float *probs,
                    int32_t *choice, double *raw, const int32_t *qpos, hipStream_t s,
                    const int64_t *nq_dev = nullptr) {
    if (nq == 0) return MSP_OK;
    QuerySet q;
    MSP_TRY(queries_prepare<P>(t, prm, target_idx, node_id, nq, uniforms, probs, choice, raw, qpos, s, nq_dev, &q));
    if (t->timing.on && t->timing.isolate) {
        MSP_TRY(launch_walk<P>(t, q, s));
        return launch_direct(t, q, s);
    }
    MSP_TRY(t->side.fork(s));
    MSP_TRY(launch_walk<P>(t, q, t->side.stream));
    MSP_TRY(launch_direct(t, q, s));
    return t->side.join(s);
}

}  // namespace

// moments and queries: the direct passes need no moments, so they start on a
// side stream while the caller's stream builds the moment pyramid, then the walk
template <int P>
int run_partner(msp_tree *t, const msp_fgt_params *prm, const int32_t *target_idx,
                const int32_t *node_id, int64_t nq, const float *uniforms, float *probs,
                int32_t *choice, hipStream_t s) {
    if (nq == 0) return partner_moments<P>(t, prm, s);
    QuerySet q;
    MSP_TRY(queries_prepare<P>(t, prm, target_idx, node_id, nq, uniforms, probs, choice, nullptr, nullptr, s,
                               nullptr, &q));
    if (t->timing.on && t->timing.isolate) {
        MSP_TRY(launch_direct(t, q, s));
        MSP_TRY(partner_moments<P>(t, prm, s));
        return launch_walk<P>(t, q, s);
    }
    MSP_TRY(t->side.fork(s));
    MSP_TRY(launch_direct(t, q, t->side.stream));
    MSP_TRY(partner_moments<P>(t, prm, s));
    MSP_TRY(launch_walk<P>(t, q, s));
    return t->side.join(s);
}

int partner_probabilities(msp_tree *t, const float *w, const msp_fgt_params *prm,
                          const int32_t *target_idx, const int32_t *node_id, int64_t nq,
                          const float *uniforms, float *probs, int32_t *choice, hipStream_t s) {
    if (t->n == 0) {
        if (nq > 0) return fail(MSP_EINVAL, "partner queries on an empty tree");
        return MSP_OK;
    }
    // MSP_WEIGHTS_STAGED: ps.w already holds w (gathered by the last call on the tree)
    if (!(prm->flags & MSP_WEIGHTS_STAGED)) MSP_TRY(stage_inputs(t, w, nullptr, s));
    switch (prm->p) {
#define CASE(P) case P: return run_partner<P>(t, prm, target_idx, node_id, nq, uniforms, probs, choice, s);
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
        CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16)
#undef CASE
    }
    return fail(MSP_EINVAL, "p out of range");
}


int partner_prepare(msp_tree *t, const float *w, const msp_fgt_params *prm, hipStream_t s) {
    MSP_TRY(stage_inputs(t, w, nullptr, s));
    switch (prm->p) {
#define CASE(P) case P: return partner_moments<P>(t, prm, s);
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
        CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16)
#undef CASE
    }
    return fail(MSP_EINVAL, "p out of range");
}

int partner_query_raw(msp_tree *t, const msp_fgt_params *prm, const int32_t *target_idx,
                      const int32_t *node_id, int64_t nq, float *probs, double *raw, const int32_t *qpos,
                      hipStream_t s, const int64_t *nq_dev) {
    switch (prm->p) {
#define CASE(P) case P: return partner_queries<P>(t, prm, target_idx, node_id, nq, nullptr, probs, nullptr, raw, qpos, s, nq_dev);
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
        CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16)
#undef CASE
    }
    return fail(MSP_EINVAL, "p out of range");
}

}  // namespace msp
