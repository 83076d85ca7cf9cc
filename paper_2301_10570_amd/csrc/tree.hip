// Octree build on the GPU: root cube, Morton keys, stable radix sort, and the
// adaptive node table (section "A Distributed Octree": a cell splits into its
// non-empty octants while it holds more than leaf_max points, up to max_depth).
//
// The node table is produced without a level-by-level descent.  For a point i in
// key order, the cells that contain it are nested and their point counts shrink
// with the level, so the cells containing i that are nodes are exactly those at
// levels 0..leaf_level(i), where leaf_level(i) = min(lambda(i) + 1, max_depth)
// and lambda(i) is the deepest level at which i's cell holds more than leaf_max
// points.  That cell holds more than leaf_max points iff some window of
// leaf_max + 1 consecutive sorted keys that contains i shares its prefix, so
// lambda(i) is a sliding-window maximum of L(j) = common-prefix level of
// key[j] and key[j + leaf_max].  A point starts a node at level l iff it is the
// first of its level-l cell (d(i) <= l, d from the highest differing bit of
// key[i-1] and key[i]) and l <= leaf_level(i).  Counting those starts per level
// gives breadth-first node order directly.
#include "internal.hpp"

#include <cmath>
#include <cstring>
#include <vector>

namespace msp {
namespace {

constexpr int kBlock = 256;
constexpr int kItems = 16;
constexpr int kTile = kBlock * kItems;   // points per block in tiled passes
// the node-level passes (point levels, node emission) take a tile with twice the
// threads: their rounds over the tile are sequential, half as many finish sooner
constexpr int kLvThreads = 512;

__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *lds, uint32_t &total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds[wid] = x;
    __syncthreads();
    uint32_t wbase = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        uint32_t s = lds[w];
        if (w < wid) wbase += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return wbase + x - v;
}

// ---- root cube --------------------------------------------------------------------------

__global__ void k_bbox_partial(const float *x, const float *y, const float *z, int64_t n,
                               float *part, int *bad) {
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    int nonfinite = 0;
    auto take = [&](float v, int k) {
        if (!isfinite(v)) {
            nonfinite = 1;
            return;
        }
        mn[k] = fminf(mn[k], v);
        mx[k] = fmaxf(mx[k], v);
    };
    auto take4 = [&](float4 v, int k) {
        take(v.x, k);
        take(v.y, k);
        take(v.z, k);
        take(v.w, k);
    };
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x, nth = (int64_t)gridDim.x * blockDim.x;
    int64_t head = 0;
    // 16-byte loads when the three arrays allow them, four of each in flight per thread
    if ((((uintptr_t)x | (uintptr_t)y | (uintptr_t)z) & 15) == 0) {
        const int64_t n4 = n >> 2;
        const float4 *x4 = reinterpret_cast<const float4 *>(x), *y4 = reinterpret_cast<const float4 *>(y),
                     *z4 = reinterpret_cast<const float4 *>(z);
        int64_t i = tid;
        for (; i + 3 * nth < n4; i += 4 * nth) {
            float4 a[4], b[4], c[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = x4[i + u * nth];
                b[u] = y4[i + u * nth];
                c[u] = z4[i + u * nth];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                take4(a[u], 0);
                take4(b[u], 1);
                take4(c[u], 2);
            }
        }
        for (; i < n4; i += nth) {
            take4(x4[i], 0);
            take4(y4[i], 1);
            take4(z4[i], 2);
        }
        head = n4 * 4;
    }
    for (int64_t i = head + tid; i < n; i += nth) {
        take(x[i], 0);
        take(y[i], 1);
        take(z[i], 2);
    }
    __shared__ float smn[3][kBlock], smx[3][kBlock];
    for (int k = 0; k < 3; ++k) { smn[k][threadIdx.x] = mn[k]; smx[k][threadIdx.x] = mx[k]; }
    if (nonfinite) atomicOr(bad, 1);
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 3; ++k) {
                smn[k][threadIdx.x] = fminf(smn[k][threadIdx.x], smn[k][threadIdx.x + s]);
                smx[k][threadIdx.x] = fmaxf(smx[k][threadIdx.x], smx[k][threadIdx.x + s]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) { part[blockIdx.x * 6 + k] = smn[k][0]; part[blockIdx.x * 6 + 3 + k] = smx[k][0]; }
}

__global__ void k_bbox_final(const float *part, int nparts, float *out) {
    __shared__ float sm[6][kBlock];
    float r[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int b = threadIdx.x; b < nparts; b += kBlock)
        for (int k = 0; k < 3; ++k) {
            r[k] = fminf(r[k], part[b * 6 + k]);
            r[3 + k] = fmaxf(r[3 + k], part[b * 6 + 3 + k]);
        }
    for (int k = 0; k < 6; ++k) sm[k][threadIdx.x] = r[k];
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int k = 0; k < 3; ++k) {
                sm[k][threadIdx.x] = fminf(sm[k][threadIdx.x], sm[k][threadIdx.x + st]);
                sm[3 + k][threadIdx.x] = fmaxf(sm[3 + k][threadIdx.x], sm[3 + k][threadIdx.x + st]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) out[threadIdx.x] = sm[threadIdx.x][0];
}

// ---- keys ----------------------------------------------------------------------------------

// The root cube comes from the bounding box in device memory, so that the build
// needs no host round trip before the keys.  One block per tile of the sort
// (kTile points, point r * kBlock + t of the tile to thread t), which also counts
// the tile's digits for the sort's first pass (bits shift .. shift + 7), in the
// layout k_rs_hist writes.
__global__ void __launch_bounds__(kBlock) k_morton(const float *x, const float *y, const float *z,
                                                   const float *w, int64_t n, const float *box, uint64_t *key,
                                                   int32_t *idx, float4 *pin, int shift, uint32_t *hist, int nblk) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    double lo[3], side, scale;
    root_cube(box, lo, side, scale);
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll 4
    for (int r = 0; r < kItems; ++r) {
        const int64_t i = base + r * kBlock + threadIdx.x;
        if (i >= n) continue;
        const float a = x[i], b = y[i], c = z[i];
        const uint64_t k = morton3(quantise(a, lo[0], scale), quantise(b, lo[1], scale), quantise(c, lo[2], scale));
        key[i] = k;
        idx[i] = (int32_t)i;
        // packed so that the sorted gather reads one line per point; the weight rides
        // along into key order when the caller gives one
        pin[i] = make_float4(a, b, c, w ? w[i] : 0.f);
        atomicAdd(&h[(k >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// ---- stable LSD radix sort of (key, index), 8 bits per pass ----------------------------------

__global__ void k_rs_hist(const uint64_t *keys, int64_t n, int shift, uint32_t *hist, int nblk) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    // every load of the thread in flight before the counting
    uint64_t k[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t i = base + r * kBlock + threadIdx.x;
        k[r] = i < n ? keys[i] : 0ull;
    }
#pragma unroll
    for (int r = 0; r < kItems; ++r)
        if (base + r * kBlock + threadIdx.x < n) atomicAdd(&h[(k[r] >> shift) & 255u], 1u);
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// One block per digit: exclusive scan of that digit's per-block counts, and its total.
__global__ void k_rs_digit_scan(uint32_t *hist, int nblk, uint32_t *total) {
    __shared__ uint32_t lds[kBlock / 64];
    uint32_t *row = hist + (int64_t)blockIdx.x * nblk;
    const int per = (nblk + kBlock - 1) / kBlock;
    const int b0 = threadIdx.x * per;
    uint32_t s = 0;
    for (int k = 0; k < per; ++k)
        if (b0 + k < nblk) s += row[b0 + k];
    uint32_t tot;
    uint32_t run = block_exclusive_scan(s, lds, tot);
    for (int k = 0; k < per; ++k)
        if (b0 + k < nblk) {
            uint32_t v = row[b0 + k];
            row[b0 + k] = run;
            run += v;
        }
    if (threadIdx.x == 0) total[blockIdx.x] = tot;
}

// Stable scatter of one 8-bit digit.  The tile is first ordered by digit in LDS
// (stable: ranks follow item order), then written out so that consecutive
// threads store consecutive positions of each digit's output run.  Each
// wavefront ranks a contiguous quarter of the tile on its own, with a digit
// counter of its own in LDS (lanes of one digit found by eight ballots, the
// last of them advancing the counter), so the ranking needs no block barrier;
// one scan over (digit, wavefront) then places the quarters in item order.
__global__ void __launch_bounds__(kBlock) k_rs_scatter(const uint64_t *kin, const int32_t *vin,
                                                       uint64_t *kout, int32_t *vout, int64_t n,
                                                       int shift, const uint32_t *hist,
                                                       const uint32_t *total, int nblk,
                                                       const float4 *pin, float4 *ps) {
    constexpr int kWaves = kBlock / 64;
    constexpr int kPerWave = kTile / kWaves;   // items of one wavefront, contiguous
    // the tile in digit order passes through LDS twice, keys then indices, in one
    // buffer (38 KB per block, so that four blocks share a compute unit)
    __shared__ uint64_t sk[kTile];
    int32_t *sv = reinterpret_cast<int32_t *>(sk);
    __shared__ uint32_t lds[kWaves];
    __shared__ uint32_t gbase[256];
    __shared__ uint32_t toff[256];
    __shared__ uint32_t wcnt[kWaves][256];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t tile = (int64_t)blockIdx.x * kTile;
    const int cnt = n - tile < kTile ? (int)(n - tile) : kTile;
    uint32_t tot;
    const uint32_t dbase = block_exclusive_scan(total[tid], lds, tot);
    gbase[tid] = dbase + hist[(int64_t)tid * nblk + blockIdx.x];
#pragma unroll
    for (int w = 0; w < kWaves; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    uint64_t k[kItems];
    int32_t v[kItems];
    uint32_t r[kItems];   // rank among the wavefront's items of the same digit
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int idx = wid * kPerWave + j * 64 + lane;
        const bool valid = idx < cnt;
        k[j] = valid ? kin[tile + idx] : 0ull;
        v[j] = valid ? vin[tile + idx] : 0;
    }
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int idx = wid * kPerWave + j * 64 + lane;
        const bool valid = idx < cnt;
        const uint32_t d = (uint32_t)(k[j] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        // every lane reads the counter before the digit's last lane writes it (one
        // wavefront's LDS accesses take effect in program order)
        const uint32_t before = wcnt[wid][d];
        r[j] = before + (uint32_t)__popcll(peers & lt);
        if (valid && (peers >> lane) == 1ull) wcnt[wid][d] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    uint32_t c = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) c += wcnt[w][tid];
    const uint32_t ex = block_exclusive_scan(c, lds, tot);
    toff[tid] = ex;
    uint32_t o = ex;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const uint32_t t = wcnt[w][tid];
        wcnt[w][tid] = o;   // now: where wavefront w's items of digit tid start in the tile
        o += t;
    }
    __syncthreads();
    uint32_t off[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const uint32_t d = (uint32_t)(k[j] >> shift) & 255u;
        off[j] = wcnt[wid][d] + r[j];
        if (wid * kPerWave + j * 64 + lane < cnt) sk[off[j]] = k[j];
    }
    __syncthreads();
    uint32_t pos[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int p = j * kBlock + tid;
        if (p < cnt) {
            const uint64_t key = sk[p];
            const uint32_t d = (uint32_t)(key >> shift) & 255u;
            pos[j] = gbase[d] + (uint32_t)p - toff[d];
            kout[pos[j]] = key;
        }
    }
    __syncthreads();   // the keys are read: the buffer takes the indices
#pragma unroll
    for (int j = 0; j < kItems; ++j)
        if (wid * kPerWave + j * 64 + lane < cnt) sv[off[j]] = v[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int p = j * kBlock + tid;
        if (p < cnt) {
            const int32_t val = sv[p];
            vout[pos[j]] = val;
            if (ps) ps[pos[j]] = pin[val];   // last pass: positions into key order
        }
    }
}

// ---- node table ------------------------------------------------------------------------------

// Level of the deepest common cell of two keys (21 if equal).
__device__ inline int common_level(uint64_t a, uint64_t b) {
    const uint64_t x = a ^ b;
    if (x == 0) return kDepth;
    const int hb = 63 - __clzll((long long)x);
    return kDepth - 1 - hb / 3;
}

// L[j] = common level of key[j] and key[j + leaf_max], j in [0, m).
__global__ void k_window_L(const uint64_t *keys, int64_t m, int leaf_max, int8_t *L) {
    int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= m) return;
    L[j] = (int8_t)common_level(keys[j], keys[j + leaf_max]);
}

// Prefix / suffix maxima of L inside consecutive blocks of W entries.
__global__ void k_window_presuf(const int8_t *L, int64_t m, int W, int8_t *pre, int8_t *suf) {
    int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t s = b * W;
    if (s >= m) return;
    int64_t e = s + W < m ? s + W : m;
    int8_t run = -1;
    for (int64_t j = s; j < e; ++j) { run = L[j] > run ? L[j] : run; pre[j] = run; }
    run = -1;
    for (int64_t j = e - 1; j >= s; --j) { run = L[j] > run ? L[j] : run; suf[j] = run; }
}

struct PointLevels {
    int d;   // first level at which the point starts a cell (22: never)
    int ll;  // level of its leaf
};

__device__ inline PointLevels point_levels(const uint64_t *keys, int64_t n, int64_t i, int leaf_max,
                                           int max_depth, const int8_t *pre, const int8_t *suf,
                                           int64_t m, int W) {
    PointLevels r;
    if (i == 0) r.d = 0;
    else {
        const uint64_t x = keys[i] ^ keys[i - 1];
        r.d = (x == 0) ? kDepth + 1 : kDepth - (63 - __clzll((long long)x)) / 3;
    }
    int lam = -1;
    if (m > 0) {
        const int64_t lo = i - leaf_max > 0 ? i - leaf_max : 0;
        const int64_t hi = i < m - 1 ? i : m - 1;
        if (lo <= hi) {
            if (lo / W == hi / W) lam = (lo % W == 0) ? pre[hi] : suf[lo];
            else lam = pre[hi] > suf[lo] ? pre[hi] : suf[lo];
        }
    }
    r.ll = lam + 1 < max_depth ? lam + 1 : max_depth;
    return r;
}

// Levels for leaf_max <= kWinMax: the window levels L(j) for the tile's windows are
// formed in LDS from the keys, and lambda(i) is the maximum over the windows
// containing i.  Points are striped over threads (coalesced); per-level start
// counts come from wave ballots.
constexpr int kWinMax = 1024;
template <int NT>
__global__ void __launch_bounds__(NT) k_levels_tile(const uint64_t *keys, int64_t n, int leaf_max,
                                                        int max_depth, uint8_t *dlev, uint8_t *llev,
                                                        uint32_t *blkcnt, int nblk) {
    __shared__ int8_t Ls[kTile + kWinMax];
    // window maxima by prefix and suffix maxima over blocks of W = leaf_max + 1
    // values (van Herk / Gil-Werman): the window [a, a + W - 1] is max(suf[a], pre[a + W - 1])
    __shared__ int8_t pre[kTile + kWinMax], suf[kTile + kWinMax];
    __shared__ uint32_t wc[NT / 64][kDepth + 1];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t tile = (int64_t)blockIdx.x * kTile;
    const int64_t m = n - leaf_max;
    const int NL = kTile + leaf_max, W = leaf_max + 1, NB = (NL + W - 1) / W;
    for (int idx = tid; idx < NL; idx += NT) {
        const int64_t j = tile - leaf_max + idx;
        Ls[idx] = (j >= 0 && j < m) ? (int8_t)common_level(keys[j], keys[j + leaf_max]) : (int8_t)-1;
    }
    if (tid <= kDepth)
        for (int w = 0; w < NT / 64; ++w) wc[w][tid] = 0;
    __syncthreads();
    for (int b = tid; b < 2 * NB; b += NT) {
        const int blk = b < NB ? b : b - NB;
        const int p0 = blk * W, p1 = p0 + W < NL ? p0 + W : NL;
        int mx = -1;
        if (b < NB) {
            for (int p = p0; p < p1; ++p) {
                mx = Ls[p] > mx ? Ls[p] : mx;
                pre[p] = (int8_t)mx;
            }
        } else {
            for (int p = p1 - 1; p >= p0; --p) {
                mx = Ls[p] > mx ? Ls[p] : mx;
                suf[p] = (int8_t)mx;
            }
        }
    }
    __syncthreads();
    uint32_t mycnt[kDepth + 1];
#pragma unroll
    for (int l = 0; l <= kDepth; ++l) mycnt[l] = 0;
    for (int r = 0; r < kTile / NT; ++r) {
        const int off = r * NT + tid;
        const int64_t i = tile + off;
        int d = 255, ll = 0;
        if (i < n) {
            if (i == 0) d = 0;
            else {
                const uint64_t x = keys[i] ^ keys[i - 1];
                d = (x == 0) ? kDepth + 1 : kDepth - (63 - __clzll((long long)x)) / 3;
            }
            const int s0 = suf[off], p1 = pre[off + leaf_max];
            const int lam = s0 > p1 ? s0 : p1;   // max of Ls[off .. off + leaf_max]
            ll = lam + 1 < max_depth ? lam + 1 : max_depth;
            dlev[i] = (uint8_t)d;
            llev[i] = (uint8_t)ll;
        }
#pragma unroll
        for (int l = 0; l <= kDepth; ++l) mycnt[l] += __popcll(__ballot(d <= l && l <= ll));
    }
    if (lane == 0)
#pragma unroll
        for (int l = 0; l <= kDepth; ++l) wc[wid][l] = mycnt[l];
    __syncthreads();
    if (tid <= kDepth) {
        uint32_t c = 0;
        for (int w = 0; w < NT / 64; ++w) c += wc[w][tid];
        blkcnt[(int64_t)tid * nblk + blockIdx.x] = c;
    }
}

// Node emission with striped points: for every level, the rank of a starting
// point among the block's starts at that level (in point order) from ballots,
// wave offsets and a running count per level.
template <int NT>
__global__ void __launch_bounds__(NT) k_emit_tile(const uint8_t *dlev, const uint8_t *llev,
                                                      int64_t n, const uint32_t *blkoff, int nblk,
                                                      const int64_t *level_off, int32_t *nfirst,
                                                      int32_t *nlevel) {
    // per-wave counts, double-buffered by item: the running totals of item r read
    // them after the second barrier while waves may already count item r + 1
    __shared__ uint32_t wcb[2][NT / 64][kDepth + 1];
    __shared__ uint32_t run[kDepth + 1];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t tile = (int64_t)blockIdx.x * kTile;
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    if (tid <= kDepth) run[tid] = 0;
    for (int r = 0; r < kTile / NT; ++r) {
        uint32_t(*wc)[kDepth + 1] = wcb[r & 1];
        const int64_t i = tile + r * NT + tid;
        const int d = i < n ? dlev[i] : 255;
        const int ll = i < n ? llev[i] : 0;
        // the levels at which some point of this wave starts a node (most points start
        // none: they continue their predecessor's cell below their leaf level)
        int lo = d <= ll ? d : kDepth + 1, hi = d <= ll ? ll : -1;
        for (int o = 32; o > 0; o >>= 1) {
            const int lo2 = __shfl_xor(lo, o, 64), hi2 = __shfl_xor(hi, o, 64);
            lo = lo2 < lo ? lo2 : lo;
            hi = hi2 > hi ? hi2 : hi;
        }
        if (lane <= kDepth) wc[wid][lane] = 0;
        wave_sync();
        for (int l = lo; l <= hi; ++l) {
            const uint64_t mk = __ballot(d <= l && l <= ll);
            if (lane == 0) wc[wid][l] = __popcll(mk);
        }
        __syncthreads();
        for (int l = lo; l <= hi; ++l) {
            const uint64_t mk = __ballot(d <= l && l <= ll);
            if (d <= l && l <= ll) {
                uint32_t off = run[l] + __popcll(mk & lt);
                for (int w = 0; w < wid; ++w) off += wc[w][l];
                const int64_t pos = level_off[l] + blkoff[(int64_t)l * nblk + blockIdx.x] + off;
                nfirst[pos] = (int32_t)i;
                nlevel[pos] = l;
            }
        }
        __syncthreads();
        if (tid <= kDepth) {
            uint32_t add = 0;
            for (int w = 0; w < NT / 64; ++w) add += wc[w][tid];
            run[tid] += add;
        }
    }
}

__global__ void k_levels(const uint64_t *keys, int64_t n, int leaf_max, int max_depth,
                         const int8_t *pre, const int8_t *suf, int64_t m, int W, uint8_t *dlev,
                         uint8_t *llev, uint32_t *blkcnt, int nblk) {
    __shared__ uint32_t cnt[kMaxLevels];
    if (threadIdx.x < kMaxLevels) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    uint32_t local[kDepth + 1];
#pragma unroll
    for (int l = 0; l <= kDepth; ++l) local[l] = 0;
    for (int k = 0; k < kItems; ++k) {
        const int64_t i = base + k;
        if (i >= n) break;
        PointLevels pl = point_levels(keys, n, i, leaf_max, max_depth, pre, suf, m, W);
        dlev[i] = (uint8_t)pl.d;
        llev[i] = (uint8_t)pl.ll;
#pragma unroll
        for (int l = 0; l <= kDepth; ++l) local[l] += (pl.d <= l && l <= pl.ll) ? 1u : 0u;
    }
#pragma unroll
    for (int l = 0; l <= kDepth; ++l)
        if (local[l]) atomicAdd(&cnt[l], local[l]);
    __syncthreads();
    if (threadIdx.x <= kDepth) blkcnt[(int64_t)threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

// One block per level: exclusive scan over blocks of that level's start counts.
__global__ void k_level_scan(uint32_t *blkcnt, int nblk, uint32_t *total) {
    __shared__ uint32_t lds[kBlock / 64];
    uint32_t *row = blkcnt + (int64_t)blockIdx.x * nblk;
    const int per = (nblk + kBlock - 1) / kBlock;
    const int b0 = threadIdx.x * per;
    uint32_t s = 0;
    for (int k = 0; k < per; ++k)
        if (b0 + k < nblk) s += row[b0 + k];
    uint32_t tot;
    uint32_t run = block_exclusive_scan(s, lds, tot);
    for (int k = 0; k < per; ++k)
        if (b0 + k < nblk) {
            uint32_t v = row[b0 + k];
            row[b0 + k] = run;
            run += v;
        }
    if (threadIdx.x == 0) total[blockIdx.x] = tot;
}

__global__ void k_level_offsets(const uint32_t *total, int64_t *level_off) {
    if (threadIdx.x != 0) return;
    int64_t run = 0;
    for (int l = 0; l <= kDepth; ++l) { level_off[l] = run; run += total[l]; }
    level_off[kDepth + 1] = run;
}

// Parent of every node: the last node one level up whose first point is at or
// before the node's own (binary search in the level's sorted firsts).
__global__ void k_parents(int64_t n_nodes, const int64_t *level_off, const int32_t *nlevel,
                          const int32_t *nfirst, int32_t *nparent) {
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= n_nodes) return;
    const int l = nlevel[v];
    nparent[v] = l == 0 ? -1
                        : (int32_t)(upper_bound_i32(nfirst, level_off[l - 1], level_off[l], nfirst[v]) - 1);
}

// Count, cell coordinates and children of every node.  The nodes of a level are
// in key order and the children of one node are consecutive among them, so a
// node ends where its next sibling starts; the last child of a node ends where
// its parent ends, which the chain of last children up to the first ancestor
// with a next sibling (or to the root, which ends at n) gives.  The children of
// an inner node are the nodes one level down from its first point to its end.
__global__ void k_nodes(const uint64_t *keys, int64_t n, const uint8_t *llev, int64_t n_nodes,
                        const int64_t *level_off, const int32_t *nlevel, const int32_t *nfirst,
                        const int32_t *nparent, int32_t *ncount, int32_t *ndigit, int32_t *nix, int32_t *niy,
                        int32_t *niz, int32_t *nfchild, int32_t *nnchild) {
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= n_nodes) return;
    const int l = nlevel[v];
    const int32_t f = nfirst[v];
    int64_t end = n;
    int64_t w = v;
    for (int guard = 0; guard <= kDepth + 1 && w > 0; ++guard) {
        const int64_t nx = w + 1;
        const int32_t pw = nparent[w];
        if (nx < level_off[nlevel[w] + 1] && nparent[nx] == pw) {
            end = nfirst[nx];
            break;
        }
        w = pw;
    }
    ncount[v] = (int32_t)(end - f);
    uint64_t prefix = 0;
    if (n > 0 && l > 0) prefix = keys[f] >> (3 * (kDepth - l));
    ndigit[v] = l > 0 ? (int32_t)(prefix & 7ull) : 0;
    nix[v] = (int32_t)compact3(prefix >> 2);
    niy[v] = (int32_t)compact3(prefix >> 1);
    niz[v] = (int32_t)compact3(prefix);
    const bool leaf = n == 0 || (int)llev[f] == l;
    if (leaf) {
        nfchild[v] = -1;
        nnchild[v] = 0;
    } else {
        const int64_t a = lower_bound_i32(nfirst, level_off[l + 1], level_off[l + 2], f);
        int64_t b = a;
        while (b < level_off[l + 2] && nfirst[b] < end && b - a < 8) ++b;
        nfchild[v] = (int32_t)a;
        nnchild[v] = (int32_t)(b - a);
    }
}

// Final ordering inside runs of equal 24-bit key prefix (level-8 cells).  The
// input is stably sorted by the prefix, so within a run the points are in index
// order; each point's place in the run is the number of run members with a
// smaller (key, index), which reproduces the stable sort by the full key.  A run
// that lies inside one wavefront's 64 entries is ranked from LDS; a run that
// crosses a wavefront boundary is found by scanning the neighbours in memory.
// Runs longer than kSegMax raise *overflow (the caller then sorts all 63 bits).
constexpr int kSegShift = 39;
constexpr int kSegMax = 256;
__global__ void __launch_bounds__(kBlock) k_seg_sort(const uint64_t *kin, const int32_t *vin, int64_t n,
                                                     uint64_t *kout, int32_t *vout, const float4 *pin,
                                                     float4 *ps, int *overflow) {
    __shared__ uint64_t sk[kBlock];
    __shared__ int32_t sv[kBlock];
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63, w0 = threadIdx.x - lane;
    const bool live = i < n;
    const uint64_t key = live ? kin[i] : ~0ull;
    const int32_t val = live ? vin[i] : 0;
    const uint64_t pre = key >> kSegShift;
    sk[threadIdx.x] = key;
    sv[threadIdx.x] = val;
    // run boundaries inside the wavefront (entries past n form runs of their own)
    const uint64_t pre_up = __shfl_up(pre, 1, 64), pre_dn = __shfl_down(pre, 1, 64);
    const bool starts = lane == 0 || pre_up != pre;
    const bool ends = lane == 63 || pre_dn != pre;
    const uint64_t smask = __ballot(starts), emask = __ballot(ends);
    __syncthreads();
    if (!live) return;
    const int s = 63 - __clzll((long long)(smask & ((lane == 63) ? ~0ull : ((2ull << lane) - 1))));
    const int e = __builtin_ctzll(emask & (~0ull << lane));
    // does the run continue into the previous or the next wavefront?
    const int64_t gs = i - lane + s, ge = i - lane + e;   // first and last entry inside this wavefront
    const bool open_lo = s == 0 && gs > 0 && (kin[gs - 1] >> kSegShift) == pre;
    const bool open_hi = e == 63 && ge + 1 < n && (kin[ge + 1] >> kSegShift) == pre;
    int64_t o;
    if (!open_lo && !open_hi) {
        o = gs;
        for (int j = s; j <= e; ++j) {
            const uint64_t kj = sk[w0 + j];
            o += (kj < key) || (kj == key && sv[w0 + j] < val);
        }
    } else {
        int64_t st = i, en = i + 1;
        int steps = 0;
        while (st > 0 && (kin[st - 1] >> kSegShift) == pre) {
            --st;
            if (++steps > kSegMax) {
                atomicOr(overflow, 1);
                return;
            }
        }
        while (en < n && (kin[en] >> kSegShift) == pre) {
            ++en;
            if (++steps > kSegMax) {
                atomicOr(overflow, 1);
                return;
            }
        }
        o = st;
        for (int64_t j = st; j < en; ++j) {
            const uint64_t kj = kin[j];
            o += (kj < key) || (kj == key && vin[j] < val);
        }
    }
    kout[o] = key;
    vout[o] = val;
    ps[o] = pin[val];
}

__global__ void k_inverse_perm(const int32_t *perm, int64_t n, int32_t *iperm) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    iperm[perm[i]] = (int32_t)i;
}

}  // namespace

int ensure_iperm(msp_tree *t, hipStream_t s) {
    if (t->iperm_valid) return MSP_OK;
    MSP_TRY(t->iperm.ensure((t->n > 0 ? t->n : 1) * 4));
    if (t->n > 0) {
        hipLaunchKernelGGL(k_inverse_perm, dim3(grid_for(t->n, kBlock)), dim3(kBlock), 0, s,
                           t->perm.as<int32_t>(), t->n, t->iperm.as<int32_t>());
        MSP_CHECK_LAUNCH();
    }
    t->iperm_valid = true;
    return MSP_OK;
}

namespace {

// bbox scratch: per-part minima/maxima (kBboxParts x 6 floats), the reduced 8
// floats, then two flags: non-finite input, and a sort run too long for k_seg_sort
constexpr int kBboxParts = 512;
inline int *bbox_flags(msp_tree *t) {
    return reinterpret_cast<int *>(t->bbox.as<float>() + kBboxParts * 6 + 8);
}

// Stable sort of (key, index), and the positions gathered into key order.
// fast: three 8-bit LSD passes over the top 24 key bits (the level-8 cell), then
// k_seg_sort inside the runs of equal prefix; it leaves a flag in the bbox
// scratch when a run is too long.  Otherwise: eight LSD passes over all bits.
// The digits of the first pass were counted by k_morton.
int sort_keys(msp_tree *t, int64_t n, int nblk, bool full, hipStream_t s) {
    PhaseScope ps(&t->timing, PH_SORT, s);
    uint64_t *ka = t->keys.as<uint64_t>(), *kb = t->keys2.as<uint64_t>();
    int32_t *va = t->perm.as<int32_t>(), *vb = t->perm2.as<int32_t>();
    uint32_t *hist = t->hist.as<uint32_t>();
    uint32_t *total = hist + (size_t)256 * nblk;
    const int first = full ? 0 : kSegShift, npass = full ? 8 : 3;
    for (int pass = 0; pass < npass; ++pass) {
        const int shift = first + pass * 8;
        if (pass > 0) {
            PhaseScope k1(&t->timing, PH_SORT_HIST, s);
            hipLaunchKernelGGL(k_rs_hist, dim3(nblk), dim3(kBlock), 0, s, ka, n, shift, hist, nblk);
            MSP_CHECK_LAUNCH();
        }
        {
            PhaseScope k2(&t->timing, PH_SORT_SCAN, s);
            hipLaunchKernelGGL(k_rs_digit_scan, dim3(256), dim3(kBlock), 0, s, hist, nblk, total);
            MSP_CHECK_LAUNCH();
        }
        const bool gather = full && pass == npass - 1;
        PhaseScope k3(&t->timing, PH_SORT_SCATTER, s);
        hipLaunchKernelGGL(k_rs_scatter, dim3(nblk), dim3(kBlock), 0, s, ka, va, kb, vb, n, shift, hist,
                           total, nblk, t->pin.as<float4>(), gather ? t->ps.as<float4>() : nullptr);
        MSP_CHECK_LAUNCH();
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (!full) {
        // three passes leave the data in keys2/perm2; the run sort writes keys/perm
        PhaseScope k4(&t->timing, PH_SORT_RUNS, s);
        int *overflow = bbox_flags(t) + 1;
        hipLaunchKernelGGL(k_seg_sort, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, ka, va, n,
                           t->keys.as<uint64_t>(), t->perm.as<int32_t>(), t->pin.as<float4>(),
                           t->ps.as<float4>(), overflow);
        MSP_CHECK_LAUNCH();
    }
    return MSP_OK;
}

}  // namespace

// ---------------------------------------------------------------------------------
// Device memory of a build.  Handle-owned buffers grow on demand; with caller
// buffers (tree_buf for what the tree keeps, ws for the build scratch) every array
// is bound to a region of them in the order below, which the size query repeats
// with counting carves.
namespace {

inline int build_blocks(int64_t n) {
    const int64_t b = (n + kTile - 1) / kTile;
    return b > 0 ? (int)b : 1;
}
constexpr size_t kBboxBytes = kBboxParts * 6 * sizeof(float) + 8 * sizeof(float) + 2 * sizeof(int);

// arrays the tree keeps, per point (sorted keys, permutation, sorted and input-order
// packed positions, inverse permutation) and the level offsets
void place_point_arrays(msp_tree *t, int64_t n, Carve &c) {
    const size_t nb = (size_t)(n > 0 ? n : 1);
    c.into(t->keys, nb * 8);
    c.into(t->perm, nb * 4);
    c.into(t->ps, nb * 16);
    c.into(t->pin, nb * 16);
    c.into(t->iperm, nb * 4);
    c.into(t->d_level_off, kMaxLevels * 8);
}

// the node table and the direct route's per-leaf list counts and offsets
void place_node_arrays(msp_tree *t, int64_t nn, Carve &c) {
    const size_t m = (size_t)(nn > 0 ? nn : 1);
    for (DevBuf *b : {&t->nlevel, &t->nfirst, &t->ncount, &t->nparent, &t->nfchild, &t->nnchild,
                      &t->ndigit, &t->nix, &t->niy, &t->niz})
        c.into(*b, m * 4);
    c.into(t->list_cnt, m * 4);
    c.into(t->list_off, (m + 1) * 8);
}

// build scratch
void place_scratch(msp_tree *t, int64_t n, Carve &c) {
    const size_t nb = (size_t)(n > 0 ? n : 1);
    const int nblk = build_blocks(n);
    c.into(t->bbox, kBboxBytes);
    c.into(t->keys2, nb * 8);
    c.into(t->perm2, nb * 4);
    c.into(t->hist, (size_t)256 * nblk * 4 + 256 * 4);
    c.into(t->dlev, nb);
    c.into(t->llev, nb);
    c.into(t->blkcnt, (size_t)kMaxLevels * nblk * 4 + kMaxLevels * 4);
    c.into(t->tmp_a, nb);
    c.into(t->tmp_b, nb);
    c.into(t->tmp_c, nb);
}

// drop caller regions left from an earlier build into caller buffers, so that a
// build into handle memory allocates its own
void unbind_fixed(msp_tree *t) {
    for (DevBuf *b : {&t->keys, &t->perm, &t->ps, &t->pin, &t->iperm, &t->d_level_off, &t->nlevel,
                      &t->nfirst, &t->ncount, &t->nparent, &t->nfchild, &t->nnchild, &t->ndigit, &t->nix,
                      &t->niy, &t->niz, &t->list_cnt, &t->list_off, &t->bbox, &t->keys2, &t->perm2, &t->hist,
                      &t->dlev, &t->llev, &t->blkcnt, &t->tmp_a, &t->tmp_b, &t->tmp_c})
        if (b->fixed) b->release();
}

}  // namespace

int64_t tree_node_bound(int64_t n, int leaf_max, int max_depth) {
    if (n <= 0) return 1;
    // a node below the root has a parent holding more than leaf_max points, and the
    // nodes of one level are disjoint and non-empty
    const int64_t inner = n / ((int64_t)leaf_max + 1);
    int64_t total = 1, pow8 = 1;
    for (int l = 1; l <= max_depth && inner > 0; ++l) {
        if (pow8 < n) pow8 *= 8;
        int64_t c = pow8 < n ? pow8 : n;
        if (8 * inner < c) c = 8 * inner;
        total += c;
    }
    return total;
}

void build_query_bytes(int64_t n, int leaf_max, int max_depth, size_t *tree_bytes, size_t *ws_bytes) {
    msp_tree probe;   // counting carves bind nothing real
    Carve tc(nullptr, 0), wc(nullptr, 0);
    place_point_arrays(&probe, n, tc);
    place_node_arrays(&probe, tree_node_bound(n, leaf_max, max_depth), tc);
    place_scratch(&probe, n, wc);
    *tree_bytes = tc.used;
    *ws_bytes = wc.used;
}

int build_tree(msp_tree *t, const float *x, const float *y, const float *z, int64_t n, int leaf_max,
               int max_depth, hipStream_t s, void *tree_buf, size_t tree_bytes, void *ws,
               size_t ws_bytes, const float *w) {
    t->built = false;
    const bool caller_mem = tree_buf != nullptr;
    Carve tc(tree_buf, tree_bytes);
    if (caller_mem) {
        Carve wc(ws, ws_bytes);
        place_point_arrays(t, n, tc);
        place_scratch(t, n, wc);
        if (!tc.fits() || !wc.fits()) {
            unbind_fixed(t);
            return fail(MSP_ENOSPC, "msp_octree_build_ws: tree buffer holds %zu bytes (%zu needed before the "
                        "node table), workspace %zu (%zu needed)", tree_bytes, tc.used, ws_bytes, wc.used);
        }
    } else {
        unbind_fixed(t);
    }
    t->iperm_valid = false;
    t->lists_valid = false;
    t->counts_valid = false;
    t->w_staged = false;
    ++t->ps_gen;   // the records are rewritten
    t->node_moments_level = -1;
    t->n = n;
    t->leaf_max = leaf_max;
    t->max_depth = max_depth;
    const int64_t nb = n > 0 ? n : 1;

    // root cube
    float box[6] = {0, 0, 0, 0, 0, 0};
    if (n > 0) {
        const int parts = kBboxParts;
        MSP_TRY(t->bbox.ensure(kBboxBytes));
        float *part = t->bbox.as<float>();
        float *out = part + parts * 6;
        int *bad = bbox_flags(t);
        MSP_HIP(hipMemsetAsync(bad, 0, 2 * sizeof(int), s));   // non-finite flag, sort-run overflow
        {
            PhaseScope ps(&t->timing, PH_BBOX, s);
            hipLaunchKernelGGL(k_bbox_partial, dim3(parts), dim3(kBlock), 0, s, x, y, z, n, part, bad);
            MSP_CHECK_LAUNCH();
            hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(kBlock), 0, s, part, parts, out);
            MSP_CHECK_LAUNCH();
        }
        // read back together with the level offsets once the keys are sorted
    }
    Geometry &g = t->geo;
    // the host geometry from the box (after the readback for n > 0)
    auto set_geometry = [&]() {
        double side = 0.0;
        root_cube(box, g.lo, side, g.scale);
        g.side = side;
        for (int k = 0; k < 3; ++k) {
            const double q = std::floor(((double)box[3 + k] - g.lo[k]) * g.scale);
            g.qmax[k] = q >= (double)kQMax ? (int32_t)kQMax : (int32_t)q;
        }
    };
    if (n == 0) set_geometry();

    // keys and sort
    MSP_TRY(t->keys.ensure(nb * 8));
    MSP_TRY(t->keys2.ensure(nb * 8));
    MSP_TRY(t->pin.ensure(nb * 16));
    MSP_TRY(t->ps.ensure(nb * 16));
    MSP_TRY(t->perm.ensure(nb * 4));
    MSP_TRY(t->perm2.ensure(nb * 4));
    const int nblk = build_blocks(n);
    MSP_TRY(t->hist.ensure((size_t)256 * nblk * 4 + 256 * 4));
    // per-point levels and node counts per level (scratch)
    MSP_TRY(t->dlev.ensure(nb));
    MSP_TRY(t->llev.ensure(nb));
    MSP_TRY(t->blkcnt.ensure((size_t)kMaxLevels * nblk * 4 + kMaxLevels * 4));
    MSP_TRY(t->d_level_off.ensure(kMaxLevels * 8));
    const int64_t m = n - leaf_max;   // windows of leaf_max + 1 keys
    const int W = leaf_max + 1;
    MSP_TRY(t->tmp_a.ensure(nb));
    MSP_TRY(t->tmp_b.ensure(nb));
    MSP_TRY(t->tmp_c.ensure(nb));
    int8_t *L = t->tmp_a.as<int8_t>(), *pre = t->tmp_b.as<int8_t>(), *suf = t->tmp_c.as<int8_t>();
    uint32_t *blkcnt = t->blkcnt.as<uint32_t>();
    uint32_t *ltot = blkcnt + (size_t)kMaxLevels * nblk;
    auto keys_and_sort = [&](bool full) -> int {
        {
            PhaseScope ps(&t->timing, PH_KEYS, s);
            hipLaunchKernelGGL(k_morton, dim3(nblk), dim3(kBlock), 0, s, x, y, z, w, n,
                               t->bbox.as<float>() + kBboxParts * 6, t->keys.as<uint64_t>(),
                               t->perm.as<int32_t>(), t->pin.as<float4>(), full ? 0 : kSegShift,
                               t->hist.as<uint32_t>(), nblk);
            MSP_CHECK_LAUNCH();
        }
        return sort_keys(t, n, nblk, full, s);
    };
    auto levels = [&]() -> int {
        PhaseScope ps(&t->timing, PH_LEVELS, s);
        if (leaf_max <= kWinMax) {
            hipLaunchKernelGGL(k_levels_tile<kLvThreads>, dim3(nblk), dim3(kLvThreads), 0, s, t->keys.as<uint64_t>(), n,
                               leaf_max, max_depth, t->dlev.as<uint8_t>(), t->llev.as<uint8_t>(),
                               blkcnt, nblk);
            MSP_CHECK_LAUNCH();
        } else {
            if (m > 0) {
                hipLaunchKernelGGL(k_window_L, dim3(grid_for(m, kBlock)), dim3(kBlock), 0, s,
                                   t->keys.as<uint64_t>(), m, leaf_max, L);
                MSP_CHECK_LAUNCH();
                const int64_t nwb = (m + W - 1) / W;
                hipLaunchKernelGGL(k_window_presuf, dim3(grid_for(nwb, kBlock)), dim3(kBlock), 0, s, L,
                                   m, W, pre, suf);
                MSP_CHECK_LAUNCH();
            }
            hipLaunchKernelGGL(k_levels, dim3(nblk), dim3(kBlock), 0, s, t->keys.as<uint64_t>(), n,
                               leaf_max, max_depth, pre, suf, m, W, t->dlev.as<uint8_t>(),
                               t->llev.as<uint8_t>(), blkcnt, nblk);
            MSP_CHECK_LAUNCH();
        }
        hipLaunchKernelGGL(k_level_scan, dim3(kDepth + 1), dim3(kBlock), 0, s, blkcnt, nblk, ltot);
        MSP_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_level_offsets, dim3(1), dim3(64), 0, s, ltot, t->d_level_off.as<int64_t>());
        MSP_CHECK_LAUNCH();
        return MSP_OK;
    };
    // one readback per build: level offsets, then the box and the two flags
    // (non-finite input, sort run overflow), into page-locked memory
    constexpr size_t kRbBox = kMaxLevels * 8;
    auto readback = [&]() -> int {
        MSP_TRY(t->build_stage.ensure(kRbBox + 8 * sizeof(float) + 2 * sizeof(int)));
        char *h = static_cast<char *>(t->build_stage.p);
        MSP_HIP(hipMemcpyAsync(h, t->d_level_off.p, kMaxLevels * 8, hipMemcpyDeviceToHost, s));
        MSP_HIP(hipMemcpyAsync(h + kRbBox, t->bbox.as<float>() + kBboxParts * 6, 8 * sizeof(float) + 2 * sizeof(int),
                               hipMemcpyDeviceToHost, s));
        MSP_HIP(hipStreamSynchronize(s));
        std::memcpy(t->level_off, h, kMaxLevels * 8);
        return MSP_OK;
    };
    // a weighted build (handle memory) also counts the sources before each position,
    // on a side stream beside the node levels and table, for the node moments of a
    // following partner call on the same weights
    const bool prefix = w != nullptr && n > 0 && !caller_mem;
    const bool side = prefix && !(t->timing.on && t->timing.isolate);
    if (n > 0) {
        MSP_TRY(keys_and_sort(false));
        if (prefix) {
            hipStream_t ps_stream = s;
            if (side) {
                MSP_TRY(t->side.fork(s));
                ps_stream = t->side.stream;
            }
            PhaseScope pc(&t->timing, PH_NODE_COUNTS, ps_stream);
            MSP_TRY(source_prefix(t, ps_stream));
        }
        MSP_TRY(levels());
        MSP_TRY(readback());
        const char *h = static_cast<const char *>(t->build_stage.p);
        int flags[2];
        std::memcpy(box, h + kRbBox, 6 * sizeof(float));
        std::memcpy(flags, h + kRbBox + 8 * sizeof(float), sizeof(flags));
        if (flags[0]) {
            if (side) MSP_TRY(t->side.join(s));
            return fail(MSP_EINVAL, "msp_octree_build: non-finite coordinate in input");
        }
        set_geometry();
        if (flags[1]) {
            // a run of equal 24-bit prefix was too long for the run sort: sort all bits
            // (after the source prefix, which read the records and is now stale)
            if (side) MSP_TRY(t->side.join(s));
            t->src_prefix_gen = -1;
            MSP_TRY(keys_and_sort(true));
            MSP_TRY(levels());
            MSP_TRY(readback());
        }
    } else {
        // empty input: a single empty root leaf
        t->level_off[0] = 0;
        for (int l = 1; l < kMaxLevels; ++l) t->level_off[l] = 1;
        MSP_HIP(hipMemcpyAsync(t->d_level_off.p, t->level_off, kMaxLevels * 8, hipMemcpyHostToDevice, s));
    }
    t->n_nodes = t->level_off[kDepth + 1];
    if (t->n_nodes > 0x7fffffffLL) return fail(MSP_EOVERFLOW, "msp_octree_build: too many nodes");
    t->depth = 0;
    for (int l = 0; l <= kDepth; ++l)
        if (t->level_off[l + 1] > t->level_off[l]) t->depth = l;

    const int64_t nn = t->n_nodes;
    if (caller_mem) {
        place_node_arrays(t, nn, tc);
        if (!tc.fits())
            return fail(MSP_ENOSPC, "msp_octree_build_ws: the tree has %lld nodes and needs %zu bytes; the tree "
                        "buffer holds %zu", (long long)nn, tc.used, tree_bytes);
    }
    for (DevBuf *b : {&t->nlevel, &t->nfirst, &t->ncount, &t->nparent, &t->nfchild, &t->nnchild,
                      &t->ndigit, &t->nix, &t->niy, &t->niz})
        MSP_TRY(b->ensure(nn * 4));
    // the direct route's per-leaf list lengths and offsets live with the node table,
    // so that a forward into a caller workspace needs no allocation for them
    MSP_TRY(t->list_cnt.ensure(nn * 4));
    MSP_TRY(t->list_off.ensure((nn + 1) * 8));
    {
    PhaseScope ps_nodes(&t->timing, PH_NODES, s);
    if (n > 0) {
        hipLaunchKernelGGL(k_emit_tile<kLvThreads>, dim3(nblk), dim3(kLvThreads), 0, s, t->dlev.as<uint8_t>(),
                           t->llev.as<uint8_t>(), n, blkcnt, nblk, t->d_level_off.as<int64_t>(),
                           t->nfirst.as<int32_t>(), t->nlevel.as<int32_t>());
        MSP_CHECK_LAUNCH();
    } else {
        int32_t zero = 0;
        MSP_HIP(hipMemcpyAsync(t->nfirst.p, &zero, 4, hipMemcpyHostToDevice, s));
        MSP_HIP(hipMemcpyAsync(t->nlevel.p, &zero, 4, hipMemcpyHostToDevice, s));
        MSP_HIP(hipStreamSynchronize(s));
    }
    hipLaunchKernelGGL(k_parents, dim3(grid_for(nn, kBlock)), dim3(kBlock), 0, s, nn,
                       t->d_level_off.as<int64_t>(), t->nlevel.as<int32_t>(), t->nfirst.as<int32_t>(),
                       t->nparent.as<int32_t>());
    MSP_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_nodes, dim3(grid_for(nn, kBlock)), dim3(kBlock), 0, s, t->keys.as<uint64_t>(),
                       n, t->llev.as<uint8_t>(), nn, t->d_level_off.as<int64_t>(), t->nlevel.as<int32_t>(),
                       t->nfirst.as<int32_t>(), t->nparent.as<int32_t>(), t->ncount.as<int32_t>(),
                       t->ndigit.as<int32_t>(), t->nix.as<int32_t>(), t->niy.as<int32_t>(),
                       t->niz.as<int32_t>(), t->nfchild.as<int32_t>(), t->nnchild.as<int32_t>());
    MSP_CHECK_LAUNCH();
    }

    if (side) MSP_TRY(t->side.join(s));   // (joining twice is harmless)
    t->built = true;
    t->w_staged = w != nullptr && n > 0;   // the sorted records carry the weights
    return MSP_OK;
}

}  // namespace msp
