// Pieces of the backward pass that the single-tree and the batched kernels share,
// so that both give the same bits: the direct sums with derivatives over the
// interaction list of one target leaf, the evaluation of a cell's Taylor series
// with derivatives at one point, and the combination of a point's two field
// records into its gradients.
//
// Record of a point (kRec floats, key order): the field A of the weights w
// (value, gradient x y z, Laplacian) at offset 0, the field B of the target
// weights g (value, gradient x y z) at offset 5.
#pragma once
#include "p2p_leaf.hpp"

namespace msp {
namespace {

constexpr int kRec = 16;   // floats per point record (64 bytes, one aligned segment)

// One tree's arrays as the direct sums with derivatives read them; the staged
// weights sit in ps.w, records go to out + i * stride (key order i).
struct GradLeafSet {
    int64_t n_nodes;
    const int32_t *nfirst, *ncount, *nnchild, *nlevel, *nix, *niy, *niz;
    BoxGeo geo;
    const int64_t *off;
    const int32_t *lst;
    const float4 *ps;
    float kexp, inv_s2;   // -log2(e) / sigma^2, 1 / sigma^2
    float *out;
};

struct GradShared {
    // staged sources (offsets from the leaf centre, weight) and their second weights
    // (two fields at once); slots 64..127 hold zeros for the idle lanes' reads
    float4 src[128];
    float sg[128];
    float red[9][64];
    int32_t efirst[64], eend[64];   // a window of list entries: point offset and end
};

// For every point of target leaf v (one wavefront; sh private to it): the sums
// over the source leaves of its list of e = w exp(-r^2/sigma^2), e (x - s) and
// e r^2, written as value, gradient and Laplacian of the field.  A block of nt <= 64
// targets splits the lanes into G = floor(64 / nt) groups of nt (the lanes past G nt
// idle), each group taking every G-th source of a staged chunk; the source points of up to 64 list entries
// at a time form one sequence staged 64 per chunk, the next chunk loaded while
// the current one is used; group partials are added in group order.
// TWO: a second field at once, with the key-order weights g2 of the sources (value
// and gradient, into out + 5): one exponential serves both, and each field's sums
// are formed exactly as a pass of its own would form them.
template <bool TWO>
__device__ inline void p2p_grad_leaf_t(const GradLeafSet &L, const float *g2, int64_t v, int stride, int want_lap,
                                       GradShared &sh) {
    if (v >= L.n_nodes || L.nnchild[v] != 0) return;
    const int lane = threadIdx.x & 63;
    float ct[3], half;
    node_box(L.geo, L.nlevel[v], L.nix[v], L.niy[v], L.niz[v], ct, half);
    const int32_t tf = L.nfirst[v], tn = L.ncount[v];
    const int64_t l0 = L.off[v];
    int64_t l1 = L.off[v + 1];
    if (l1 - l0 > L.n_nodes) l1 = l0 + L.n_nodes;   // a list names each node at most once
    sh.src[64 + lane] = make_float4(0.f, 0.f, 0.f, 0.f);
    sh.sg[64 + lane] = 0.f;
    for (int t0 = 0; t0 < tn; t0 += 64) {
        const int nt = tn - t0 < 64 ? tn - t0 : 64;
        const int tp = __builtin_amdgcn_readfirstlane(nt);
        const int G = 64 / tp;
        // lane / tp as a multiply by ceil(2^16 / tp): exact for lane < 64, tp <= 64
        const int grp = (lane * ((65536 + tp - 1) / tp)) >> 16;   // grp == G: an idle lane
        const int a = lane - grp * tp;
        const int32_t ti = tf + t0 + a;
        const float4 qt = L.ps[ti];
        const float tx = qt.x - ct[0], ty = qt.y - ct[1], tz = qt.z - ct[2];
        float su = 0.f, sx = 0.f, sy = 0.f, sz = 0.f, sr = 0.f;
        float gu = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
        for (int64_t w0 = l0; w0 < l1; w0 += 64) {
            const int nw = l1 - w0 < 64 ? (int)(l1 - w0) : 64;
            int32_t esf = 0, esn = 0;
            if (lane < nw) {
                const int32_t u = L.lst[w0 + lane];
                if (u >= 0 && u < L.n_nodes) {
                    esf = L.nfirst[u];
                    esn = L.ncount[u];
                }
            }
            const int incl = p2p_incl_scan(esn, lane);
            const int tot = __shfl(incl, 63, 64);
            wave_sync();   // previous window's entries and points are no longer read
            sh.efirst[lane] = esf - (incl - esn);
            sh.eend[lane] = esn > 0 ? incl : -1;
            wave_sync();
            int owner = 0;
            float4 nxt = make_float4(0.f, 0.f, 0.f, 0.f);
            float ngw = 0.f;
            auto fetch = [&](int c0) {
                const int j = c0 + lane;
                if (j < tot) {
                    while (sh.eend[owner] <= j) ++owner;
                    const int32_t pj = sh.efirst[owner] + j;
                    nxt = L.ps[pj];
                    if (TWO) ngw = g2[pj];
                }
            };
            fetch(0);
            for (int c0 = 0; c0 < tot; c0 += 64) {
                const int ns = tot - c0 < 64 ? tot - c0 : 64;
                wave_sync();
                // slots past the chunk's end hold a zero record (weights 0)
                const bool live = lane < ns;
                sh.src[lane] = live ? make_float4(nxt.x - ct[0], nxt.y - ct[1], nxt.z - ct[2], nxt.w)
                                    : make_float4(0.f, 0.f, 0.f, 0.f);
                if (TWO) sh.sg[lane] = live ? ngw : 0.f;
                wave_sync();
                if (c0 + 64 < tot) fetch(c0 + 64);
                // group grp takes sources grp, grp + G, ...: the same trip count on every lane
                // (a scalar loop); the slots read stay below ns + G <= 128, and a slot past the
                // chunk's end adds zeros
                const int nit = __builtin_amdgcn_readfirstlane((ns + G - 1) / G);
                const int Gs = __builtin_amdgcn_readfirstlane(G);
                for (int it = 0; it < nit; ++it) {
                    const int j = it * Gs + grp;
                    const float4 s4 = sh.src[j];
                    const float dx = tx - s4.x, dy = ty - s4.y, dz = tz - s4.z;
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    const float k = __builtin_amdgcn_exp2f(r2 * L.kexp);
                    // no contraction: either field's sums carry the same bits as a pass of its own
                    const float e = __fmul_rn(s4.w, k);
                    su = __fadd_rn(su, e);
                    sx = fmaf(e, dx, sx);
                    sy = fmaf(e, dy, sy);
                    sz = fmaf(e, dz, sz);
                    sr = fmaf(e, r2, sr);
                    if (TWO) {
                        const float eg = __fmul_rn(sh.sg[j], k);
                        gu = __fadd_rn(gu, eg);
                        gx = fmaf(eg, dx, gx);
                        gy = fmaf(eg, dy, gy);
                        gz = fmaf(eg, dz, gz);
                    }
                }
            }
        }
        wave_sync();
        sh.red[0][lane] = su;
        sh.red[1][lane] = sx;
        sh.red[2][lane] = sy;
        sh.red[3][lane] = sz;
        sh.red[4][lane] = sr;
        if (TWO) {
            sh.red[5][lane] = gu;
            sh.red[6][lane] = gx;
            sh.red[7][lane] = gy;
            sh.red[8][lane] = gz;
        }
        wave_sync();
        if (grp == 0 && a < nt) {
            constexpr int NR = TWO ? 9 : 5;
            float r[NR];
#pragma unroll
            for (int k = 0; k < NR; ++k) r[k] = 0.f;
            for (int q = 0; q < G; ++q)
#pragma unroll
                for (int k = 0; k < NR; ++k) r[k] += sh.red[k][q * tp + a];
            float *o = L.out + (int64_t)ti * stride;   // value, gradient x y z, Laplacian
            o[0] = r[0];
            o[1] = -2.f * L.inv_s2 * r[1];
            o[2] = -2.f * L.inv_s2 * r[2];
            o[3] = -2.f * L.inv_s2 * r[3];
            if (want_lap) o[4] = 4.f * L.inv_s2 * L.inv_s2 * r[4] - 6.f * L.inv_s2 * r[0];
            if (TWO) {
                o[5] = r[5];
                o[6] = -2.f * L.inv_s2 * r[6];
                o[7] = -2.f * L.inv_s2 * r[7];
                o[8] = -2.f * L.inv_s2 * r[8];
            }
        }
    }
}

__device__ inline void p2p_grad_leaf(const GradLeafSet &L, int64_t v, int stride, int want_lap, GradShared &sh) {
    p2p_grad_leaf_t<false>(L, nullptr, v, stride, want_lap, sh);
}

// The gradients of input point j from its record (rec4: the record as float4),
// its target weight g and weight wj; returns its term of the sigma derivative.
__device__ inline double combine_point(const float4 *rec4, float g, float wj, int want_w, int want_pos,
                                       int want_sigma, double sigma, int exclude_self, float *gw, float *gx,
                                       float *gy, float *gz) {
    const float4 a = rec4[0], b = rec4[1], c = rec4[2];
    // a = (Av, Agx, Agy, Agz), b = (Alap, Bv, Bgx, Bgy), c = (Bgz, -, -, -)
    if (want_w) *gw = exclude_self ? b.y - g : b.y;
    if (want_pos) {
        *gx = g * a.y + wj * b.z;
        *gy = g * a.z + wj * b.w;
        *gz = g * a.w + wj * c.x;
    }
    return want_sigma ? (double)g * (0.5 * sigma * (double)b.x + 3.0 / sigma * (double)a.x) : 0.0;
}

}  // namespace
}  // namespace msp
