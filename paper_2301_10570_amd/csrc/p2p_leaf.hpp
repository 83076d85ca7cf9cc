// P2P of one target leaf against its interaction list (Eq. (8)); shared by the
// single-tree direct route and the batched persistent kernel.
//
// One wavefront per target leaf (sh is private to the wave).  A block of nt <= 64
// targets splits the lanes into G = floor(64 / nt) groups of nt (the lanes past G nt
// idle); each group takes every G-th source of a staged chunk, and the group
// partials are added in group order at the end.  The source
// leaves of the list are read 64 entries at a time and their points concatenated,
// so that a chunk of 64 staged sources may span several leaves.  Chunk partials
// are added with compensation.  exp(-d^2/sigma^2) is evaluated as
// exp2(-(k d)^2) with k^2 = log2(e)/sigma^2 (k = k_scale); the sources of a chunk
// sit in LDS as one 16-byte record each.
#pragma once
#include "internal.hpp"

namespace msp {
namespace {

struct BoxGeo {
    double lo[3];
    double side;
};

__device__ inline void node_box(const BoxGeo &g, int level, int ix, int iy, int iz, float c[3],
                                float &half) {
    const double h = g.side / (double)(1ll << level);
    c[0] = (float)(g.lo[0] + (ix + 0.5) * h);
    c[1] = (float)(g.lo[1] + (iy + 0.5) * h);
    c[2] = (float)(g.lo[2] + (iz + 0.5) * h);
    half = (float)(0.5 * h);
}

// One tree's arrays as the P2P pass reads them.
struct LeafSet {
    int64_t n_nodes;
    const int32_t *nfirst, *ncount, *nnchild, *nlevel, *nix, *niy, *niz;
    BoxGeo geo;
    const int64_t *off;
    const int32_t *lst;
    const float4 *ps;
    const uint8_t *tflag;
    float k_scale;
    int exclude_self;
    float *usort;
};

struct P2PShared {
    // staged sources (scaled offsets from the leaf centre, weight) and their point
    // indices; slots 64..127 hold zero records for the idle lanes' reads
    float4 sp[128];
    int32_t sid[128];
    float red[64];
    int32_t efirst[64], eend[64];   // a window of list entries: point offset and end
};

__device__ inline int p2p_incl_scan(int v, int lane) {
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

__device__ inline void p2p_leaf(const LeafSet &L, int64_t v, P2PShared &sh) {
    if (v >= L.n_nodes || L.nnchild[v] != 0) return;
    const int lane = threadIdx.x & 63;
    float ct[3], ht;
    node_box(L.geo, L.nlevel[v], L.nix[v], L.niy[v], L.niz[v], ct, ht);
    const int32_t tf = L.nfirst[v], tn = L.ncount[v];
    const int64_t l0 = L.off[v];
    int64_t l1 = L.off[v + 1];
    if (l1 - l0 > L.n_nodes) l1 = l0 + L.n_nodes;   // a list names each node at most once
    sh.sp[64 + lane] = make_float4(0.f, 0.f, 0.f, 0.f);
    sh.sid[64 + lane] = -1;
    for (int t0 = 0; t0 < tn; t0 += 64) {
        const int nt = tn - t0 < 64 ? tn - t0 : 64;
        const int tp = __builtin_amdgcn_readfirstlane(nt);
        const int G = 64 / tp;
        // lane / tp as a multiply by ceil(2^16 / tp): exact for lane < 64, tp <= 64
        const int grp = (lane * ((65536 + tp - 1) / tp)) >> 16;   // grp == G: an idle lane
        const int a = lane - grp * tp;
        const int32_t ti = tf + t0 + a;
        const float4 qt = L.ps[ti];
        const float tx = (qt.x - ct[0]) * L.k_scale;
        const float ty = (qt.y - ct[1]) * L.k_scale;
        const float tz = (qt.z - ct[2]) * L.k_scale;
        float total = 0.f, comp = 0.f;
        // the source points of up to 64 list entries at a time form one sequence that is
        // staged 64 points per chunk; the next chunk is loaded while the current one is used
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
            int32_t nid = -1;
            auto fetch = [&](int c0) {
                const int j = c0 + lane;
                if (j < tot) {
                    while (sh.eend[owner] <= j) ++owner;
                    nid = sh.efirst[owner] + j;
                    nxt = L.ps[nid];
                }
            };
            fetch(0);
            for (int c0 = 0; c0 < tot; c0 += 64) {
                const int ns = tot - c0 < 64 ? tot - c0 : 64;
                wave_sync();
                // slots past the chunk's end hold a zero record (weight 0, no point)
                const bool live = lane < ns;
                sh.sp[lane] = live ? make_float4((nxt.x - ct[0]) * L.k_scale, (nxt.y - ct[1]) * L.k_scale,
                                                 (nxt.z - ct[2]) * L.k_scale, nxt.w)
                                   : make_float4(0.f, 0.f, 0.f, 0.f);
                sh.sid[lane] = live ? nid : -1;
                wave_sync();
                if (c0 + 64 < tot) fetch(c0 + 64);
                // a group takes sources grp, grp + G, ... of the chunk.  The trip count is the
                // same for every lane (a scalar loop that unrolls); the slots read stay below
                // ns + G <= 128, and a slot past the chunk's end adds exactly 0
                float part = 0.f;
                const int nit = __builtin_amdgcn_readfirstlane((ns + G - 1) / G);
                const float4 *sp = sh.sp + grp;
                const int32_t *sid = sh.sid + grp;
                const int Gs = __builtin_amdgcn_readfirstlane(G);
                if (L.exclude_self) {
#pragma unroll 4
                    for (int it = 0; it < nit; ++it) {
                        const float4 q = sp[it * Gs];
                        const float dx = tx - q.x, dy = ty - q.y, dz = tz - q.z;
                        const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                        const float e = q.w * __builtin_amdgcn_exp2f(-d2);
                        part += sid[it * Gs] == ti ? 0.f : e;
                    }
                } else {
#pragma unroll 4
                    for (int it = 0; it < nit; ++it) {
                        const float4 q = sp[it * Gs];
                        const float dx = tx - q.x, dy = ty - q.y, dz = tz - q.z;
                        const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                        part = fmaf(q.w, __builtin_amdgcn_exp2f(-d2), part);
                    }
                }
                // compensated addition of the chunk partial
                const float y = part - comp;
                const float tt = total + y;
                comp = (tt - total) - y;
                total = tt;
            }
        }
        wave_sync();
        sh.red[lane] = total;
        wave_sync();
        if (grp == 0 && a < nt) {
            float s = 0.f;
            for (int q = 0; q < G; ++q) s += sh.red[q * tp + a];
            L.usort[ti] = L.tflag[ti] ? s : 0.f;
        }
    }
}

}  // namespace
}  // namespace msp
