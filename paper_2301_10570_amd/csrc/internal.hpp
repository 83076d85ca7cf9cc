// Internal declarations shared by the library's translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <memory>
#include <string>
#include <vector>

#include "../../include/mspfmm.h"

namespace msp {

constexpr int kDepth = 21;                    // levels resolved by a 63-bit key
constexpr uint32_t kQMax = (1u << kDepth) - 1;
constexpr int kMaxLevels = kDepth + 2;        // level_offset entries
constexpr int kMaxP = 16;

// Thread-local error text, set by fail().
void set_error(const char *fmt, ...);
int fail(int code, const char *fmt, ...);

#define MSP_HIP(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::msp::fail(MSP_EHIP, "%s failed: %s (%s:%d)", #expr,               \
                               hipGetErrorString(e_), __FILE__, __LINE__);             \
    } while (0)

#define MSP_CHECK_LAUNCH() MSP_HIP(hipGetLastError())

#define MSP_TRY(expr)                \
    do {                             \
        int rc_ = (expr);            \
        if (rc_ != MSP_OK) return rc_; \
    } while (0)

// A grow-only device allocation owned by a handle, or a region of caller memory
// bound to it (fixed: never reallocated or freed; a request beyond its size is
// MSP_ENOSPC).
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    bool fixed = false;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    int ensure(size_t need);
    void release();
    void bind(void *ext, size_t n) {
        release();
        p = ext;
        bytes = n;
        fixed = true;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// Consecutive 256-byte aligned regions of one caller buffer.  With base == NULL it
// only counts, so a size query and the call that uses the buffer share one layout.
struct Carve {
    char *base = nullptr;
    size_t cap = 0, used = 0;
    Carve(void *b, size_t c) : base(static_cast<char *>(b)), cap(c) {}
    void *take(size_t n) {
        used = (used + 255) & ~(size_t)255;
        void *r = base ? base + used : nullptr;
        used += n > 0 ? n : 1;
        return r;
    }
    // bind the next n bytes to b
    void into(DevBuf &b, size_t n) {
        void *r = take(n);
        b.bind(r, n > 0 ? n : 1);
    }
    bool fits() const { return used <= cap; }
};

// Replaces some of a handle's buffers by regions of a caller workspace for the
// length of one call and puts the handle's own buffers back afterwards (nothing
// is allocated or freed).
struct BufSwap {
    static constexpr int kMax = 8;
    DevBuf *buf[kMax];
    void *p[kMax];
    size_t bytes[kMax];
    bool fixed[kMax];
    int n = 0;
    void bind(DevBuf &b, Carve &c, size_t need) {
        buf[n] = &b;
        p[n] = b.p;
        bytes[n] = b.bytes;
        fixed[n] = b.fixed;
        ++n;
        b.p = c.take(need);
        b.bytes = need > 0 ? need : 1;
        b.fixed = true;
    }
    ~BufSwap() {
        for (int k = 0; k < n; ++k) {
            buf[k]->p = p[k];
            buf[k]->bytes = bytes[k];
            buf[k]->fixed = fixed[k];
        }
    }
};

// A grow-only page-locked host allocation owned by a handle (staging of uploads).
struct HostBuf {
    void *p = nullptr;
    size_t bytes = 0;
    HostBuf() = default;
    HostBuf(const HostBuf &) = delete;
    HostBuf &operator=(const HostBuf &) = delete;
    ~HostBuf() { release(); }
    int ensure(size_t need);
    void release();
};

// Parameters that kernels need about the tree's geometry.
struct Geometry {
    double lo[3];
    double side;
    double scale;   // 2^21 / side
    int32_t qmax[3];
};

enum Phase {
    PH_BBOX = 0, PH_KEYS, PH_SORT, PH_LEVELS, PH_NODES, PH_GATHER,
    PH_STAGE, PH_OPS, PH_P2M, PH_M2L_X, PH_M2L_Y, PH_M2L_Z, PH_L2P, PH_LISTS, PH_P2P, PH_SCATTER,
    PH_NODE_MOMENTS, PH_PARTNER, PH_DIRECT, PH_BACKWARD, PH_SORT_HIST, PH_SORT_SCAN, PH_SORT_SCATTER,
    PH_NODE_COUNTS, PH_PARTNER_DIRECT, PH_SORT_RUNS, PH_PARTNER_WAVE, PH_DESC_BOXES, PH_DESC_CHOOSE, PH_DESC_PAIRS, PH_COUNT_
};
static_assert(PH_COUNT_ <= MSP_PHASE_COUNT, "phase table too small");

// Pairs of events recorded around library phases when timing is on.
struct Timing {
    bool on = false;
    bool isolate = false;   // no side streams: overlapping passes run one after another
    struct Rec { int phase; hipEvent_t a, b; };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    double ms[MSP_PHASE_COUNT] = {};
    int64_t launches[MSP_PHASE_COUNT] = {};
    hipEvent_t get();
    void resolve();
    ~Timing();
};

// Records the start of a phase on construction and its end on destruction.
struct PhaseScope {
    Timing *tm;
    hipStream_t s;
    int phase;
    hipEvent_t a = nullptr;
    PhaseScope(Timing *tm_, int ph, hipStream_t s_) : tm(tm_), s(s_), phase(ph) {
        if (tm && tm->on) { a = tm->get(); (void)hipEventRecord(a, s); }
    }
    ~PhaseScope() {
        if (tm && tm->on && a) {
            hipEvent_t b = tm->get();
            (void)hipEventRecord(b, s);
            tm->pending.push_back({phase, a, b});
        }
    }
};

// A stream forked from a caller's stream and joined back to it (default priority),
// created on first use.
struct SideStream {
    hipStream_t stream = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    SideStream() = default;
    SideStream(const SideStream &) = delete;
    SideStream &operator=(const SideStream &) = delete;
    ~SideStream() {
        if (stream) (void)hipStreamDestroy(stream);
        if (fork_ev) (void)hipEventDestroy(fork_ev);
        if (join_ev) (void)hipEventDestroy(join_ev);
    }
    // work enqueued on `stream` from here on follows what `s` holds so far
    int fork(hipStream_t s) {
        if (!stream) {
            MSP_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
            MSP_HIP(hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming));
            MSP_HIP(hipEventCreateWithFlags(&join_ev, hipEventDisableTiming));
        }
        MSP_HIP(hipEventRecord(fork_ev, s));
        MSP_HIP(hipStreamWaitEvent(stream, fork_ev, 0));
        return MSP_OK;
    }
    // work enqueued on `s` from here on follows what `stream` holds so far
    int join(hipStream_t s) {
        MSP_HIP(hipEventRecord(join_ev, stream));
        MSP_HIP(hipStreamWaitEvent(s, join_ev, 0));
        return MSP_OK;
    }
};

}  // namespace msp

struct msp_tree {
    msp::Timing timing;
    int device = -1;
    bool built = false;
    int64_t n = 0;
    int32_t leaf_max = 0, max_depth = 0, depth = 0;
    int64_t n_nodes = 0;
    int64_t level_off[msp::kMaxLevels] = {};
    msp::Geometry geo{};

    // points in key order
    msp::DevBuf keys, perm, iperm, ps;
    bool iperm_valid = false;   // ps: float4 (x, y, z, staged weight) in key order
    bool w_staged = false;      // ps.w holds the weights of the last weight-taking call
    int64_t ps_gen = 0;         // bumped by every write of ps.w
    int64_t src_prefix_gen = -1;   // ps_gen that src_prefix was computed from
    // node table (SoA, int32)
    msp::DevBuf nlevel, nfirst, ncount, nparent, nfchild, nnchild, ndigit, nix, niy, niz;
    msp::DevBuf d_level_off;  // int64[kMaxLevels] on the device

    // build scratch
    msp::DevBuf keys2, perm2, pin, hist, tmp_a, tmp_b, tmp_c, dlev, llev, blkcnt, bbox;

    // per-call staging
    msp::DevBuf tflag, usort;
    msp::DevBuf bwd;   // backward scratch: field values, gradients, Laplacians, reductions
    // expansion grids and translation operators
    msp::DevBuf gridA, gridB, ops;
    bool ops_valid = false;     // M2L operator tables in ops match ops_sig (p, grid, cell / sigma)
    uint64_t ops_sig[5] = {};
    int64_t grid_bytes_valid = 0;
    // direct-route interaction lists (cached per sigma/cutoff)
    msp::DevBuf list_off, list_idx, list_cnt;
    int64_t list_total = 0;
    float list_sigma = -1.f, list_cutoff = -2.f;
    bool counts_valid = false;  // list_cnt / list_off / list_total match list_sigma, list_cutoff
    bool lists_valid = false;   // list_idx holds those lists too
    // node moments for partner queries
    msp::DevBuf nodeA, node_hasA, node_nsrc;
    msp::DevBuf src_prefix;   // sources before each point in key order, then per-tile offsets
    msp::HostBuf build_stage;  // page-locked readback of the build: level offsets, box, flags
    msp::DevBuf partner_qpos; // key-order positions of the last query batch's targets
    msp::DevBuf partner_order; // walk queries by level of the query node (segments), then tallies
    msp::SideStream side;      // the partner walk runs here, beside the direct passes
    // partner descent: frontier, per-pair and per-unit tables, query and task
    // lists, counters (desc_lists, carved), query sums, direct sums; the frontier
    // size after each step is copied to desc_stage (page-locked); kept for the
    // next descent
    msp::DevBuf desc_lists, desc_raw, desc_probs, desc_dv, desc_prefix;
    msp::HostBuf desc_stage;
    // box-pair attractions of a descent: box table, pair lists and values, box
    // moments, axon weights in key order
    msp::DevBuf desc_box, desc_pairs, desc_boxmom, desc_akey;
    int desc_box_level = -1;                  // box level of the last descent (-1: no box pairs)
    int64_t desc_nbox = 0, desc_npair = 0;
    // partner work counters (int64[MSP_WORK_COUNT]) while counting is on
    msp::DevBuf work;
    bool counting = false;
    int node_moments_level = -1, node_moments_p = 0;
    int64_t node_moments_bytes = 0;
};

namespace msp {

// One expansion-route population of a batch, as the batched kernels read it.
struct FgtPop {
    const uint64_t *keys;
    const float4 *ps;
    const int32_t *perm;
    int64_t n;
    const int32_t *nlevel, *nfirst, *ncount, *nnchild;
    int64_t n_nodes;
    const float *w;
    const uint8_t *is_target;
    float *u_out;
    float *rec;          // backward records in key order (batched backward only)
    int subtract_self;
    float *A, *B, *Tmp, *opsx, *opsy, *opsz;
    int level, G[3];
    int band[3];         // largest cell offset per axis whose translation is not negligible
    double lo[3], cell, inv_sigma, step;
    int pop;
};
// Device-side offsets of a batch of expansion-route populations (prefix sums over
// the populations of their operator counts, wavefronts of 64 points, grid floats
// and M2L tiles).
// cells: the occupied grid cells (population, first point, points, cell index),
// small ones from the front (count ncells[0]), large ones from the back (ncells[1]);
// cap entries.
struct FgtBatchPlan {
    const FgtPop *pops;
    int npop, p;
    const int64_t *ops_off, *pw_off, *grid_off, *tile_off[3];
    int64_t n_ops, n_pw, n_grid, n_tiles[3];
    int4 *cells;
    int32_t *ncells;
    int64_t cap;
    unsigned long long *stamps;
    int cus;
    int gemm;          // M2L passes as whole-K GEMM tiles of 32 rows with cell-major grids
                       // (else 32 x 32 tiles on interleaved grids)
    int split;         // the GEMM tiles with split bfloat16 products (p = 8)
    size_t gemm_lds;   // dynamic LDS of the GEMM tiles (largest population)
};

}  // namespace msp

// A batch of independent populations (batch.hip).
struct msp_batch {
    int device = -1;
    int32_t npop = 0;
    int64_t generation = 0;
    std::vector<int64_t> off;
    std::vector<std::unique_ptr<msp_tree>> pops;
    std::vector<int32_t> leaf_max, route;
    // batched direct route
    msp::DevBuf desc, pt_off, item_off, counter, stamps;
    int32_t n_direct = 0;
    int cus = 256;
    int64_t direct_points = 0, direct_items = 0;
    // populations of the direct-route launch; the pair-count query's sum and the
    // state (build generation, tree buffers) the last forward prepared its descriptors on
    std::vector<int32_t> direct_pops;
    msp::DevBuf pair_sum;
    int64_t pair_gen = -1;
    std::vector<uintptr_t> dsig;
    // expansion-route populations: descriptors, offsets, range list, launch plan
    msp::DevBuf fdesc, foff, franges;
    msp::FgtBatchPlan fplan{};
    // branch stream for the expansion-route populations (forked from the caller's stream)
    static constexpr int kBranches = 1;
    hipStream_t side[kBranches] = {};
    hipEvent_t fork = nullptr, join[kBranches] = {};
    // batched backward: its own descriptors, offsets and scratch (target weights gt,
    // block partials of the sigma derivative), and one plan per field (weights w, g)
    msp::DevBuf bw_fdesc, bw_foff, bw_franges, bw_stamps, bw_desc, bw_pt_off, bw_item_off, bw_counter,
        bw_comb, bw_boff, bw_partial, bw_gt;
    msp::FgtBatchPlan bw_plan[2]{};
    int32_t bw_nd = 0;
    int64_t bw_points = 0, bw_items = 0, bw_nblk = 0;
    // branch stream of the backward's expansion-route populations
    hipStream_t bside = nullptr;
    hipEvent_t bfork = nullptr, bjoin = nullptr;
    // graph of the last forward signature, and the populations' state it was captured with
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<unsigned char> key;
    std::vector<uintptr_t> fsig;
    int64_t launches = 0;   // kernel launches issued by the last eager forward
    // graph of the last backward signature
    hipGraph_t bgraph = nullptr;
    hipGraphExec_t bexec = nullptr;
    std::vector<unsigned char> bkey;
    std::vector<uintptr_t> bsig;
    void drop_fwd_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        key.clear();
        fsig.clear();
    }
    void drop_bwd_graph() {
        if (bexec) (void)hipGraphExecDestroy(bexec);
        if (bgraph) (void)hipGraphDestroy(bgraph);
        bexec = nullptr;
        bgraph = nullptr;
        bkey.clear();
        bsig.clear();
    }
    void drop_graph() {
        drop_fwd_graph();
        drop_bwd_graph();
    }
    ~msp_batch() {
        drop_graph();
        if (cap) (void)hipStreamDestroy(cap);
        for (int k = 0; k < kBranches; ++k) {
            if (side[k]) (void)hipStreamDestroy(side[k]);
            if (join[k]) (void)hipEventDestroy(join[k]);
        }
        if (fork) (void)hipEventDestroy(fork);
        if (bside) (void)hipStreamDestroy(bside);
        if (bjoin) (void)hipEventDestroy(bjoin);
        if (bfork) (void)hipEventDestroy(bfork);
    }
};

namespace msp {


// batch.hip
int batch_build(msp_batch *b, const float *x, const float *y, const float *z, const int64_t *offsets,
                int32_t npop, const int32_t *leaf_max, int32_t max_depth, hipStream_t s);
int batch_forward(msp_batch *b, const float *w, const uint8_t *is_target, const float *sigma,
                  const msp_fgt_params *prm, float *u_out, int use_graph, hipStream_t s);
int batch_backward(msp_batch *b, const float *w, const uint8_t *is_target, const float *sigma,
                   const msp_fgt_params *prm, const float *grad_u, float *grad_w, float *grad_x,
                   float *grad_y, float *grad_z, double *grad_sigma, int use_graph, hipStream_t s);
int batch_autotune(msp_batch *b, const float *x, const float *y, const float *z, const int64_t *offsets,
                   int32_t npop, const float *w, const uint8_t *is_target, const float *sigma,
                   const msp_fgt_params *prm, const int32_t *cand, int32_t ncand, int32_t max_depth,
                   float *scratch_u, int32_t *leaf_out, int32_t *route_out, hipStream_t s);
int batch_instance_ms(msp_batch *b, double *ms);
int batch_info(const msp_batch *b, int32_t *npop, int64_t *launches);
int batch_pair_count(msp_batch *b, int64_t *pairs, double *span_ms, hipStream_t s);

// tree.hip
// tree_buf == NULL: handle-owned memory; otherwise the tree's arrays go to tree_buf
// and the build scratch to ws (MSP_ENOSPC when they do not fit)
// w (or NULL): weights carried into key order with the positions (ps.w)
int build_tree(msp_tree *t, const float *x, const float *y, const float *z, int64_t n, int leaf_max,
               int max_depth, hipStream_t s, void *tree_buf = nullptr, size_t tree_bytes = 0,
               void *ws = nullptr, size_t ws_bytes = 0, const float *w = nullptr);
// upper bound on the node count of a tree over n points
int64_t tree_node_bound(int64_t n, int leaf_max, int max_depth);
// caller buffer sizes of msp_octree_build_ws
void build_query_bytes(int64_t n, int leaf_max, int max_depth, size_t *tree_bytes, size_t *ws_bytes);

// fgt.hip
struct FgtPlan {
    int route;
    int level;
    int p;
    int G[3];
    double rho;
    double cell;      // cell side at `level`
    double fgt_cost, direct_cost;
    int pf;           // > 0: terms at the sub-cells two levels down (two-level variant)
};

// fgt.hip: grid buffers of a population (allocated here) and the batched forward
int fgt_pop_prepare(msp_tree *t, const FgtPlan &pl, const msp_fgt_params *prm, FgtPop *out);
int64_t fgt_pop_tiles(const FgtPop &f, int p, int pass, bool gemm);
size_t fgt_pop_gemm_lds(const FgtPop &f, int p, bool split = false);
int fgt_batch_forward(const FgtBatchPlan &bp, hipStream_t s);
// value, gradient and (want_lap) Laplacian of every population's field at all its
// points, into f.rec + i * stride + slot (key order i)
int fgt_batch_field_grad(const FgtBatchPlan &bp, int stride, int slot, int want_lap, hipStream_t s);
int plan_fgt(const msp_tree *t, const msp_fgt_params *prm, FgtPlan *plan);
// bytes of one expansion grid, and of the buffer holding a third grid and the
// operator tables
void fgt_grid_bytes(const FgtPlan &pl, size_t *grid, size_t *ops);
double rho_max_for_p(int p);
int stage_inputs(msp_tree *t, const float *w, const uint8_t *is_target, hipStream_t s);
int fgt_forward_grid(msp_tree *t, const FgtPlan &plan, const msp_fgt_params *prm, const float *w,
                     const uint8_t *is_target, float *u_out, hipStream_t s);
int ensure_iperm(msp_tree *t, hipStream_t s);
// Value, gradient (x, y, z) and, with want_lap, Laplacian of the field of weights w
// at every point, in key order: point i writes out[i * stride + 0 .. 4].
int fgt_field_grad(msp_tree *t, const FgtPlan &pl, const msp_fgt_params *prm, const float *w,
                   float *out, int stride, int want_lap, hipStream_t s);
int direct_field_grad(msp_tree *t, const msp_fgt_params *prm, float *out, int stride, int want_lap,
                      hipStream_t s);
int fgt_backward(msp_tree *t, const float *w, const uint8_t *is_target, const msp_fgt_params *prm,
                 const float *grad_u, float *grad_w, float *grad_x, float *grad_y, float *grad_z,
                 double *grad_sigma, hipStream_t s);
int scatter_output(msp_tree *t, float *u_out, uint32_t flags, bool subtract_self, hipStream_t s);

// p2p.hip
// lists_ready: t->list_idx already holds the lists of prm (else they are built or
// taken from the handle's cache)
int direct_route(msp_tree *t, const msp_fgt_params *prm, hipStream_t s, bool lists_ready = false);
int direct_route_lists(msp_tree *t, const msp_fgt_params *prm, hipStream_t s);
// per-leaf list lengths and offsets for prm's sigma and cutoff (one host
// synchronisation when they change), and the list entries into t->list_idx
int direct_route_counts(msp_tree *t, const msp_fgt_params *prm, hipStream_t s);
int direct_route_fill(msp_tree *t, const msp_fgt_params *prm, hipStream_t s);
int direct_all_pairs(const float *tx, const float *ty, const float *tz, int64_t nt, const float *sx,
                     const float *sy, const float *sz, const float *w, int64_t ns, float sigma,
                     float *u, hipStream_t s);

// partner.hip
int partner_probabilities(msp_tree *t, const float *w, const msp_fgt_params *prm,
                          const int32_t *target_idx, const int32_t *node_id, int64_t nq,
                          const float *uniforms, float *probs, int32_t *choice, hipStream_t s);
// stage the weights and node moments once; then any number of query batches with
// the unnormalised per-octant sums (raw: double[nq * 8]); qpos: key-order positions
// of the targets, or NULL to look them up; nq_dev (or NULL): the number of queries
// in device memory, at most nq (the arrays' size)
int partner_prepare(msp_tree *t, const float *w, const msp_fgt_params *prm, hipStream_t s);
// the sources (records with w != 0) before each key-order position, from ps.w
int source_prefix(msp_tree *t, hipStream_t s);
int partner_query_raw(msp_tree *t, const msp_fgt_params *prm, const int32_t *target_idx,
                      const int32_t *node_id, int64_t nq, float *probs, double *raw, const int32_t *qpos,
                      hipStream_t s, const int64_t *nq_dev = nullptr);

// api.hip: msp_fgt_forward with every per-call buffer in the workspace ws (checked
// against the call's need, MSP_ENOSPC if short), and that need in bytes
int forward_in_workspace(msp_tree *t, const float *w, const uint8_t *is_target, const msp_fgt_params *prm,
                         float *u_out, void *ws, size_t ws_bytes, hipStream_t s);
int forward_workspace_bytes(msp_tree *t, const msp_fgt_params *prm, size_t *bytes, hipStream_t s);

// descent.hip
int descent_step(msp_tree *t, const float *w, const float *a, const msp_fgt_params *prm, uint64_t seed,
                 int32_t step, const int64_t *S_in, const int64_t *T_in, int64_t m, int64_t *S_out,
                 int64_t *T_out, int64_t cap, int64_t *m_out, int32_t *req_axon, int32_t *req_dendrite,
                 int64_t req_cap, int64_t *n_req, hipStream_t s);
int partner_descent(msp_tree *t, const float *w, const float *a, const msp_fgt_params *prm, uint64_t seed,
                    int32_t *req_axon, int32_t *req_dendrite, uint8_t *accepted, int64_t *n_req,
                    int32_t *n_steps, hipStream_t s);

// helpers
inline unsigned grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace msp

// ---------------------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------------------
namespace msp {

// Spread the low 21 bits of v so that bit b lands at bit 3b.
__host__ __device__ inline uint64_t spread3(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

// Inverse of spread3: gather every third bit starting at bit 0.
__host__ __device__ inline uint32_t compact3(uint64_t v) {
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
    v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
    v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
    v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
    v = (v ^ (v >> 32)) & 0x1fffffull;
    return (uint32_t)v;
}

// q = min(floor((x - lo) * scale), 2^21 - 1) in float64: a subtraction, then a
// multiplication, each rounded once (no contraction is possible in this form).
// The root cube from the bounding box (min x, y, z, max x, y, z): lower corner,
// side (the largest extent, 1 for a single point) and the 21-bit quantisation
// scale.  Host and device compute it alike, so keys and geometry agree.
__host__ __device__ inline void root_cube(const float *box, double lo[3], double &side, double &scale) {
    side = 0.0;
    for (int k = 0; k < 3; ++k) {
        lo[k] = (double)box[k];
        const double ext = (double)box[3 + k] - lo[k];
        if (ext > side) side = ext;
    }
    if (side == 0.0) side = 1.0;
    scale = 2097152.0 / side;
}

__device__ inline uint32_t quantise(float v, double lo, double scale) {
    double q = floor(((double)v - lo) * scale);
    return q >= (double)kQMax ? kQMax : (uint32_t)q;
}

__host__ __device__ inline uint64_t morton3(uint32_t qx, uint32_t qy, uint32_t qz) {
    return (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
}

// First index in [lo, hi) with keys[idx] >= v.
// Orders one wavefront's LDS accesses at this point.  A wavefront executes in lock
// step and its LDS operations complete in order, so LDS data private to one wave
// needs no workgroup barrier; this keeps the compiler from moving accesses across.
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int64_t lower_bound_u64(const uint64_t *keys, int64_t lo, int64_t hi, uint64_t v) {
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if (keys[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// First index in [lo, hi) with a[idx] >= v (int32 array).
__device__ inline int64_t lower_bound_i32(const int32_t *a, int64_t lo, int64_t hi, int32_t v) {
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// First index in [lo, hi) with a[idx] > v (int32 array).
__device__ inline int64_t upper_bound_i32(const int32_t *a, int64_t lo, int64_t hi, int32_t v) {
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] <= v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

}  // namespace msp
