/*
 * mspfmm: Gaussian attraction sums of the Model of Structural Plasticity on one
 * AMD Instinct MI355X (gfx950), evaluated by an octree fast Gauss transform.
 *
 * The quantity is the n-body sum of the paper's section "Mathematical
 * Formulation of the Fast Multipole Method" (Eq. (2)) with the Gaussian kernel
 * of the direct evaluation in the algorithm section (Eq. (8)):
 *
 *     u(t_i) = sum_j w_j exp(-|t_i - s_j|^2 / sigma^2)
 *
 * t_i runs over targets (neurons with vacant axons), s_j over sources (neurons
 * with vacant dendrites, w_j = number of vacant dendrites).  One point set holds
 * both roles: a neuron is a target if its is_target flag is set and a source
 * if its weight is non-zero.  The per-neuron attraction is a_i * u(t_i) with a_i
 * the number of vacant axons; forming that product is left to the caller.
 *
 * Conventions for every entry point
 *   - Array arguments are DEVICE pointers on the current HIP device unless a
 *     comment says "host".  The caller owns them; the library never frees or
 *     retains them beyond the call.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work
 *     is enqueued on it.  Calls return before the GPU finishes except where a
 *     comment says the call synchronises the stream.
 *   - Internal device memory (sorted copies, node table, expansion grids,
 *     interaction lists) belongs to the msp_tree handle: allocated on demand,
 *     reused by later calls, released by msp_tree_destroy.  A handle must not be
 *     used from two host threads at once, and two calls on one handle must use
 *     the same stream (or be ordered by the caller).  One exception: after a
 *     weighted build (msp_octree_build_weighted), msp_fgt_forward on the
 *     expansion route (MSP_ROUTE_FGT, or AUTO resolving to it) and
 *     msp_partner_probabilities, both with MSP_WEIGHTS_STAGED, only read the
 *     tree and write disjoint buffers, so they may run on two streams at once;
 *     both must be ordered after the build, and the next call that writes the
 *     tree (a build, a backward, a call without MSP_WEIGHTS_STAGED) after both.
 *   - Callers that own all device memory use the *_query / *_ws pairs instead:
 *     msp_octree_build_ws keeps the tree's arrays in a caller buffer and builds
 *     in a caller workspace, msp_fgt_forward_ws evaluates in a caller workspace;
 *     neither allocates device memory.
 *   - Return value: MSP_OK (0) or a negative MSP_E* code; msp_last_error()
 *     then gives a human-readable reason (thread-local).  No C++ exception
 *     crosses this interface.
 *   - Positions are float32 micrometres (any unit works if sigma uses it).
 *     Indices are int32, so n < 2^31.
 */
#ifndef MSPFMM_H
#define MSPFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum msp_status {
    MSP_OK = 0,
    MSP_EINVAL = -1,    /* bad argument: NULL pointer, size, sigma, p, flags, non-finite position */
    MSP_ENOSPC = -2,    /* a required buffer would exceed the library's size limits, or a
                           caller-supplied buffer is too small */
    MSP_EOVERFLOW = -3, /* more than 2^31-1 points or nodes */
    MSP_EHIP = -4,      /* HIP runtime error (allocation, launch, copy) */
    MSP_ENOTSUP = -5,   /* unsupported device or option combination */
    MSP_ESTATE = -6     /* handle not ready (e.g. no tree built yet) */
};

enum msp_route {
    MSP_ROUTE_AUTO = 0,   /* pick by a cost model (see msp_fgt_info.route) */
    MSP_ROUTE_FGT = 1,    /* expansions on one level of the octree (P2M, M2L, L2P) */
    MSP_ROUTE_DIRECT = 2  /* near-field pairs only: leaf interaction lists + P2P */
};

enum msp_flags {
    /* Skip the pair j == i (a neuron does not attract its own axons).  The direct
     * route skips the pair exactly; the expansion route subtracts w_i after the
     * fact, which loses relative accuracy when u_i is close to w_i. */
    MSP_EXCLUDE_SELF = 1u << 0,
    /* Run the Hermite-to-Taylor translation on the vector ALUs instead of the
     * matrix cores (same result up to float32 rounding; for cross-checks). */
    MSP_M2L_VALU = 1u << 1,
    /* Two-level variant of the expansion route: P2M and L2P at the 4x4x4
     * sub-cells two levels below the expansion level with fewer terms, joined to
     * it by M2M and L2L shifts (used when p is 6..8 and cells hold >= 512 points;
     * msp_fgt_info.fine_terms reports it). */
    MSP_TWO_LEVEL = 1u << 2,
    /* Run the Hermite-to-Taylor translation as split bfloat16 products on the
     * matrix cores: every float32 operand x becomes hi = bf16(x) plus
     * lo = bf16(x - hi), and hi*hi + hi*lo + lo*hi is accumulated in float32
     * (about 2^-16 of each product is lost).  Exclusive with MSP_M2L_VALU. */
    MSP_M2L_BF16X3 = 1u << 3,
    /* For msp_fgt_forward (and its _ws / _noalloc forms) and
     * msp_partner_probabilities: `w` equals the weights the tree already holds in
     * key order, from msp_octree_build_weighted or from the last msp_fgt_forward
     * (on the direct route, or with MSP_STAGE_WEIGHTS), msp_partner_probabilities
     * or msp_partner_descent call on this tree (an MSP step evaluates the sums and
     * then the partner probabilities with the same vacant element counts).  Those
     * weights are used instead of gathering `w` through the permutation again (the
     * expansion route still reads `w` in input order for MSP_EXCLUDE_SELF).
     * MSP_ESTATE if the tree holds no such weights (none staged since the build,
     * or a backward call since, which stages other weights); the contents of `w`
     * are not checked. */
    MSP_WEIGHTS_STAGED = 1u << 4,
    /* For msp_fgt_forward on the expansion route: keep the weights its P2M
     * gathers into key order for a following MSP_WEIGHTS_STAGED call (the extra
     * writes cost a little; a forward on its own does without). */
    MSP_STAGE_WEIGHTS = 1u << 5
};

typedef struct msp_tree msp_tree; /* opaque handle */

/* Geometry and shape of a built tree (host struct, filled by msp_tree_get_info). */
typedef struct msp_tree_info {
    int64_t n;              /* points */
    int64_t n_nodes;        /* nodes, breadth-first: by level, then Morton order */
    int32_t depth;          /* deepest level that holds a node */
    int32_t leaf_max;
    int32_t max_depth;
    int32_t qmax[3];        /* largest quantised coordinate per axis (0 .. 2^21-1) */
    double lo[3];           /* lower corner of the root cube (min over points) */
    double side;            /* side of the root cube (max extent over axes; 1 if 0) */
    int64_t level_offset[23]; /* first node of each level; entries past depth+1 equal n_nodes */
} msp_tree_info;

/* Device destinations for msp_tree_export; any member may be NULL (skipped).
 * Node arrays have n_nodes entries, point arrays n entries. */
typedef struct msp_tree_arrays {
    uint64_t *keys;          /* sorted 63-bit Morton keys */
    int32_t *perm;           /* perm[k] = input index of the k-th point in key order */
    int32_t *node_level;
    int32_t *node_first;     /* first point (key order) */
    int32_t *node_count;     /* number of points */
    int32_t *node_parent;    /* -1 for the root */
    int32_t *node_first_child; /* -1 for a leaf; children are contiguous */
    int32_t *node_n_children;
    int32_t *node_digit;     /* octant inside the parent: (x<<2)|(y<<1)|z of the next bit */
    int32_t *node_ix, *node_iy, *node_iz; /* lattice coordinates at the node's level */
} msp_tree_arrays;

typedef struct msp_fgt_params {
    int32_t p;            /* expansion terms per axis, 1..16 (p^3 coefficients per box) */
    int32_t level;        /* octree level whose cells carry expansions; -1 = choose from p, sigma, side */
    float sigma;          /* kernel width, > 0 and finite */
    float cutoff_sigmas;  /* direct route: sources farther than cutoff_sigmas*sigma from a target
                             leaf's box are dropped; <= 0 means no cutoff */
    int32_t route;        /* enum msp_route */
    uint32_t flags;       /* enum msp_flags */
} msp_fgt_params;

/* What a forward call will do for given params (host struct). */
typedef struct msp_fgt_info {
    int32_t route;        /* MSP_ROUTE_FGT or MSP_ROUTE_DIRECT after resolving AUTO */
    int32_t level;        /* expansion level (FGT route) */
    int32_t grid[3];      /* cells per axis on that level (bounding box of occupied cells) */
    int32_t p;
    double rho;           /* cell half-side / sigma on that level */
    double fgt_cost;      /* cost-model estimates (arbitrary units, same scale) */
    double direct_cost;
    int32_t fine_terms;   /* > 0: P2M and L2P run at the sub-cells two levels below `level`
                             with this many terms per axis, joined to `level` by M2M and L2L */
} msp_fgt_info;

/* Status text for a code (static string). */
const char *msp_status_string(int status);
/* Reason for the last failure on this host thread (empty if none). */
const char *msp_last_error(void);

/* Create / destroy a handle.  Destroy synchronises the device before freeing. */
int msp_tree_create(msp_tree **out);
void msp_tree_destroy(msp_tree *t);

/* Build the adaptive octree of the points (section "A Distributed Octree": a cell
 * is split into its non-empty octants while it holds more than leaf_max points
 * and its level is below max_depth).  Root cube: lower corner = per-axis minimum,
 * side = largest per-axis extent.  Each coordinate is quantised to 21 bits as
 * min(floor((x - lo) * (2^21 / side)), 2^21 - 1) in float64 and the three are
 * interleaved (x highest within each 3-bit digit) into a 63-bit key; points are
 * stably sorted by key.  x, y, z: device float32[n], input order.  leaf_max >= 1,
 * 0 <= max_depth <= 21, 0 <= n < 2^31.  Synchronises `stream` once: the level
 * offsets, the root cube and the input checks come back in one page-locked
 * readback (a second build pass, with its own readback, runs only when more
 * points than the run sort takes share one 24-bit key prefix).  MSP_EINVAL for a
 * non-finite coordinate.  Replaces any tree held by the handle. */
int msp_octree_build(msp_tree *t, const float *x, const float *y, const float *z, int64_t n,
                     int32_t leaf_max, int32_t max_depth, void *stream);

/* msp_octree_build, with the weights w (device float32[n], input order) carried
 * into key order beside the positions by the same passes (one more coalesced
 * 4-byte read per point), so that a following msp_fgt_forward or
 * msp_partner_probabilities with MSP_WEIGHTS_STAGED and the same w needs no
 * gather of the weights through the permutation: the MSP step when positions and
 * vacant element counts both changed since the last one. */
int msp_octree_build_weighted(msp_tree *t, const float *x, const float *y, const float *z, const float *w,
                              int64_t n, int32_t leaf_max, int32_t max_depth, void *stream);

/* Sizes (host outputs, bytes) of the caller buffers of msp_octree_build_ws for n
 * points: tree_bytes for the arrays the tree keeps (sorted keys, permutation,
 * packed positions in key and in input order, inverse permutation, level offsets,
 * node table and the direct route's per-leaf list lengths), sized for the largest
 * node count such a tree can have (1 + the sum over levels l >= 1 of
 * min(8^l, n, 8 floor(n / (leaf_max + 1))): every node below the root has a parent
 * with more than leaf_max points, and the nodes of one level are disjoint);
 * ws_bytes for the build's scratch (sort buffers, per-point levels, block
 * counts).  Argument rules as msp_octree_build.  No device work. */
int msp_octree_build_query(int64_t n, int32_t leaf_max, int32_t max_depth, size_t *tree_bytes,
                           size_t *ws_bytes);

/* msp_octree_build with caller-owned device memory: the tree's arrays are placed
 * in tree_buf, which the tree uses until it is rebuilt or destroyed (the caller
 * keeps it alive and unmodified meanwhile), and the build's scratch in ws, which
 * the caller may reuse for work enqueued on `stream` after this call.  Both are
 * device pointers aligned to 256 bytes.  tree_bytes may be smaller than the
 * query's bound: MSP_ENOSPC (the message names the bytes needed) only if the tree
 * actually built does not fit; ws_bytes must reach the query's figure.  Device
 * memory that the handle owned from an earlier build is released.  The other
 * entry points use a tree built this way like any other (those that need more
 * memory than the tree still allocate it in the handle).  Synchronises `stream`
 * as msp_octree_build. */
int msp_octree_build_ws(msp_tree *t, const float *x, const float *y, const float *z, int64_t n,
                        int32_t leaf_max, int32_t max_depth, void *tree_buf, size_t tree_bytes, void *ws,
                        size_t ws_bytes, void *stream);

/* Host copy of the tree's geometry and shape. */
int msp_tree_get_info(const msp_tree *t, msp_tree_info *info);

/* Copy the sorted keys, permutation and node table into caller buffers (device). */
int msp_tree_export(const msp_tree *t, const msp_tree_arrays *dst, void *stream);

/* Resolve route and level for params without running anything. */
int msp_fgt_plan(msp_tree *t, const msp_fgt_params *prm, msp_fgt_info *info);

/* u_out[i] = u(t_i) for every point i with is_target[i] != 0, and 0 for the others.
 * w: device float32[n] source weights (0 = not a source; any finite value works,
 * the sum is linear in w).  is_target: device uint8[n], or NULL for all points.
 * u_out: device float32[n].  All in input order.
 * FGT route: moments (Eq. (7)) of the sources in every cell of one octree level,
 * Hermite-to-Taylor translation between every pair of cells of that level (the
 * transform the paper's Eqs. (6)-(7) combine), and evaluation of each cell's
 * Taylor series (Eq. (6)) at its targets.  With MSP_TWO_LEVEL, moments and
 * evaluation move to the sub-cells two levels down with fewer terms, joined to
 * the expansion level by M2M and L2L shifts (msp_fgt_info.fine_terms).  Direct route: Eq. (8) summed over all
 * source leaves within the cutoff of each target leaf.  The direct route
 * synchronises `stream` once when its interaction lists are (re)built. */
int msp_fgt_forward(msp_tree *t, const float *w, const uint8_t *is_target,
                    const msp_fgt_params *prm, float *u_out, void *stream);

/* Bytes of the workspace that msp_fgt_forward_ws needs for this tree and params
 * (host output): on the expansion route two expansion grids (cells * p^3 floats
 * each) and a third with the per-axis translation tables; on the direct
 * route per-point target flags and key-order sums and the leaf interaction lists.
 * The direct route's list lengths are counted on the device first when sigma or
 * the cutoff changed since they were last counted (this synchronises `stream`). */
int msp_fgt_forward_query(msp_tree *t, const msp_fgt_params *prm, size_t *ws_bytes, void *stream);

/* msp_fgt_forward with every per-call buffer in the caller's workspace ws (device,
 * 256-byte aligned, ws_bytes >= the query's figure, else MSP_ENOSPC).  Allocates
 * no device memory.  The result has the bits of msp_fgt_forward with the same
 * arguments.  The workspace holds nothing between calls: the translation tables
 * and the direct route's lists are rebuilt in it on every call, and the debug
 * buffers of msp_fgt_debug_buffer are not kept.  The direct route synchronises
 * `stream` as msp_fgt_forward_query does when the list lengths must be
 * recounted. */
int msp_fgt_forward_ws(msp_tree *t, const float *w, const uint8_t *is_target, const msp_fgt_params *prm,
                       float *u_out, void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory at all (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): msp_fgt_forward
 * with its per-call buffers in a fixed 64 MiB device array that the library holds
 * on every device it runs a call on, from the first such call until the process
 * ends (no workspace argument, no allocation).  Same arguments and the same bits
 * as msp_fgt_forward; the tree must live on the current device.  MSP_ENOSPC when
 * the call needs more than 64 MiB (msp_fgt_forward_query gives the need).  Calls
 * on one device share that array: calls that overlap in time on one device (other
 * streams, other host threads) race and must be ordered by the caller.  The array
 * holds nothing between calls (tables and lists are rebuilt on every call).  The
 * direct route synchronises `stream` when its list lengths must be recounted
 * (new sigma or cutoff on this tree): call msp_fgt_forward_query first, outside
 * any capture. */
int msp_fgt_forward_noalloc(msp_tree *t, const float *w, const uint8_t *is_target, const msp_fgt_params *prm,
                            float *u_out, void *stream);
/* Derivatives of L = sum_i g_i u(t_i) over the targets i (the adjoint of
 * msp_fgt_forward with the same w, is_target and params).  With
 * K = exp(-|t - s|^2/sigma^2) and v(x) = sum_i g_i K(t_i, x) (the transposed sum,
 * computed by the same route with weights g at the targets):
 *   grad_w[j]          = v(x_j)                       (for every point, w_j = 0 included)
 *   grad_{x,y,z}[k]    = g_k grad u(x_k) + w_k grad v(x_k)
 *   grad_sigma[0]      = sum_i g_i ((sigma/2) lap u(t_i) + (3/sigma) u(t_i))
 * The sigma form is the heat equation of the Gaussian, dK/dsigma =
 * (sigma/2) lap K + (3/sigma) K, applied to the local expansions or the direct
 * sums.  grad_u: device float32[n] (entries of non-targets are ignored).
 * grad_w, grad_x, grad_y, grad_z: device float32[n] or NULL (all three position
 * arrays or none); grad_sigma: device float64[1] or NULL.  Input order throughout.
 * With MSP_EXCLUDE_SELF the self pair drops out of grad_w (it adds nothing to the
 * other derivatives). */
int msp_fgt_backward(msp_tree *t, const float *w, const uint8_t *is_target,
                     const msp_fgt_params *prm, const float *grad_u, float *grad_w, float *grad_x,
                     float *grad_y, float *grad_z, double *grad_sigma, void *stream);

/* All-pairs direct sum on the GPU, Eq. (8), no tree and no cutoff (the baseline
 * that the transform is measured against).  Targets tx,ty,tz: device float32[nt];
 * sources sx,sy,sz,w: device float32[ns]; u: device float32[nt].  The sum over
 * sources is accumulated in float32 per tile of 1024 sources with compensated
 * addition of the tile sums. */
int msp_direct_sum(const float *tx, const float *ty, const float *tz, int64_t nt, const float *sx,
                   const float *sy, const float *sz, const float *w, int64_t ns, float sigma,
                   float *u, void *stream);

/* Child probabilities for proportional partner choice (Algorithm 2).  For query q
 * (target point target_idx[q], an input index, and tree node node_id[q]) the
 * attraction of child c of that node is S_c = sum_{j below c} w_j K(t, s_j), and
 * probs[8*q + octant(c)] = S_c / sum_c' S_c' (0 for absent children).  Weights
 * are expected to be >= 0 (they are counts of free elements); with negative
 * weights the result is unspecified.  The children are walked nearest first.  A
 * node holding more than 70 sources (Algorithm 2's threshold) carries Hermite
 * moments (Eq. (7)) and is evaluated from them (Eq. (8)) when the truncation
 * model of `prm->p` puts the error below 1e-5 of the node's smallest term or
 * below 1e-7 of the query's running total; it is dropped when even all of its
 * weight at its nearest point stays below 1e-12 of the running total.  All other
 * sources are summed directly: for nodes of at most 16384 points each term in
 * float32 relative to the node's closest approach to the target (float64 when the
 * node is so wide that a term could fall below exp(-60) of the largest possible
 * one), in float64 during the walk of larger nodes; the sums in float64.  If `uniforms`
 * (device float32[nq] in [0,1)) is non-NULL, choice[q] receives the node id of
 * the first child, in octant order, whose running sum of S exceeds
 * uniforms[q] * total, or -1 when the total is 0 or the node is a leaf.
 * prm->flags & MSP_EXCLUDE_SELF skips the query's own point.  probs: device
 * float32[8*nq]; choice: device int32[nq] or NULL. */
int msp_partner_probabilities(msp_tree *t, const float *w, const msp_fgt_params *prm,
                              const int32_t *target_idx, const int32_t *node_id, int64_t nq,
                              const float *uniforms, float *probs, int32_t *choice, void *stream);

/* Partner descent: Algorithm 1 over pairs of (axon item, dendrite item), driven by
 * the proportional choice of Algorithm 2, then the acceptance of the requests at
 * the dendrites.  Items: a tree node v (v >= 0) or one neuron with input index i,
 * encoded -(i + 1).  A neuron is the paper's leaf; the children of an inner node
 * are its child nodes in octant order, those of a leaf node its neurons in key
 * order.  Every choice compares Att(S, C) = sum_{i in S} sum_{j in C, j != i}
 * a_i w_j exp(-|t_i - s_j|^2 / sigma^2) over the candidates C:
 *   S, T neurons       request S -> T
 *   S neuron, T node   choose a child C of T by Att(S, C)
 *   S node, T neuron   choose a child S' of S by Att(S', T); the other children drop out
 *   S, T nodes         each child S_c of S holding axons chooses a child C of T by Att(S_c, C)
 * A choice takes the first candidate whose running sum exceeds r times the total,
 * r = (mix(mix(seed ^ ((step + 1) * 0x9E3779B97F4A7C15)) ^ item) >> 11) * 2^-53 with
 * mix the SplitMix64 output for a state and item the choosing item (two's
 * complement); all-zero values drop the pair.  Att over the children of an inner
 * node: while both nodes of the pair lie above the box level (one below the
 * coarsest level whose half side is within rho_max(p) sigma, the level the
 * expansion route picks), the sum of box-pair attractions over the boxes of S_c
 * and of C (boxes: the nodes at or below the box level whose parent lies above
 * it, and the leaves above it).  A box pair is summed directly (each term in
 * float32 relative to the two boxes' closest approach, to about 1e-5; float64
 * sums) or,
 * when both boxes lie at or below the box level, hold more than 70 axons /
 * dendrites (Algorithm 2's c2 / c1) and their centres are within 2.5 sigma, taken
 * from the dendrite box's Hermite moments (Eq. (7)) translated to a Taylor
 * series at the axon box (Eq. (6)) and contracted with the axon box's power
 * sums; with a cutoff, box pairs whose boxes lie farther apart than
 * cutoff_sigmas * sigma are left out.  For p > 10, or without a cutoff when the
 * axon boxes times the dendrite boxes exceed 2^22, and below the box level, Att
 * is accumulated per axon neuron from partner queries (the accuracy contract of
 * msp_partner_probabilities, prm->cutoff_sigmas applies); over neurons it is
 * summed directly in float64.  w: vacant dendritic elements, a: vacant axonal
 * elements, both device float32[n] in input order (>= 0).  prm: sigma, p and
 * cutoff; self pairs are always skipped.  The frontier stays in device memory and
 * every step runs in kernels; the call synchronises `stream` while it sets up
 * (tree topology, box pairs) and at the end, and waits for step k - 2 before it
 * launches step k. */

/* One step of msp_partner_descent from the frontier (S_in[k], T_in[k]), k < m
 * (host arrays, copied to the device): the next frontier goes to S_out/T_out
 * (host int64[cap]; *m_out pairs, dropped pairs left out), the requests to
 * req_axon / req_dendrite (host int32[req_cap], input indices; *n_req).
 * MSP_ENOSPC when a capacity is exceeded (the counts are still set). */
int msp_descent_step(msp_tree *t, const float *w, const float *a, const msp_fgt_params *prm, uint64_t seed,
                     int32_t step, const int64_t *S_in, const int64_t *T_in, int64_t m, int64_t *S_out,
                     int64_t *T_out, int64_t cap, int64_t *m_out, int32_t *req_axon, int32_t *req_dendrite,
                     int64_t req_cap, int64_t *n_req, void *stream);

/* The whole descent from (root, root) until the frontier is empty (steps numbered
 * from 0), then acceptance: dendrite neuron j takes at most floor(w_j) requests,
 * those with the smallest priority mix(mix(seed ^ 0xD1B54A32D192ED03) ^ i) of the
 * axon's input index i, ties by i.  req_axon, req_dendrite: device int32[n]
 * (input indices; at most one request per neuron with axons); accepted: device
 * uint8[n]; *n_req, *n_steps: host. */
int msp_partner_descent(msp_tree *t, const float *w, const float *a, const msp_fgt_params *prm, uint64_t seed,
                        int32_t *req_axon, int32_t *req_dendrite, uint8_t *accepted, int64_t *n_req,
                        int32_t *n_steps, void *stream);

/* Copy an internal buffer, for pass-level checks.
 *   which 0: Hermite moment grid after P2M of the last expansion-route forward call
 *   which 1: Taylor grid after M2L of that call
 *     layout of both: float32 [kz][az][ky][ay][kx][ax], with (kx,ky,kz) the cell's
 *     lattice coordinates inside the grid reported by msp_fgt_plan and (ax,ay,az)
 *     the coefficient multi-index (p values each);
 *   which 2: node moments of the last partner call, float32 [node - first][az][ay][ax]
 *     for the nodes from the first node of the moment level on (entries of nodes
 *     without moments are unspecified);
 *   which 3: per-node flag of that call (uint8 [n_nodes], 1 = node carries moments);
 *   which 4: box-pair attractions Att(s, c) of the last msp_partner_descent or
 *     msp_descent_step call, float64 [npair], pairs grouped by axon box in key order;
 *   which 5, 6: the axon box and the dendrite box of each pair (int32 [npair], box indices);
 *   which 7: the tree node of each box (int32 [nbox], boxes in key order);
 *     4..7 give MSP_ESTATE when that call used no box pairs;
 *   which 8: the points in key order as the last call left them, float32 [n][4]
 *     (x, y, z, staged weight; the weight slot is unspecified before any call that
 *     stages weights);
 *   which 9: the inverse permutation (int32 [n], input index -> key-order position),
 *     computed on `stream` first if the build did not leave it.
 * *bytes receives the buffer size; if dst (device) is non-NULL and dst_bytes >= *bytes
 * the buffer is copied there on `stream`, otherwise MSP_EINVAL (dst too small). */
int msp_fgt_debug_buffer(msp_tree *t, int32_t which, void *dst, size_t dst_bytes, size_t *bytes,
                         void *stream);

/* ---------------------------------------------------------------------------
 * Batches of independent populations (many uneven-size networks, each with its
 * own sigma).  The caller concatenates the populations: population k owns the
 * indices offsets[k] .. offsets[k+1]-1 of every per-point array (x, y, z, w,
 * is_target, u_out, gradients).  Every population gets its own octree; the
 * kernels of a forward call cover all of them: populations on the expansion
 * route run their own short sequence, and all populations on the direct route
 * share one persistent launch that takes (population, node) work items from a
 * device counter.  The first forward call with a given argument set runs
 * eagerly and captures the sequence into a hipGraph; later calls with the same
 * pointers, sigmas and parameters replay it on `stream`.  Calls on one batch
 * must not overlap (they share the work counter and scratch).
 * ------------------------------------------------------------------------- */
typedef struct msp_batch msp_batch; /* opaque handle */

int msp_batch_create(msp_batch **out);
void msp_batch_destroy(msp_batch *b);

/* Build the octrees.  offsets: host int64[npop + 1], offsets[0] = 0, non-decreasing;
 * leaf_max: host int32[npop] or NULL (64 for all); max_depth as msp_octree_build.
 * Synchronises `stream`.  Invalidates a captured graph. */
int msp_batch_build(msp_batch *b, const float *x, const float *y, const float *z, const int64_t *offsets,
                    int32_t npop, const int32_t *leaf_max, int32_t max_depth, void *stream);

/* Autotuner: for every population, build its tree at each candidate leaf size
 * (host int32[ncand]), time three forward calls on each route whose grid fits,
 * keep the fastest (leaf size, route) pair, and build the batch with the choices
 * (later forward calls with prm->route == MSP_ROUTE_AUTO use the chosen routes).
 * scratch_u: device float32[offsets[npop]] written during the trials.  leaf_out,
 * route_out: host int32[npop] or NULL.  Synchronises `stream`. */
int msp_batch_autotune(msp_batch *b, const float *x, const float *y, const float *z,
                       const int64_t *offsets, int32_t npop, const float *w, const uint8_t *is_target,
                       const float *sigma, const msp_fgt_params *prm, const int32_t *cand, int32_t ncand,
                       int32_t max_depth, float *scratch_u, int32_t *leaf_out, int32_t *route_out,
                       void *stream);

/* Forward of every population (as msp_fgt_forward on its slice).  sigma: host
 * float32[npop] (prm->sigma is ignored); the other fields of prm apply to all.
 * use_graph = 0 runs eagerly every time.  The batched translation runs on the
 * matrix cores on one level, in fp32 or (MSP_M2L_BF16X3, p = 8 only) as split
 * bfloat16 products; MSP_M2L_VALU, MSP_TWO_LEVEL, MSP_M2L_BF16X3 with p != 8 and
 * the weight-staging flags give MSP_ENOTSUP here and in msp_batch_backward and
 * msp_batch_autotune. */
int msp_batch_forward(msp_batch *b, const float *w, const uint8_t *is_target, const float *sigma,
                      const msp_fgt_params *prm, float *u_out, int32_t use_graph, void *stream);

/* Backward of every population (as msp_fgt_backward on its slice); grad_sigma:
 * device float64[npop] or NULL.  One fixed launch sequence covers all populations:
 * the two fields (weights w, and the upstream gradient at the targets) of the
 * expansion-route populations as batched P2M / M2L / L2P-with-derivatives passes
 * on an internal stream that forks from `stream` and joins it again, beside one
 * persistent P2P-with-derivatives launch per field for the direct-route
 * populations, then one combination launch and one sigma-reduction launch.  The
 * direct route gives the bits of msp_fgt_backward; the expansion route agrees with
 * it to float32 rounding (moments and translations summed in another order).  The
 * call returns once everything is enqueued.  use_graph = 1: the first call with
 * given pointers, sigma and parameters runs eagerly (it may synchronise) and
 * records the same work into a hipGraph; later calls with the same arguments, while
 * the populations' buffers stay where they were, launch that graph on `stream`.
 * use_graph = 0 runs eagerly every time (outputs at new addresses on every call
 * gain nothing from a graph). */
int msp_batch_backward(msp_batch *b, const float *w, const uint8_t *is_target, const float *sigma,
                       const msp_fgt_params *prm, const float *grad_u, float *grad_w, float *grad_x,
                       float *grad_y, float *grad_z, double *grad_sigma, int32_t use_graph, void *stream);

/* Per-population latency of the last forward call, from device timestamps
 * (host double[npop], milliseconds; 0 for empty populations).  Waits for the
 * device.  For direct-route populations it spans the first to the last work
 * item of the population inside the shared persistent launch. */
int msp_batch_instance_ms(msp_batch *b, double *ms);

/* Number of populations; launches of the last eager forward call. */
int msp_batch_info(const msp_batch *b, int32_t *npop, int64_t *launches);

/* Work of the direct-route populations in the last forward call (Eq. (8) over the
 * leaf interaction lists): *pairs (or NULL) gets the number of (target point,
 * source point) pairs their P2P pass evaluates, the sum over leaves of the leaf's
 * point count times the point counts of the leaves its list names, counted on the
 * device on `stream` (one small launch, then a wait for `stream`); *span_ms (or
 * NULL) gets the time from the first to the last work item of the shared
 * persistent launch, from device timestamps (0 without direct-route populations).
 * Both are 0 when no population took the direct route.  MSP_ESTATE before the
 * first forward after a build, or when a later call rebuilt or moved the
 * populations' lists (a backward with other parameters). */
int msp_batch_pair_count(msp_batch *b, int64_t *pairs, double *span_ms, void *stream);

/* Per-phase GPU timing.  When enabled, the library records a pair of HIP events
 * around each phase it launches, on the stream that runs it; msp_tree_get_timing
 * waits for them and returns, per phase, the summed milliseconds and the number
 * of launches since the last reset.  Phase names come from msp_phase_name.
 * enable: 0 off, 1 on, 2 on and isolated: the passes the library otherwise runs
 * beside each other (the partner walk on a side stream beside the direct passes)
 * run one after another on the caller's stream, so that each phase's time is
 * that of its kernels alone.  Other values: MSP_EINVAL. */
enum { MSP_PHASE_COUNT = 32 };
int msp_tree_set_timing(msp_tree *t, int enable);
int msp_tree_get_timing(msp_tree *t, double *ms /* host [MSP_PHASE_COUNT] */,
                        int64_t *launches /* host [MSP_PHASE_COUNT] */, int reset);
const char *msp_phase_name(int phase);

/* Work counters of the partner queries (msp_partner_probabilities and the
 * queries of a descent), for a work model of those kernels.  While counting is
 * enabled the query kernels add up, per pass:
 *   [0] queries and [1] point pairs summed by the eight-lane pass (nodes of at
 *       most 512 points), [2] queries and [3] pairs of the wavefront pass (at
 *       most 16384 points),
 *   [4] queries of the walk (larger nodes), [5] nodes it visited, [6] expansions
 *       (Eq. (7)) it evaluated, [7] point pairs it summed, [8] its stack rounds
 *       (per query, summed);
 * the other entries are 0.  msp_tree_get_work_counts waits for the device, copies
 * the counters to counts (host int64[MSP_WORK_COUNT]) and clears them if reset.
 * Counting adds atomic additions to those kernels: time them with it off.
 * Enabling clears the counters. */
enum { MSP_WORK_COUNT = 16 };
int msp_tree_set_work_counting(msp_tree *t, int enable);
int msp_tree_get_work_counts(msp_tree *t, int64_t *counts, int reset);

#ifdef __cplusplus
}
#endif
#endif /* MSPFMM_H */
