// C-ABI entry points declared in include/mspfmm.h: argument checks, handle
// management, and the order of the steps of a forward call.
#include "internal.hpp"

#include <cmath>
#include <cstdarg>
#include <algorithm>
#include <cstring>
#include <new>

namespace msp {

static thread_local char g_err[512];

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int DevBuf::ensure(size_t need) {
    if (need == 0) need = 1;
    if (need <= bytes) return MSP_OK;
    if (fixed)
        return fail(MSP_ENOSPC, "caller buffer region holds %zu bytes, %zu needed", bytes, need);
    if (p) {
        hipError_t e = hipFree(p);
        p = nullptr;
        bytes = 0;
        if (e != hipSuccess) return fail(MSP_EHIP, "hipFree: %s", hipGetErrorString(e));
    }
    hipError_t e = hipMalloc(&p, need);
    if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        return fail(MSP_EHIP, "hipMalloc(%zu bytes): %s", need, hipGetErrorString(e));
    }
    bytes = need;
    return MSP_OK;
}

void DevBuf::release() {
    if (p && !fixed) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    fixed = false;
}

int HostBuf::ensure(size_t need) {
    if (need == 0) need = 1;
    if (need <= bytes) return MSP_OK;
    release();
    hipError_t e = hipHostMalloc(&p, need, hipHostMallocDefault);
    if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        return fail(MSP_EHIP, "hipHostMalloc(%zu bytes): %s", need, hipGetErrorString(e));
    }
    bytes = need;
    return MSP_OK;
}

void HostBuf::release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
}

hipEvent_t Timing::get() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

void Timing::resolve() {
    for (const Rec &r : pending) {
        float ms_ = 0.f;
        (void)hipEventSynchronize(r.b);
        if (hipEventElapsedTime(&ms_, r.a, r.b) == hipSuccess) {
            ms[r.phase] += ms_;
            launches[r.phase] += 1;
        }
        pool.push_back(r.a);
        pool.push_back(r.b);
    }
    pending.clear();
}

Timing::~Timing() {
    for (const Rec &r : pending) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

static int check_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(MSP_EHIP, "no HIP device");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return fail(MSP_EHIP, "hipGetDeviceProperties failed");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(MSP_ENOTSUP, "device %d is %s; this library is built for gfx950 only", dev, prop.gcnArchName);
    return MSP_OK;
}

static bool misaligned(const void *p) { return ((uintptr_t)p & 255) != 0; }

// MSP_WEIGHTS_STAGED needs weights in the sorted records: from a weighted build,
// or kept by an earlier call since the build (and no backward since)
static int check_staged(const msp_tree *t, const msp_fgt_params *prm) {
    if ((prm->flags & MSP_WEIGHTS_STAGED) && !t->w_staged)
        return fail(MSP_ESTATE, "MSP_WEIGHTS_STAGED: the tree holds no staged weights (weighted build, or a "
                    "forward with MSP_STAGE_WEIGHTS, since the build or the last backward)");
    return MSP_OK;
}

static int check_params(const msp_fgt_params *prm) {
    if (!prm) return fail(MSP_EINVAL, "params is NULL");
    if (prm->p < 1 || prm->p > kMaxP) return fail(MSP_EINVAL, "p = %d outside 1..%d", prm->p, kMaxP);
    if (!(prm->sigma > 0.f) || !std::isfinite(prm->sigma)) return fail(MSP_EINVAL, "sigma must be finite and > 0");
    if (prm->level < -1 || prm->level > kDepth) return fail(MSP_EINVAL, "level = %d outside -1..21", prm->level);
    if (prm->route < MSP_ROUTE_AUTO || prm->route > MSP_ROUTE_DIRECT) return fail(MSP_EINVAL, "bad route %d", prm->route);
    if (prm->flags & ~(uint32_t)(MSP_EXCLUDE_SELF | MSP_M2L_VALU | MSP_TWO_LEVEL | MSP_M2L_BF16X3 |
                                 MSP_WEIGHTS_STAGED | MSP_STAGE_WEIGHTS))
        return fail(MSP_EINVAL, "unknown flags 0x%x", prm->flags);
    if ((prm->flags & MSP_M2L_VALU) && (prm->flags & MSP_M2L_BF16X3))
        return fail(MSP_EINVAL, "MSP_M2L_VALU and MSP_M2L_BF16X3 exclude each other");
    if (std::isnan(prm->cutoff_sigmas)) return fail(MSP_EINVAL, "cutoff_sigmas is NaN");
    return MSP_OK;
}

}  // namespace msp

using namespace msp;

extern "C" {

const char *msp_status_string(int status) {
    switch (status) {
        case MSP_OK: return "ok";
        case MSP_EINVAL: return "invalid argument";
        case MSP_ENOSPC: return "size limit exceeded";
        case MSP_EOVERFLOW: return "index overflow";
        case MSP_EHIP: return "HIP runtime error";
        case MSP_ENOTSUP: return "not supported";
        case MSP_ESTATE: return "handle not ready";
    }
    return "unknown status";
}

const char *msp_last_error(void) { return g_err; }

int msp_tree_create(msp_tree **out) {
    if (!out) return fail(MSP_EINVAL, "out is NULL");
    *out = nullptr;
    MSP_TRY(check_device());
    msp_tree *t = new (std::nothrow) msp_tree();
    if (!t) return fail(MSP_ENOSPC, "host allocation failed");
    (void)hipGetDevice(&t->device);
    // page-locked landing area of the build's one readback, made here so that a
    // build into caller buffers allocates nothing
    const int rc = t->build_stage.ensure(256);
    if (rc != MSP_OK) {
        delete t;
        return rc;
    }
    *out = t;
    return MSP_OK;
}

void msp_tree_destroy(msp_tree *t) {
    if (!t) return;
    (void)hipDeviceSynchronize();
    delete t;
}

int msp_octree_build(msp_tree *t, const float *x, const float *y, const float *z, int64_t n,
                     int32_t leaf_max, int32_t max_depth, void *stream) {
    g_err[0] = 0;
    if (!t) return fail(MSP_EINVAL, "tree handle is NULL");
    if (n < 0) return fail(MSP_EINVAL, "n = %lld < 0", (long long)n);
    if (n > 0x7fffffffLL) return fail(MSP_EOVERFLOW, "n = %lld exceeds 2^31-1", (long long)n);
    if (n > 0 && (!x || !y || !z)) return fail(MSP_EINVAL, "NULL coordinate array");
    if (leaf_max < 1) return fail(MSP_EINVAL, "leaf_max = %d < 1", leaf_max);
    if (max_depth < 0 || max_depth > kDepth) return fail(MSP_EINVAL, "max_depth = %d outside 0..21", max_depth);
    return build_tree(t, x, y, z, n, leaf_max, max_depth, (hipStream_t)stream);
}

int msp_octree_build_weighted(msp_tree *t, const float *x, const float *y, const float *z, const float *w,
                              int64_t n, int32_t leaf_max, int32_t max_depth, void *stream) {
    g_err[0] = 0;
    if (!t) return fail(MSP_EINVAL, "tree handle is NULL");
    if (n < 0) return fail(MSP_EINVAL, "n = %lld < 0", (long long)n);
    if (n > 0x7fffffffLL) return fail(MSP_EOVERFLOW, "n = %lld exceeds 2^31-1", (long long)n);
    if (n > 0 && (!x || !y || !z || !w)) return fail(MSP_EINVAL, "NULL coordinate or weight array");
    if (leaf_max < 1) return fail(MSP_EINVAL, "leaf_max = %d < 1", leaf_max);
    if (max_depth < 0 || max_depth > kDepth) return fail(MSP_EINVAL, "max_depth = %d outside 0..21", max_depth);
    return build_tree(t, x, y, z, n, leaf_max, max_depth, (hipStream_t)stream, nullptr, 0, nullptr, 0, w);
}

int msp_octree_build_query(int64_t n, int32_t leaf_max, int32_t max_depth, size_t *tree_bytes,
                           size_t *ws_bytes) {
    g_err[0] = 0;
    if (!tree_bytes || !ws_bytes) return fail(MSP_EINVAL, "NULL size output");
    if (n < 0) return fail(MSP_EINVAL, "n = %lld < 0", (long long)n);
    if (n > 0x7fffffffLL) return fail(MSP_EOVERFLOW, "n = %lld exceeds 2^31-1", (long long)n);
    if (leaf_max < 1) return fail(MSP_EINVAL, "leaf_max = %d < 1", leaf_max);
    if (max_depth < 0 || max_depth > kDepth) return fail(MSP_EINVAL, "max_depth = %d outside 0..21", max_depth);
    build_query_bytes(n, leaf_max, max_depth, tree_bytes, ws_bytes);
    return MSP_OK;
}

int msp_octree_build_ws(msp_tree *t, const float *x, const float *y, const float *z, int64_t n,
                        int32_t leaf_max, int32_t max_depth, void *tree_buf, size_t tree_bytes, void *ws,
                        size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    if (!t) return fail(MSP_EINVAL, "tree handle is NULL");
    if (n < 0) return fail(MSP_EINVAL, "n = %lld < 0", (long long)n);
    if (n > 0x7fffffffLL) return fail(MSP_EOVERFLOW, "n = %lld exceeds 2^31-1", (long long)n);
    if (n > 0 && (!x || !y || !z)) return fail(MSP_EINVAL, "NULL coordinate array");
    if (leaf_max < 1) return fail(MSP_EINVAL, "leaf_max = %d < 1", leaf_max);
    if (max_depth < 0 || max_depth > kDepth) return fail(MSP_EINVAL, "max_depth = %d outside 0..21", max_depth);
    if (!tree_buf || !ws) return fail(MSP_EINVAL, "NULL tree buffer or workspace");
    if (misaligned(tree_buf) || misaligned(ws)) return fail(MSP_EINVAL, "buffers must be 256-byte aligned");
    return build_tree(t, x, y, z, n, leaf_max, max_depth, (hipStream_t)stream, tree_buf, tree_bytes, ws,
                      ws_bytes);
}

int msp_tree_get_info(const msp_tree *t, msp_tree_info *info) {
    if (!t || !info) return fail(MSP_EINVAL, "NULL argument");
    if (!t->built) return fail(MSP_ESTATE, "no tree built");
    std::memset(info, 0, sizeof(*info));
    info->n = t->n;
    info->n_nodes = t->n_nodes;
    info->depth = t->depth;
    info->leaf_max = t->leaf_max;
    info->max_depth = t->max_depth;
    for (int k = 0; k < 3; ++k) {
        info->qmax[k] = t->geo.qmax[k];
        info->lo[k] = t->geo.lo[k];
    }
    info->side = t->geo.side;
    for (int l = 0; l < kMaxLevels; ++l) info->level_offset[l] = t->level_off[l];
    return MSP_OK;
}

int msp_tree_export(const msp_tree *t, const msp_tree_arrays *d, void *stream) {
    if (!t || !d) return fail(MSP_EINVAL, "NULL argument");
    if (!t->built) return fail(MSP_ESTATE, "no tree built");
    hipStream_t s = (hipStream_t)stream;
    const size_t nb = (size_t)t->n, nn = (size_t)t->n_nodes;
    struct Item { void *dst; const DevBuf *src; size_t bytes; };
    const Item items[] = {
        {d->keys, &t->keys, nb * 8},          {d->perm, &t->perm, nb * 4},
        {d->node_level, &t->nlevel, nn * 4},  {d->node_first, &t->nfirst, nn * 4},
        {d->node_count, &t->ncount, nn * 4},  {d->node_parent, &t->nparent, nn * 4},
        {d->node_first_child, &t->nfchild, nn * 4}, {d->node_n_children, &t->nnchild, nn * 4},
        {d->node_digit, &t->ndigit, nn * 4},  {d->node_ix, &t->nix, nn * 4},
        {d->node_iy, &t->niy, nn * 4},        {d->node_iz, &t->niz, nn * 4},
    };
    for (const Item &it : items)
        if (it.dst && it.bytes) MSP_HIP(hipMemcpyAsync(it.dst, it.src->p, it.bytes, hipMemcpyDeviceToDevice, s));
    return MSP_OK;
}

int msp_fgt_plan(msp_tree *t, const msp_fgt_params *prm, msp_fgt_info *info) {
    if (!t || !info) return fail(MSP_EINVAL, "NULL argument");
    if (!t->built) return fail(MSP_ESTATE, "no tree built");
    MSP_TRY(check_params(prm));
    FgtPlan pl;
    MSP_TRY(plan_fgt(t, prm, &pl));
    info->route = pl.route;
    info->level = pl.level;
    for (int k = 0; k < 3; ++k) info->grid[k] = pl.G[k];
    info->p = pl.p;
    info->rho = pl.rho;
    info->fgt_cost = pl.fgt_cost;
    info->direct_cost = pl.direct_cost;
    info->fine_terms = pl.route == MSP_ROUTE_FGT ? pl.pf : 0;
    return MSP_OK;
}

int msp_fgt_forward(msp_tree *t, const float *w, const uint8_t *is_target,
                    const msp_fgt_params *prm, float *u_out, void *stream) {
    g_err[0] = 0;
    if (!t) return fail(MSP_EINVAL, "tree handle is NULL");
    if (!t->built) return fail(MSP_ESTATE, "no tree built");
    MSP_TRY(check_params(prm));
    if (t->n > 0 && (!w || !u_out)) return fail(MSP_EINVAL, "NULL weight or output array");
    hipStream_t s = (hipStream_t)stream;
    FgtPlan pl;
    MSP_TRY(plan_fgt(t, prm, &pl));
    MSP_TRY(check_staged(t, prm));
    t->w_staged = false;   // set again by the paths that gather w into ps.w
    if (pl.route == MSP_ROUTE_FGT) {
        const int rc = fgt_forward_grid(t, pl, prm, w, is_target, u_out, s);
        // the records keep staged weights; the single-level P2M gathers w into them
        // when asked to
        t->w_staged = rc == MSP_OK && ((prm->flags & MSP_WEIGHTS_STAGED) ||
                                       (pl.pf == 0 && (prm->flags & MSP_STAGE_WEIGHTS)));
        return rc;
    }
    MSP_TRY(stage_inputs(t, w, is_target, s));
    t->w_staged = true;
    MSP_TRY(direct_route(t, prm, s));
    return scatter_output(t, u_out, prm->flags, false, s);
}

}  // extern "C"

namespace msp {
namespace {
// The regions of a forward call's workspace, in order: the expansion route's two
// grids and the buffer of its third grid and operator tables, or the direct
// route's target flags, key-order sums and list entries (whose count needs the
// list lengths).  sw == NULL only counts.
void forward_layout(msp_tree *t, const FgtPlan &pl, Carve &c, BufSwap *sw) {
    auto put = [&](DevBuf &b, size_t bytes) {
        if (sw) sw->bind(b, c, bytes);
        else c.take(bytes);
    };
    if (pl.route == MSP_ROUTE_FGT) {
        size_t g = 0, o = 0;
        fgt_grid_bytes(pl, &g, &o);
        put(t->gridA, g);
        put(t->gridB, g);
        put(t->ops, o);
    } else {
        const size_t nb = (size_t)(t->n > 0 ? t->n : 1);
        put(t->tflag, nb);
        put(t->usort, nb * 4);
        put(t->list_idx, (size_t)(t->list_total > 0 ? t->list_total : 1) * 4);
    }
}
}  // namespace
}  // namespace msp

extern "C" {

int msp_fgt_forward_query(msp_tree *t, const msp_fgt_params *prm, size_t *ws_bytes, void *stream) {
    g_err[0] = 0;
    if (!ws_bytes) return fail(MSP_EINVAL, "NULL size output");
    return forward_workspace_bytes(t, prm, ws_bytes, (hipStream_t)stream);
}

int msp_fgt_forward_ws(msp_tree *t, const float *w, const uint8_t *is_target, const msp_fgt_params *prm,
                       float *u_out, void *ws, size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    if (!ws) return fail(MSP_EINVAL, "workspace is NULL");
    return forward_in_workspace(t, w, is_target, prm, u_out, ws, ws_bytes, (hipStream_t)stream);
}

}  // extern "C"

namespace msp {
int forward_in_workspace(msp_tree *t, const float *w, const uint8_t *is_target, const msp_fgt_params *prm,
                         float *u_out, void *ws, size_t ws_bytes, hipStream_t s) {
    if (!t) return fail(MSP_EINVAL, "tree handle is NULL");
    if (!t->built) return fail(MSP_ESTATE, "no tree built");
    MSP_TRY(check_params(prm));
    if (t->n > 0 && (!w || !u_out)) return fail(MSP_EINVAL, "NULL weight or output array");
    if (misaligned(ws)) return fail(MSP_EINVAL, "workspace must be 256-byte aligned");
    FgtPlan pl;
    MSP_TRY(plan_fgt(t, prm, &pl));
    if (pl.route == MSP_ROUTE_DIRECT) MSP_TRY(direct_route_counts(t, prm, s));
    {
        Carve probe(nullptr, 0);
        forward_layout(t, pl, probe, nullptr);
        if (probe.used > ws_bytes)
            return fail(MSP_ENOSPC, "workspace holds %zu bytes, the call needs %zu (msp_fgt_forward_query)",
                        ws_bytes, probe.used);
    }
    MSP_TRY(check_staged(t, prm));
    t->w_staged = false;
    t->grid_bytes_valid = 0;   // the grids of this call live in the caller's workspace
    Carve c(ws, ws_bytes);
    BufSwap sw;
    forward_layout(t, pl, c, &sw);
    if (pl.route == MSP_ROUTE_FGT) {
        // the operator tables are rebuilt in the workspace; the handle's own copy
        // stays as it was
        const bool ops_valid = t->ops_valid;
        uint64_t ops_sig[5];
        std::copy(t->ops_sig, t->ops_sig + 5, ops_sig);
        t->ops_valid = false;
        const int rc = fgt_forward_grid(t, pl, prm, w, is_target, u_out, s);
        t->ops_valid = ops_valid;
        std::copy(ops_sig, ops_sig + 5, t->ops_sig);
        t->grid_bytes_valid = 0;
        t->w_staged = rc == MSP_OK && ((prm->flags & MSP_WEIGHTS_STAGED) ||
                                       (pl.pf == 0 && (prm->flags & MSP_STAGE_WEIGHTS)));
        return rc;
    }
    MSP_TRY(stage_inputs(t, w, is_target, s));
    MSP_TRY(direct_route_fill(t, prm, s));
    MSP_TRY(direct_route(t, prm, s, true));
    MSP_TRY(scatter_output(t, u_out, prm->flags, false, s));
    t->w_staged = true;
    return MSP_OK;
}

int forward_workspace_bytes(msp_tree *t, const msp_fgt_params *prm, size_t *bytes, hipStream_t s) {
    if (!t) return fail(MSP_EINVAL, "tree handle is NULL");
    if (!t->built) return fail(MSP_ESTATE, "no tree built");
    MSP_TRY(check_params(prm));
    FgtPlan pl;
    MSP_TRY(plan_fgt(t, prm, &pl));
    if (pl.route == MSP_ROUTE_DIRECT) MSP_TRY(direct_route_counts(t, prm, s));
    Carve c(nullptr, 0);
    forward_layout(t, pl, c, nullptr);
    *bytes = c.used;
    return MSP_OK;
}
}  // namespace msp

extern "C" {

int msp_fgt_backward(msp_tree *t, const float *w, const uint8_t *is_target,
                     const msp_fgt_params *prm, const float *grad_u, float *grad_w, float *grad_x,
                     float *grad_y, float *grad_z, double *grad_sigma, void *stream) {
    g_err[0] = 0;
    if (!t) return fail(MSP_EINVAL, "tree handle is NULL");
    if (!t->built) return fail(MSP_ESTATE, "no tree built");
    MSP_TRY(check_params(prm));
    if (t->n > 0 && (!w || !grad_u)) return fail(MSP_EINVAL, "NULL weight or upstream gradient");
    const int npos = (grad_x != nullptr) + (grad_y != nullptr) + (grad_z != nullptr);
    if (npos != 0 && npos != 3) return fail(MSP_EINVAL, "give all three position gradients or none");
    t->w_staged = false;   // the backward gathers the upstream gradient into ps.w too
    return fgt_backward(t, w, is_target, prm, grad_u, grad_w, grad_x, grad_y, grad_z, grad_sigma,
                        (hipStream_t)stream);
}

int msp_direct_sum(const float *tx, const float *ty, const float *tz, int64_t nt, const float *sx,
                   const float *sy, const float *sz, const float *w, int64_t ns, float sigma,
                   float *u, void *stream) {
    g_err[0] = 0;
    if (nt < 0 || ns < 0) return fail(MSP_EINVAL, "negative size");
    if (nt > 0x7fffffffLL || ns > 0x7fffffffLL) return fail(MSP_EOVERFLOW, "size exceeds 2^31-1");
    if (nt > 0 && (!tx || !ty || !tz || !u)) return fail(MSP_EINVAL, "NULL target array");
    if (ns > 0 && (!sx || !sy || !sz || !w)) return fail(MSP_EINVAL, "NULL source array");
    if (!(sigma > 0.f) || !std::isfinite(sigma)) return fail(MSP_EINVAL, "sigma must be finite and > 0");
    MSP_TRY(check_device());
    return direct_all_pairs(tx, ty, tz, nt, sx, sy, sz, w, ns, sigma, u, (hipStream_t)stream);
}

int msp_partner_probabilities(msp_tree *t, const float *w, const msp_fgt_params *prm,
                              const int32_t *target_idx, const int32_t *node_id, int64_t nq,
                              const float *uniforms, float *probs, int32_t *choice, void *stream) {
    g_err[0] = 0;
    if (!t) return fail(MSP_EINVAL, "tree handle is NULL");
    if (!t->built) return fail(MSP_ESTATE, "no tree built");
    MSP_TRY(check_params(prm));
    if (nq < 0) return fail(MSP_EINVAL, "nq < 0");
    if (nq > 0 && (!w || !target_idx || !node_id || !probs)) return fail(MSP_EINVAL, "NULL array");
    if (nq > 0x7fffffffLL) return fail(MSP_EOVERFLOW, "nq exceeds 2^31-1");
    MSP_TRY(check_staged(t, prm));
    const int rc = partner_probabilities(t, w, prm, target_idx, node_id, nq, uniforms, probs, choice,
                                         (hipStream_t)stream);
    t->w_staged = rc == MSP_OK;
    return rc;
}

int msp_descent_step(msp_tree *t, const float *w, const float *a, const msp_fgt_params *prm, uint64_t seed,
                     int32_t step, const int64_t *S_in, const int64_t *T_in, int64_t m, int64_t *S_out,
                     int64_t *T_out, int64_t cap, int64_t *m_out, int32_t *req_axon, int32_t *req_dendrite,
                     int64_t req_cap, int64_t *n_req, void *stream) {
    g_err[0] = 0;
    if (!t) return fail(MSP_EINVAL, "tree handle is NULL");
    if (!t->built) return fail(MSP_ESTATE, "no tree built");
    MSP_TRY(check_params(prm));
    if (m < 0 || cap < 0 || req_cap < 0 || step < 0) return fail(MSP_EINVAL, "negative size or step");
    if (!m_out || !n_req) return fail(MSP_EINVAL, "NULL count output");
    if (m > 0 && (!S_in || !T_in)) return fail(MSP_EINVAL, "NULL frontier");
    if ((cap > 0 && (!S_out || !T_out)) || (req_cap > 0 && (!req_axon || !req_dendrite)))
        return fail(MSP_EINVAL, "NULL output array");
    if (t->n > 0 && (!w || !a)) return fail(MSP_EINVAL, "NULL weight array");
    if (t->n == 0) {
        if (m > 0) return fail(MSP_EINVAL, "descent on an empty tree");
        *m_out = 0;
        *n_req = 0;
        return MSP_OK;
    }
    const int rc = descent_step(t, w, a, prm, seed, step, S_in, T_in, m, S_out, T_out, cap, m_out, req_axon,
                                req_dendrite, req_cap, n_req, (hipStream_t)stream);
    t->w_staged = rc == MSP_OK;
    return rc;
}

int msp_partner_descent(msp_tree *t, const float *w, const float *a, const msp_fgt_params *prm, uint64_t seed,
                        int32_t *req_axon, int32_t *req_dendrite, uint8_t *accepted, int64_t *n_req,
                        int32_t *n_steps, void *stream) {
    g_err[0] = 0;
    if (!t) return fail(MSP_EINVAL, "tree handle is NULL");
    if (!t->built) return fail(MSP_ESTATE, "no tree built");
    MSP_TRY(check_params(prm));
    if (!n_req) return fail(MSP_EINVAL, "NULL count output");
    if (t->n > 0 && (!w || !a || !req_axon || !req_dendrite || !accepted)) return fail(MSP_EINVAL, "NULL array");
    if (t->n == 0) {
        *n_req = 0;
        if (n_steps) *n_steps = 0;
        return MSP_OK;
    }
    const int rc = partner_descent(t, w, a, prm, seed, req_axon, req_dendrite, accepted, n_req, n_steps,
                                   (hipStream_t)stream);
    t->w_staged = rc == MSP_OK;
    return rc;
}

int msp_fgt_debug_buffer(msp_tree *t, int32_t which, void *dst, size_t dst_bytes, size_t *bytes,
                         void *stream) {
    if (!t || !bytes) return fail(MSP_EINVAL, "NULL argument");
    const void *src = nullptr;
    if (which == 0 || which == 1) {
        if (t->grid_bytes_valid <= 0) return fail(MSP_ESTATE, "no expansion-route call yet");
        *bytes = (size_t)t->grid_bytes_valid;
        src = which == 0 ? t->gridA.p : t->gridB.p;
    } else if (which == 2 || which == 3) {
        if (t->node_moments_level < 0) return fail(MSP_ESTATE, "no partner call yet");
        *bytes = which == 2 ? (size_t)t->node_moments_bytes : (size_t)t->n_nodes;
        src = which == 2 ? t->nodeA.p : t->node_hasA.p;
    } else if (which >= 4 && which <= 7) {
        if (t->desc_box_level < 0) return fail(MSP_ESTATE, "the last descent used no box pairs");
        const size_t np = (size_t)t->desc_npair, pa = (np * 4 + 255) / 256 * 256;
        const char *dp = t->desc_pairs.as<char>();
        if (which == 4) {
            *bytes = np * 8;
            src = dp + 2 * pa;
        } else if (which == 5 || which == 6) {
            *bytes = np * 4;
            src = dp + (which == 6 ? pa : 0);
        } else {
            *bytes = (size_t)t->desc_nbox * 4;
            src = t->desc_box.as<char>() + ((size_t)t->n_nodes * 4 + 255) / 256 * 256;
        }
    } else if (which == 8 || which == 9) {
        if (!t->built) return fail(MSP_ESTATE, "no tree built");
        if (which == 9) MSP_TRY(ensure_iperm(t, (hipStream_t)stream));
        *bytes = (size_t)t->n * (which == 8 ? 16 : 4);
        src = which == 8 ? t->ps.p : t->iperm.p;
    } else {
        return fail(MSP_EINVAL, "which must be 0..9");
    }
    if (!dst) return MSP_OK;
    if (dst_bytes < *bytes) return fail(MSP_EINVAL, "destination holds %zu bytes, need %zu", dst_bytes, *bytes);
    MSP_HIP(hipMemcpyAsync(dst, src, *bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return MSP_OK;
}

int msp_tree_set_work_counting(msp_tree *t, int enable) {
    set_error("%s", "");
    if (!t) return fail(MSP_EINVAL, "tree handle is NULL");
    if (enable && !t->counting) {
        MSP_TRY(t->work.ensure((size_t)MSP_WORK_COUNT * 8));
        MSP_HIP(hipMemset(t->work.p, 0, (size_t)MSP_WORK_COUNT * 8));
    }
    t->counting = enable != 0;
    return MSP_OK;
}

int msp_tree_get_work_counts(msp_tree *t, int64_t *counts, int reset) {
    set_error("%s", "");
    if (!t || !counts) return fail(MSP_EINVAL, "NULL argument");
    if (!t->work.p) {
        for (int k = 0; k < MSP_WORK_COUNT; ++k) counts[k] = 0;
        return MSP_OK;
    }
    MSP_HIP(hipDeviceSynchronize());
    MSP_HIP(hipMemcpy(counts, t->work.p, (size_t)MSP_WORK_COUNT * 8, hipMemcpyDeviceToHost));
    if (reset) MSP_HIP(hipMemset(t->work.p, 0, (size_t)MSP_WORK_COUNT * 8));
    return MSP_OK;
}

int msp_tree_set_timing(msp_tree *t, int enable) {
    if (!t) return fail(MSP_EINVAL, "tree handle is NULL");
    if (enable < 0 || enable > 2) return fail(MSP_EINVAL, "timing mode %d outside 0..2", enable);
    t->timing.on = enable != 0;
    t->timing.isolate = enable == 2;
    return MSP_OK;
}

int msp_tree_get_timing(msp_tree *t, double *ms, int64_t *launches, int reset) {
    if (!t) return fail(MSP_EINVAL, "tree handle is NULL");
    t->timing.resolve();
    for (int k = 0; k < MSP_PHASE_COUNT; ++k) {
        if (ms) ms[k] = t->timing.ms[k];
        if (launches) launches[k] = t->timing.launches[k];
        if (reset) { t->timing.ms[k] = 0.0; t->timing.launches[k] = 0; }
    }
    return MSP_OK;
}

int msp_batch_create(msp_batch **out) {
    if (!out) return fail(MSP_EINVAL, "out is NULL");
    *out = nullptr;
    MSP_TRY(check_device());
    msp_batch *b = new (std::nothrow) msp_batch();
    if (!b) return fail(MSP_ENOSPC, "host allocation failed");
    (void)hipGetDevice(&b->device);
    *out = b;
    return MSP_OK;
}

void msp_batch_destroy(msp_batch *b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    delete b;
}

// the batched kernels translate on the matrix cores on one level (fp32, or split
// bfloat16 at p = 8), and the weight-staging flags have no meaning for a batch
static int check_batch_flags(const msp_fgt_params *prm) {
    const uint32_t bad = prm->flags & (uint32_t)(MSP_M2L_VALU | MSP_TWO_LEVEL | MSP_WEIGHTS_STAGED |
                                                 MSP_STAGE_WEIGHTS);
    if (bad) return fail(MSP_ENOTSUP, "flags 0x%x are not supported by the batch entry points", bad);
    if ((prm->flags & MSP_M2L_BF16X3) && prm->p != 8)
        return fail(MSP_ENOTSUP, "split-bfloat16 translation in a batch is not supported for p != 8");
    return MSP_OK;
}

static int check_offsets(const int64_t *offsets, int32_t npop) {
    if (npop < 0) return fail(MSP_EINVAL, "npop = %d < 0", npop);
    if (!offsets) return fail(MSP_EINVAL, "offsets is NULL");
    if (offsets[0] != 0) return fail(MSP_EINVAL, "offsets[0] must be 0");
    for (int32_t k = 0; k < npop; ++k) {
        if (offsets[k + 1] < offsets[k]) return fail(MSP_EINVAL, "offsets decrease at %d", k);
        if (offsets[k + 1] - offsets[k] > 0x7fffffffLL) return fail(MSP_EOVERFLOW, "population %d too large", k);
    }
    return MSP_OK;
}

int msp_batch_build(msp_batch *b, const float *x, const float *y, const float *z, const int64_t *offsets,
                    int32_t npop, const int32_t *leaf_max, int32_t max_depth, void *stream) {
    g_err[0] = 0;
    if (!b) return fail(MSP_EINVAL, "batch handle is NULL");
    MSP_TRY(check_offsets(offsets, npop));
    if (offsets[npop] > 0 && (!x || !y || !z)) return fail(MSP_EINVAL, "NULL coordinate array");
    if (max_depth < 0 || max_depth > kDepth) return fail(MSP_EINVAL, "max_depth = %d outside 0..21", max_depth);
    if (leaf_max)
        for (int32_t k = 0; k < npop; ++k)
            if (leaf_max[k] < 1) return fail(MSP_EINVAL, "leaf_max[%d] < 1", k);
    return batch_build(b, x, y, z, offsets, npop, leaf_max, max_depth, (hipStream_t)stream);
}

int msp_batch_autotune(msp_batch *b, const float *x, const float *y, const float *z,
                       const int64_t *offsets, int32_t npop, const float *w, const uint8_t *is_target,
                       const float *sigma, const msp_fgt_params *prm, const int32_t *cand, int32_t ncand,
                       int32_t max_depth, float *scratch_u, int32_t *leaf_out, int32_t *route_out,
                       void *stream) {
    g_err[0] = 0;
    MSP_TRY(check_params(prm));
    MSP_TRY(check_batch_flags(prm));
    if (!b) return fail(MSP_EINVAL, "batch handle is NULL");
    MSP_TRY(check_offsets(offsets, npop));
    if (offsets[npop] > 0 && (!x || !y || !z || !w || !scratch_u)) return fail(MSP_EINVAL, "NULL array");
    if (npop > 0 && !sigma) return fail(MSP_EINVAL, "sigma is NULL");
    if (!cand || ncand < 1) return fail(MSP_EINVAL, "no candidate leaf sizes");
    for (int32_t c = 0; c < ncand; ++c)
        if (cand[c] < 1) return fail(MSP_EINVAL, "candidate leaf size %d < 1", cand[c]);
    if (max_depth < 0 || max_depth > kDepth) return fail(MSP_EINVAL, "max_depth = %d outside 0..21", max_depth);
    return batch_autotune(b, x, y, z, offsets, npop, w, is_target, sigma, prm, cand, ncand, max_depth,
                          scratch_u, leaf_out, route_out, (hipStream_t)stream);
}

int msp_batch_forward(msp_batch *b, const float *w, const uint8_t *is_target, const float *sigma,
                      const msp_fgt_params *prm, float *u_out, int32_t use_graph, void *stream) {
    g_err[0] = 0;
    MSP_TRY(check_params(prm));
    MSP_TRY(check_batch_flags(prm));
    if (!b) return fail(MSP_EINVAL, "batch handle is NULL");
    if (b->npop > 0 && !sigma) return fail(MSP_EINVAL, "sigma is NULL");
    if (b->npop > 0 && b->off[b->npop] > 0 && (!w || !u_out)) return fail(MSP_EINVAL, "NULL weight or output array");
    return batch_forward(b, w, is_target, sigma, prm, u_out, use_graph, (hipStream_t)stream);
}

int msp_batch_backward(msp_batch *b, const float *w, const uint8_t *is_target, const float *sigma,
                       const msp_fgt_params *prm, const float *grad_u, float *grad_w, float *grad_x,
                       float *grad_y, float *grad_z, double *grad_sigma, int32_t use_graph, void *stream) {
    g_err[0] = 0;
    MSP_TRY(check_params(prm));
    MSP_TRY(check_batch_flags(prm));
    if (!b) return fail(MSP_EINVAL, "batch handle is NULL");
    if (b->npop > 0 && !sigma) return fail(MSP_EINVAL, "sigma is NULL");
    if (b->npop > 0 && b->off[b->npop] > 0 && (!w || !grad_u)) return fail(MSP_EINVAL, "NULL weight or upstream gradient");
    const int npos = (grad_x != nullptr) + (grad_y != nullptr) + (grad_z != nullptr);
    if (npos != 0 && npos != 3) return fail(MSP_EINVAL, "give all three position gradients or none");
    return batch_backward(b, w, is_target, sigma, prm, grad_u, grad_w, grad_x, grad_y, grad_z, grad_sigma,
                          use_graph, (hipStream_t)stream);
}

int msp_batch_instance_ms(msp_batch *b, double *ms) {
    if (!b || (b->npop > 0 && !ms)) return fail(MSP_EINVAL, "NULL argument");
    return batch_instance_ms(b, ms);
}

int msp_batch_info(const msp_batch *b, int32_t *npop, int64_t *launches) {
    if (!b) return fail(MSP_EINVAL, "batch handle is NULL");
    return batch_info(b, npop, launches);
}

int msp_batch_pair_count(msp_batch *b, int64_t *pairs, double *span_ms, void *stream) {
    if (!b) return fail(MSP_EINVAL, "batch handle is NULL");
    return batch_pair_count(b, pairs, span_ms, (hipStream_t)stream);
}

const char *msp_phase_name(int phase) {
    static const char *names[PH_COUNT_] = {"bbox", "morton", "radix_sort", "node_levels", "node_table",
                                           "gather_sorted", "stage", "m2l_operators", "p2m", "m2l_x",
                                           "m2l_y", "m2l_z", "l2p", "interaction_lists", "p2p",
                                           "scatter", "node_moments", "partner", "direct",
                                           "backward_combine", "sort_hist", "sort_digit_scan",
                                           "sort_scatter", "node_source_counts", "partner_direct",
                                           "sort_runs", "partner_wave", "descent_boxes", "descent_choose",
                                           "descent_pairs"};
    if (phase < 0 || phase >= PH_COUNT_) return "";
    return names[phase];
}

}  // extern "C"
