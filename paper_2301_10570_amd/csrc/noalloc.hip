// msp_fgt_forward_noalloc: the forward sum for callers that cannot allocate device
// memory.  Its per-call buffers (the expansion route's grids and translation
// tables, or the direct route's flags, key-order sums and interaction lists) live
// in a fixed device array of this file instead of the handle's memory or a caller
// workspace; everything else is the workspace forward of api.hip.
#include "internal.hpp"

#include <mutex>

namespace msp {
namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;   // 64 MiB on every device that runs a call
constexpr int kMaxDevices = 64;

// One copy per device, held from the first call on that device until the process
// ends.  Host code must not use this name as a device address: it takes the
// address from hipGetSymbolAddress (scratch_on_device) instead.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// The device address of the current device's scratch array, looked up once per
// device with that device current.
int scratch_on_device(void **out) {
    int dev = 0;
    MSP_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(MSP_ENOTSUP, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        MSP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(MSP_EHIP, "hipGetSymbolAddress returned NULL for the scratch array");
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return MSP_OK;
}

}  // namespace
}  // namespace msp

using namespace msp;

extern "C" {

int msp_fgt_forward_noalloc(msp_tree *t, const float *w, const uint8_t *is_target, const msp_fgt_params *prm,
                            float *u_out, void *stream) {
    set_error("%s", "");
    hipStream_t s = (hipStream_t)stream;
    if (t && t->built && t->device >= 0) {
        int dev = -1;
        MSP_HIP(hipGetDevice(&dev));
        if (dev != t->device)
            return fail(MSP_EINVAL, "the tree lives on device %d, the current device is %d", t->device, dev);
    }
    size_t need = 0;
    MSP_TRY(forward_workspace_bytes(t, prm, &need, s));
    if (need > kScratchBytes)
        return fail(MSP_ENOSPC, "the call needs %zu bytes of scratch; the fixed scratch holds %zu", need,
                    kScratchBytes);
    void *ws = nullptr;
    MSP_TRY(scratch_on_device(&ws));
    return forward_in_workspace(t, w, is_target, prm, u_out, ws, kScratchBytes, s);
}

}  // extern "C"
