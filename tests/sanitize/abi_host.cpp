// Host-side checks of the C ABI (argument validation, size queries, status text)
// run under AddressSanitizer and UndefinedBehaviorSanitizer.  No GPU is needed:
// every call here is refused or answered before any device work.
#include <cstdio>
#include <cstring>

#include "mspfmm.h"

static int fails = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);          \
            ++fails;                                                          \
        }                                                                     \
    } while (0)

int main() {
    CHECK(std::strcmp(msp_status_string(MSP_OK), "ok") == 0);
    CHECK(std::strcmp(msp_status_string(-99), "unknown status") == 0);
    for (int code = -7; code <= 0; ++code) CHECK(msp_status_string(code) != nullptr);

    size_t tb = 0, wb = 0;
    CHECK(msp_octree_build_query(4194304, 64, 21, &tb, &wb) == MSP_OK && tb > 48ull * 4194304 && wb > 0);
    CHECK(msp_octree_build_query(0, 1, 0, &tb, &wb) == MSP_OK);
    CHECK(msp_octree_build_query(-1, 64, 21, &tb, &wb) == MSP_EINVAL);
    CHECK(msp_octree_build_query(1ll << 31, 64, 21, &tb, &wb) == MSP_EOVERFLOW);
    CHECK(msp_octree_build_query(10, 0, 21, &tb, &wb) == MSP_EINVAL);
    CHECK(msp_octree_build_query(10, 64, 22, &tb, &wb) == MSP_EINVAL);
    CHECK(msp_octree_build_query(10, 64, 21, nullptr, &wb) == MSP_EINVAL);
    CHECK(std::strlen(msp_last_error()) > 0);

    // NULL handles are refused by every entry point that takes one
    msp_fgt_params prm = {8, -1, 100.f, 4.5f, MSP_ROUTE_AUTO, 0u};
    size_t bytes = 0;
    msp_tree_info info;
    msp_fgt_info finfo;
    CHECK(msp_octree_build(nullptr, nullptr, nullptr, nullptr, 10, 64, 21, nullptr) == MSP_EINVAL);
    CHECK(msp_octree_build_weighted(nullptr, nullptr, nullptr, nullptr, nullptr, 10, 64, 21, nullptr) == MSP_EINVAL);
    CHECK(msp_octree_build_ws(nullptr, nullptr, nullptr, nullptr, 10, 64, 21, nullptr, 0, nullptr, 0, nullptr) ==
          MSP_EINVAL);
    CHECK(msp_tree_get_info(nullptr, &info) == MSP_EINVAL);
    CHECK(msp_tree_export(nullptr, nullptr, nullptr) == MSP_EINVAL);
    CHECK(msp_fgt_plan(nullptr, &prm, &finfo) == MSP_EINVAL);
    CHECK(msp_fgt_forward(nullptr, nullptr, nullptr, &prm, nullptr, nullptr) == MSP_EINVAL);
    CHECK(msp_fgt_forward_query(nullptr, &prm, &bytes, nullptr) == MSP_EINVAL);
    CHECK(msp_fgt_forward_ws(nullptr, nullptr, nullptr, &prm, nullptr, nullptr, 0, nullptr) == MSP_EINVAL);
    CHECK(msp_fgt_backward(nullptr, nullptr, nullptr, &prm, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                           nullptr) == MSP_EINVAL);
    CHECK(msp_partner_probabilities(nullptr, nullptr, &prm, nullptr, nullptr, 0, nullptr, nullptr, nullptr,
                                    nullptr) == MSP_EINVAL);
    int64_t m = 0, nr = 0;
    CHECK(msp_descent_step(nullptr, nullptr, nullptr, &prm, 1, 0, nullptr, nullptr, 0, nullptr, nullptr, 0, &m,
                           nullptr, nullptr, 0, &nr, nullptr) == MSP_EINVAL);
    CHECK(msp_partner_descent(nullptr, nullptr, nullptr, &prm, 1, nullptr, nullptr, nullptr, &nr, nullptr,
                              nullptr) == MSP_EINVAL);
    CHECK(msp_fgt_debug_buffer(nullptr, 0, nullptr, 0, &bytes, nullptr) == MSP_EINVAL);
    CHECK(msp_tree_set_timing(nullptr, 1) == MSP_EINVAL);
    CHECK(msp_batch_build(nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr, 21, nullptr) == MSP_EINVAL);
    CHECK(msp_batch_info(nullptr, nullptr, nullptr) == MSP_EINVAL);

    // direct sum: sizes and sigma are checked before the device
    CHECK(msp_direct_sum(nullptr, nullptr, nullptr, -1, nullptr, nullptr, nullptr, nullptr, 0, 1.f, nullptr,
                         nullptr) == MSP_EINVAL);
    CHECK(msp_direct_sum(nullptr, nullptr, nullptr, 1ll << 40, nullptr, nullptr, nullptr, nullptr, 0, 1.f,
                         nullptr, nullptr) == MSP_EOVERFLOW);

    // parameter checks of the batch entry points come before the handle
    const uint32_t refused[] = {MSP_M2L_VALU, MSP_TWO_LEVEL, MSP_M2L_BF16X3, MSP_WEIGHTS_STAGED,
                                MSP_STAGE_WEIGHTS};
    for (uint32_t f : refused) {
        msp_fgt_params q = prm;
        q.flags = f;
        if (f == MSP_M2L_BF16X3) q.p = 6;   // split bfloat16 is built for p = 8 only
        CHECK(msp_batch_forward(nullptr, nullptr, nullptr, nullptr, &q, nullptr, 1, nullptr) == MSP_ENOTSUP);
        CHECK(msp_batch_backward(nullptr, nullptr, nullptr, nullptr, &q, nullptr, nullptr, nullptr, nullptr,
                                 nullptr, nullptr, 0, nullptr) == MSP_ENOTSUP);
    }
    msp_fgt_params bad = prm;
    bad.p = 0;
    CHECK(msp_batch_forward(nullptr, nullptr, nullptr, nullptr, &bad, nullptr, 1, nullptr) == MSP_EINVAL);
    bad = prm;
    bad.sigma = -1.f;
    CHECK(msp_batch_forward(nullptr, nullptr, nullptr, nullptr, &bad, nullptr, 1, nullptr) == MSP_EINVAL);
    bad = prm;
    bad.flags = 1u << 20;
    CHECK(msp_batch_forward(nullptr, nullptr, nullptr, nullptr, &bad, nullptr, 1, nullptr) == MSP_EINVAL);

    // a handle without a device: refused cleanly, or (with a device) created and destroyed
    msp_tree *t = nullptr;
    const int rc = msp_tree_create(&t);
    CHECK(rc == MSP_OK || t == nullptr);
    if (t) msp_tree_destroy(t);
    msp_tree_destroy(nullptr);
    msp_batch_destroy(nullptr);
    for (int ph = -1; ph <= MSP_PHASE_COUNT; ++ph) CHECK(msp_phase_name(ph) != nullptr);

    std::printf("%d failures\n", fails);
    return fails != 0;
}
