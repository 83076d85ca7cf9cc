// Child probabilities for proportional partner choice (Algorithm 2).
#include "internal.hpp"

namespace msp {

int partner_probabilities(msp_tree *t, const float *w, const msp_fgt_params *prm,
                          const int32_t *target_idx, const int32_t *node_id, int64_t nq,
                          const float *uniforms, float *probs, int32_t *choice, hipStream_t s) {
    (void)t; (void)w; (void)prm; (void)target_idx; (void)node_id; (void)nq; (void)uniforms;
    (void)probs; (void)choice; (void)s;
    return fail(MSP_ENOTSUP, "partner probabilities: not built yet");
}

}  // namespace msp
