// tape.hip -- checkpoint tape and discrete adjoint (backward) driver.
#include <hip/hip_runtime.h>

#include "ctx.hpp"

using namespace lbm;

namespace lbm {
struct TapeState {
    int K = 0;
};
}  // namespace lbm

int lbm::tape_after_step(lbm_ctx *c) {
    (void)c;
    return LBM_OK;
}

void lbm::tape_release(lbm_ctx *c) {
    delete c->tape;
    c->tape = nullptr;
    c->tape_recording = false;
}

extern "C" int lbm_tape_begin(lbm_ctx *c, int K, int max_steps) {
    (void)K;
    (void)max_steps;
    if (!c) return fail(LBM_EINVAL, "null context");
    return fail(LBM_EUNSUPPORTED, "tape not available");
}

extern "C" int lbm_tape_end(lbm_ctx *c) {
    if (!c) return fail(LBM_EINVAL, "null context");
    c->tape_recording = false;
    return LBM_OK;
}

extern "C" int lbm_tape_free(lbm_ctx *c) {
    if (!c) return fail(LBM_EINVAL, "null context");
    tape_release(c);
    return LBM_OK;
}

extern "C" int lbm_backward(lbm_ctx *c, const void *dL_drho, const void *dL_du, int dtype, float *dL_ds,
                            double *dL_dtau, double *dL_duw) {
    (void)dL_drho; (void)dL_du; (void)dtype; (void)dL_ds; (void)dL_dtau; (void)dL_duw;
    if (!c) return fail(LBM_EINVAL, "null context");
    return fail(LBM_ESTATE, "no tape recorded");
}
