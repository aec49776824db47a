// batch.hip -- many independent domains advanced together.
#include <hip/hip_runtime.h>

#include "ctx.hpp"

using namespace lbm;

namespace lbm {
struct BatchState {
    int dummy = 0;
};
}  // namespace lbm

int lbm::batch_upload(lbm_ctx *c) { (void)c; return fail(LBM_EUNSUPPORTED, "batch not available"); }
void lbm::batch_release(lbm_ctx *c) { delete c->bs; c->bs = nullptr; }
hipError_t lbm::batch_init(lbm_ctx *, const void *, const void *, bool) { return hipErrorNotSupported; }
hipError_t lbm::batch_step(lbm_ctx *) { return hipErrorNotSupported; }
hipError_t lbm::batch_moments(lbm_ctx *, bool, void *, void *, bool, double *) { return hipErrorNotSupported; }

extern "C" lbm_ctx *lbm_create_batch(int lattice, int n, const int *nx, const int *ny, const int *nz,
                                     const double *tau, const lbm_bc *bcs) {
    (void)lattice; (void)n; (void)nx; (void)ny; (void)nz; (void)tau; (void)bcs;
    fail(LBM_EUNSUPPORTED, "batch not available");
    return nullptr;
}

extern "C" int lbm_batch_offsets(const lbm_ctx *c, int64_t *off) {
    if (!c || !off) return fail(LBM_EINVAL, "null argument");
    return fail(LBM_EINVAL, "not a batch context");
}
