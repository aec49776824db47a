// kernels_d2q9_f32.hip -- D2Q9 / float instantiations of the forward kernels.
#include "kernels_impl.hpp"

namespace lbm {
template hipError_t dispatch_one<D2Q9, float>(const Launch &, int, int, bool, const void *, const void *, void *,
                                          void *, double *, int64_t);
template hipError_t solid_t<D2Q9>(const Launch &, const uint8_t *, uint8_t *, uint32_t *);
}  // namespace lbm
