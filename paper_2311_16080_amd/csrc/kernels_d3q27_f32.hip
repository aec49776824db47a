// kernels_d3q27_f32.hip -- D3Q27 / float instantiations of the forward kernels.
#include "kernels_impl.hpp"

namespace lbm {
template hipError_t dispatch_one<D3Q27, float>(const Launch &, int, int, bool, const void *, const void *, void *,
                                          void *, double *, int64_t);
template hipError_t solid_t<D3Q27>(const Launch &, const uint8_t *, uint8_t *, uint32_t *);
}  // namespace lbm
