// kernels_d3q19.hip -- D3Q19 instantiations of the forward kernels.
#include "kernels_impl.hpp"

namespace lbm {
template hipError_t dispatch_storage<D3Q19>(const Launch &, int, int, bool, const void *, const void *, void *, void *,
                                          double *, int64_t);
template hipError_t solid_t<D3Q19>(const Launch &, const uint8_t *, uint8_t *, uint32_t *);
}  // namespace lbm
