// kernels_d3q19_f64.hip -- D3Q19 / double instantiations of the forward kernels.
#include "kernels_impl.hpp"

namespace lbm {
template hipError_t dispatch_one<D3Q19, double>(const Launch &, int, int, bool, const void *, const void *, void *,
                                          void *, double *, int64_t);
}  // namespace lbm
