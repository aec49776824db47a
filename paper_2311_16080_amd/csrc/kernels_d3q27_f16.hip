// kernels_d3q27_f16.hip -- D3Q27 / _Float16 instantiations of the forward kernels.
#include "kernels_impl.hpp"

namespace lbm {
template hipError_t dispatch_one<D3Q27, _Float16>(const Launch &, int, int, bool, const void *, const void *, void *,
                                          void *, double *, int64_t);
}  // namespace lbm
