// kernels_d2q9_f16.hip -- D2Q9 / _Float16 instantiations of the forward kernels.
#include "kernels_impl.hpp"

namespace lbm {
template hipError_t dispatch_one<D2Q9, _Float16>(const Launch &, int, int, bool, const void *, const void *, void *,
                                          void *, double *, int64_t);
}  // namespace lbm
