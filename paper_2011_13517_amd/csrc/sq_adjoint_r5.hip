// Adjoint kernels for FD radius 5 (split out so the instantiations build in parallel).
#include "sq_adjoint_kernel.h"

namespace sqk {
template hipError_t adjoint_dispatch_r<5>(int, int, bool, bool, const void *, int, hipStream_t,
                                           int *);
}  // namespace sqk
