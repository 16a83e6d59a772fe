// FP64 instantiation of the adjoint kernels (lbm_adjoint_impl.h), built without contraction like the
// forward FP64 kernels.
#include "lbm_adjoint_impl.h"

namespace lbm {
LBM_INSTANTIATE_ADJOINT(double)
}  // namespace lbm
