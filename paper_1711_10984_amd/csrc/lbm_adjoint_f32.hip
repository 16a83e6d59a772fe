// FP32 instantiation of the adjoint kernels (lbm_adjoint_impl.h), built with contraction like the forward
// FP32 kernels.
#include "lbm_adjoint_impl.h"

namespace lbm {
LBM_INSTANTIATE_ADJOINT(float)
}  // namespace lbm
