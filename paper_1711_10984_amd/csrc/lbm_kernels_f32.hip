// FP32 instantiation of the timestep kernels (lbm_kernels_impl.h).  Built with fused multiply-add
// contraction (the FP32 path is compared with the FP64 oracle within single-precision bounds, not bit
// for bit); packed FP32 instructions stay disabled.
#include "lbm_kernels_impl.h"

namespace lbm {

LBM_INSTANTIATE_FIELDS(float)
LBM_INSTANTIATE_POPS(float, float)

}  // namespace lbm
