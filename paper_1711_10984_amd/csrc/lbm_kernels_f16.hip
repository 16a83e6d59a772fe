// Instantiation of the timestep kernels (lbm_kernels_impl.h) with FP32 arithmetic and fields and FP16
// population storage: each population is kept as its deviation f_i - w_i n0 from the rest state, rounded
// to FP16, and widened back to FP32 on load.  Built like the FP32 unit (fused multiply-add contraction,
// no packed FP32 instructions).
#include "lbm_kernels_impl.h"

namespace lbm {

LBM_INSTANTIATE_POPS(float, _Float16)

}  // namespace lbm
