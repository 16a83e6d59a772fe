// FP64 instantiation of the timestep kernels (lbm_kernels_impl.h) and the centre-of-mass reduction.
// Built without floating-point contraction: every FP64 expression is evaluated term by term in the
// order written, which is the order of the plain definitions.
#include "lbm_kernels_impl.h"

namespace lbm {

hipError_t launch_reduce(hipStream_t s, int tiling, int ndrop_total, const InstDev* inst, DropDev* drops,
                         const double* part, const uint64_t* mask, int64_t* step, int increment) {
  hipLaunchKernelGGL(k_reduce, dim3(ndrop_total > 0 ? ndrop_total : 1), dim3(NTHREADS), 0, s, tiling,
                     ndrop_total, inst, drops, part, mask, step, increment);
  return hipGetLastError();
}

LBM_INSTANTIATE_FIELDS(double)
LBM_INSTANTIATE_POPS(double, double)

}  // namespace lbm
