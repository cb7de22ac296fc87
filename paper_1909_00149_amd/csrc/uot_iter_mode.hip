// Instantiations of the fused Algorithm-1 kernels (every residual variant,
// boundary/norm code and tile shape) and of the check kernel for one mode,
// UOT_MODE = 0 (DIST), 1 (PROX) or 2 (PROX_FIXED).  The build compiles this
// file once per mode, so the three sets compile in parallel.
#include "uot_iter_impl.hpp"

#ifndef UOT_MODE
#error "compile with -DUOT_MODE=0, 1 or 2"
#endif

#define UOT_CAT2(a, b) a##b
#define UOT_CAT(a, b) UOT_CAT2(a, b)

namespace uot {

hipError_t UOT_CAT(launch_iter_mode, UOT_MODE)(int resid, int bcn, int ty, int grid, const IterArgs& a,
                                               hipStream_t s) {
  return iter_res<UOT_MODE>(resid, bcn, ty, grid, a, s);
}

hipError_t UOT_CAT(iter_occupancy_mode, UOT_MODE)(int resid, int bcn, int ty, int* n) {
  return occ_res<UOT_MODE>(resid, bcn, ty, n);
}

hipError_t UOT_CAT(launch_iter_chk_mode, UOT_MODE)(int resid, int bcn, int ty, int grid, const IterArgs& a,
                                                   hipStream_t s) {
  const IterKernel k = chk_kernel<UOT_MODE>(resid, bcn, ty);
  if (!k) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k, dim3(grid), dim3(BLOCK), 0, s, a);
  return hipGetLastError();
}

hipError_t UOT_CAT(iter_chk_occupancy_mode, UOT_MODE)(int resid, int bcn, int ty, int* n) {
  const IterKernel k = chk_kernel<UOT_MODE>(resid, bcn, ty);
  if (!k) return hipErrorInvalidValue;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, k, BLOCK, 0);
}

hipError_t UOT_CAT(launch_check_mode, UOT_MODE)(int resid, int bcn, int grid, const CheckArgs& a, hipStream_t s) {
  return check_res<UOT_MODE>(resid, bcn, grid, a, s);
}

}  // namespace uot
