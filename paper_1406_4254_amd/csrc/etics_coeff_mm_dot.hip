// etics_coeff_mm_dot.hip -- instantiations of the time-derivative coefficient kernels
// whose outer-product phase runs on the matrix cores (FP32 modes; etics_coeff_wg.hpp).
#include <hip/hip_runtime.h>

#include "etics_coeff_wg.hpp"

namespace etics {

int launch_coeff_mm_dual(const CoeffPlan& p, const CoeffArgs& a, int grid, hipStream_t st) {
  return launch_coeff_modes<false, true, true>(p, a, grid, st);
}
int launch_coeff_mm_dual(const CoeffPlan& p, const BatchedCoeffArgs& a, int grid, hipStream_t st) {
  return launch_coeff_modes<true, true, true>(p, a, grid, st);
}

}  // namespace etics
