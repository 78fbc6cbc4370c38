// etics_coeff_mm.hip -- instantiations of the coefficient kernels whose outer-product
// phase runs on the matrix cores (FP32 modes; the kernels are in etics_coeff_wg.hpp).
#include <hip/hip_runtime.h>

#include "etics_coeff_wg.hpp"

namespace etics {

int launch_coeff_mm(const CoeffPlan& p, const CoeffArgs& a, int grid, hipStream_t st) {
  return launch_coeff_modes<false, false, true>(p, a, grid, st);
}
int launch_coeff_mm(const CoeffPlan& p, const BatchedCoeffArgs& a, int grid, hipStream_t st) {
  return launch_coeff_modes<true, false, true>(p, a, grid, st);
}

}  // namespace etics
