// etics_coeff_dot.hip -- time derivatives of the SCF coefficients along the particles'
// velocities, the first half of the jerk (the paper notes that Hernquist's SCF code
// computes the jerk, Section 3.4; the fourth-order Hermite scheme that uses it is named
// for SCF in Section 5.4):
//   dA_nlm/dt = (2 - delta_m0) Atilde_nl sum_k m_k d/dt [PhiT_nl(r_k) Ybar_lm(theta_k) cos(m phi_k)]
// along x_k(t) = x_k + v_k t, and dB/dt likewise with sin.  The coefficient kernels of
// etics_coeff_wg.hpp run with DUAL set (each particle gives two rows of a tile, see
// there), and the partial vectors go through the same fixed-order reductions, so the
// derivatives are scaled and ordered exactly as the coefficients are.
#include <hip/hip_runtime.h>

#include "etics_coeff_wg.hpp"
#include "etics_internal.hpp"

namespace etics {

int launch_scf_coeffs_dot(const CoeffPlan& p0, const double* x, const double* y, const double* z,
                          const double* vx, const double* vy, const double* vz, const double* m,
                          int64_t n, double* Ad, double* Bd, void* ws, hipStream_t st) {
  CoeffPlan p;
  if (!dot_plan(p0, n, &p)) {
    set_error("no tile plan for the coefficient time derivatives at these cutoffs");
    return ETICS_EUNSUPPORTED;
  }
  CoeffArgs a = coeff_args(p, x, y, z, m, n, p.tp / 2, ws);
  a.vx = vx;
  a.vy = vy;
  a.vz = vz;
  int rc = launch_coeff_any<false, true>(p, a, p.grid, st);
  if (rc) return rc;
  return launch_coeff_reduce(p, ws, p.grid, Ad, Bd, st);
}

int launch_scf_coeffs_dot_batched(const CoeffPlan& p0, const double* x, const double* y,
                                  const double* z, const double* vx, const double* vy,
                                  const double* vz, const double* m, const int64_t* offsets,
                                  const int* ustart, const int* usys, int nsys, int64_t ntotal,
                                  double* Ad, double* Bd, void* partials, hipStream_t st) {
  CoeffPlan p;
  if (!dot_plan(p0, ntotal, &p)) {
    set_error("no tile plan for the coefficient time derivatives at these cutoffs");
    return ETICS_EUNSUPPORTED;
  }
  BatchedCoeffArgs a = batched_coeff_args(p, x, y, z, m, offsets, ustart, usys, nsys, ntotal, partials);
  a.vx = vx;
  a.vy = vy;
  a.vz = vz;
  const int grid = coeff_grid(p, max_units(ntotal, nsys, p.unit));
  int rc = launch_coeff_any<true, true>(p, a, grid, st);
  if (rc) return rc;
  return launch_coeff_reduce_batched(p, partials, ustart, nsys, Ad, Bd, st);
}

}  // namespace etics
