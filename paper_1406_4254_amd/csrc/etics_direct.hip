// etics_direct.hip -- unsoftened direct-summation potential and acceleration (FP64).
//
// The accuracy study of the paper (Section 4.1) compares the expansion forces with
// direct summation, in double precision and without softening, and with the smooth
// force of the model.  For every particle i:
//   Phi_i = -sum_{j, r_ij > 0} m_j / r_ij,   a_i = sum_{j, r_ij > 0} m_j (x_j - x_i) / r_ij^3
// (G = 1).  The particle itself, and any other particle at exactly the same position,
// adds nothing.  One target particle per lane; the sources stream through LDS in tiles
// of 256 (x, y, z, m), read by every lane of the workgroup at the same address (a
// broadcast); each lane adds its sources in index order.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "etics_device.hpp"
#include "etics_internal.hpp"

namespace etics {

constexpr int kDirectThreads = 256;

__global__ __launch_bounds__(kDirectThreads) void direct_force_kernel(
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const double* __restrict__ m, int64_t n, int want_pot, int want_acc, double* __restrict__ pot,
    double* __restrict__ ax, double* __restrict__ ay, double* __restrict__ az) {
  __shared__ double4 src[kDirectThreads];
  const int t = threadIdx.x;
  const int64_t i = int64_t(blockIdx.x) * kDirectThreads + t;
  const bool valid = i < n;
  const double xi = valid ? x[i] : 0.0, yi = valid ? y[i] : 0.0, zi = valid ? z[i] : 0.0;
  double P = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
  for (int64_t j0 = 0; j0 < n; j0 += kDirectThreads) {
    const int64_t j = j0 + t;
    src[t] = j < n ? make_double4(x[j], y[j], z[j], m[j]) : make_double4(0.0, 0.0, 0.0, 0.0);
    __syncthreads();
    const int cnt = n - j0 < kDirectThreads ? int(n - j0) : kDirectThreads;
#pragma unroll 4
    for (int k = 0; k < cnt; ++k) {
      const double4 s = src[k];
      const double dx = s.x - xi, dy = s.y - yi, dz = s.z - zi;
      const double r2 = dx * dx + dy * dy + dz * dz;
      // the reciprocal square root runs for every pair (of 1 at zero separation), and
      // a select drops the pairs at zero separation: no branch in the loop
      const bool apart = r2 > 0.0;
      const double rs = rsqrt(apart ? r2 : 1.0);
      const double rinv = apart ? rs : 0.0;
      const double mr = s.w * rinv;
      const double mr3 = mr * rinv * rinv;
      P -= mr;
      gx += mr3 * dx;
      gy += mr3 * dy;
      gz += mr3 * dz;
    }
    __syncthreads();
  }
  if (!valid) return;
  if (want_pot) pot[i] = P;
  if (want_acc) {
    ax[i] = gx;
    ay[i] = gy;
    az[i] = gz;
  }
}

int launch_direct_force(const double* x, const double* y, const double* z, const double* m,
                        int64_t n, int outputs, double* pot, double* ax, double* ay, double* az,
                        hipStream_t st) {
  const int64_t blocks = (n + kDirectThreads - 1) / kDirectThreads;
  int rc = hook_before(st);
  if (rc) return rc;
  hipLaunchKernelGGL(direct_force_kernel, dim3(unsigned(blocks)), dim3(kDirectThreads), 0, st, x,
                     y, z, m, n, (outputs & ETICS_POT) ? 1 : 0, (outputs & ETICS_ACC) ? 1 : 0, pot,
                     ax, ay, az);
  rc = hip_fail(hipGetLastError(), "direct_force_kernel launch");
  return rc ? rc : hook_after(st);
}

}  // namespace etics
