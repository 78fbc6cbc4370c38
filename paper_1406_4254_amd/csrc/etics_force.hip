// etics_force.hip -- SCF potential and acceleration on gfx950 (MI355X).
//
// The second part of an SCF force calculation (paper Section 3.3): every particle's
// potential and acceleration from the coefficients A, B.  One particle per lane.
// For each l the two radial recurrences (Gegenbauer in monic form, for the
// potential and for d/dr) run over n while the coefficients, the same for every
// lane, stream through the scalar cache into SGPR operands of the FMAs; the l and m
// loops are compile-time, so the recurrence and derivative constants are instruction
// literals.  The angular synthesis uses division-free identities for dYbar/dtheta
// and m Ybar/sin(theta), and the result is rotated to Cartesian components.  In the
// batched leapfrog the epilogue applies the kicks (and drift) to the particle instead
// of storing its acceleration.  No MFMA: the work is basis evaluation and short
// reductions with ragged shapes.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "etics_device.hpp"
#include "etics_force_synth.hpp"
#include "etics_internal.hpp"

namespace etics {

// ------------------------------------------------------------------ force prep
// Coefficients rescaled for the force kernel, four arrays of K in compute precision:
//   [0,K)   -sqrt(4pi) k_n A          (potential / radial part, with monic C_n)
//   [K,2K)  -sqrt(4pi) k_n B
//   [2K,3K) -sqrt(4pi) 2 a_l c k'_{n-1} A  (d/dr part: dC_n^(a)/dxi = 2a C_{n-1}^(a+1))
//   [3K,4K) -sqrt(4pi) 2 a_l c k'_{n-1} B
// where dxi/dr = c g(r): Hernquist-Ostriker c = 2, g = u^2; Clutton-Brock c = 4,
// g = t u^3 (g is applied per particle by the force kernel).
template <typename T>
__global__ __launch_bounds__(256) void scf_force_prep_kernel(const double* __restrict__ A,
                                                            const double* __restrict__ B,
                                                            int nmax, int lmax, int nsys, int basis,
                                                            T* __restrict__ cf) {
  const int K = (nmax + 1) * (lmax + 1) * (lmax + 2) / 2;
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= int64_t(nsys) * K) return;
  const int sys = int(g / K);
  const int k = int(g - int64_t(sys) * K);
  const int L2 = (lmax + 1) * (lmax + 2) / 2;
  const int n = k / L2;
  const int lm = k - n * L2;
  int l = 0;
  while ((l + 1) * (l + 2) / 2 <= lm) ++l;
  const double al = basis_alpha(basis, l);
  const double dxi_c = basis == kBasisCB ? 4.0 : 2.0;
  const double s4 = -2.0 * sqrt(kPi);
  const double su = s4 * gegen_k(n, al);
  const double sw = n >= 1 ? s4 * 2.0 * al * dxi_c * gegen_k(n - 1, al + 1.0) : 0.0;
  const double a = A[g], b = B[g];
  T* c = cf + size_t(sys) * 4 * K;
  c[k] = T(su * a);
  c[K + k] = T(su * b);
  c[2 * K + k] = T(sw * a);
  c[3 * K + k] = T(sw * b);
}

// ------------------------------------------------------------------------ force
struct ForceArgs {
  const double *x, *y, *z;
  int64_t n;
  const void* cf;  // 4K prepared coefficients (T)
  double *pot, *ax, *ay, *az;
  int K, nmax, lmax;
  int want_pot;
  LfUpdate lf;     // lf.mode = 0: write a; otherwise update v (and x) instead
};

// the outputs of point i: potential and acceleration, or the leapfrog update
template <typename T, bool ACC>
__device__ __forceinline__ void force_store(const ForceArgs& a, int64_t i, T pot, T gx, T gy, T gz) {
  if (a.want_pot) a.pot[i] = double(pot);
  if constexpr (ACC) {
    if (a.lf.mode == 0) {
      a.ax[i] = double(gx);
      a.ay[i] = double(gy);
      a.az[i] = double(gz);
    } else {
      // leapfrog: closing kick, then (mode 2) the next step's opening kick and drift;
      // only this thread touches particle i, so x is updated in place after its use
      const double h = a.lf.h;
      double vx = __builtin_fma(h, double(gx), a.lf.vx[i]);
      double vy = __builtin_fma(h, double(gy), a.lf.vy[i]);
      double vz = __builtin_fma(h, double(gz), a.lf.vz[i]);
      if (a.lf.mode == 2) {
        vx = __builtin_fma(h, double(gx), vx);
        vy = __builtin_fma(h, double(gy), vy);
        vz = __builtin_fma(h, double(gz), vz);
        a.lf.x[i] = __builtin_fma(a.lf.dt, vx, a.x[i]);
        a.lf.y[i] = __builtin_fma(a.lf.dt, vy, a.y[i]);
        a.lf.z[i] = __builtin_fma(a.lf.dt, vz, a.z[i]);
      }
      a.lf.vx[i] = vx;
      a.lf.vy[i] = vy;
      a.lf.vz[i] = vz;
    }
  }
}

// potential / acceleration of point i from one system's prepared coefficients cf
template <typename T, int LB, bool ACC, int BASIS = kBasisHO>
__device__ __forceinline__ void force_point(const ForceArgs& a, const T* __restrict__ cf,
                                            int64_t i) {
  const Sph<T> s = sph<T, BASIS>(a.x[i], a.y[i], a.z[i]);
  const ForceOut<T> o = synth_point<T, LB, ACC, BASIS>(s, ConstPtr<T>(cf), a.K, a.nmax, a.lmax);
  force_store<T, ACC>(a, i, o.pot, o.gx, o.gy, o.gz);
}

template <typename T, int LB, bool ACC, int BASIS>
__global__ __launch_bounds__(256) void scf_force_kernel(const ForceArgs a) {
  const T* __restrict__ cf = reinterpret_cast<const T*>(a.cf);
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n;
       i += int64_t(gridDim.x) * blockDim.x)
    force_point<T, LB, ACC, BASIS>(a, cf, i);
}

// FP64: the workgroup copies the prepared coefficients to LDS once, as [K][4], and every
// lane reads them as broadcast VGPR operands (as SGPR operands each FP64 coefficient
// takes two SGPRs and the n loop's set overflows them); a grid of a few workgroups per
// CU, each walking many points, keeps the copies few.
template <int LB, bool ACC, int BASIS>
__global__ __launch_bounds__(256) void scf_force_lds_kernel(const ForceArgs a) {
  extern __shared__ __align__(16) double lds_cf[];
  const double* __restrict__ cf = reinterpret_cast<const double*>(a.cf);
  for (int i = threadIdx.x; i < 4 * a.K; i += blockDim.x) {
    const int which = i / a.K, idx = i - which * a.K;
    lds_cf[4 * idx + which] = cf[i];
  }
  __syncthreads();
  const LdsPtr<double> src = (LdsPtr<double>)(lds_cf);
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const Sph<double> s = sph<double, BASIS>(a.x[i], a.y[i], a.z[i]);
    const ForceOut<double> o =
        synth_point<double, LB, ACC, BASIS, LdsPtr<double>, true>(s, src, a.K, a.nmax, a.lmax);
    force_store<double, ACC>(a, i, o.pot, o.gx, o.gy, o.gz);
  }
}

// batched systems: `split` workgroups per unit of `unit` particles of one system (each a
// contiguous part of it), so the coefficient pointer (and with it every coefficient
// operand) is uniform across the workgroup; splitting the coefficient kernel's units
// gives the force pass more workgroups.  The system's prepared coefficients are copied
// to LDS as [K][4] first, as in scf_force_lds_kernel, and read as broadcast VGPR
// operands (measured faster than SGPR operands here in FP32 too).
template <typename T, int LB, bool ACC>
__global__ __launch_bounds__(256) void scf_force_batched_kernel(const ForceArgs a,
                                                                const int64_t* __restrict__ offsets,
                                                                const int* __restrict__ ustart,
                                                                const int* __restrict__ usys,
                                                                int nsys, int unit, int split) {
  extern __shared__ __align__(16) double lds_cf[];
  const int u = blockIdx.x / split;
  const int part = blockIdx.x % split;
  if (u >= ustart[nsys]) return;
  const int sys = usys[u];
  int64_t b = offsets[sys], e = offsets[sys + 1];
  b = b < 0 ? 0 : (b > a.n ? a.n : b);
  e = e < b ? b : (e > a.n ? a.n : e);
  const int64_t kPart = (unit + split - 1) / split;
  const int64_t u0 = b + int64_t(u - ustart[sys]) * unit;
  const int64_t ue0 = u0 + unit < e ? u0 + unit : e;
  const int64_t ub = u0 + part * kPart < ue0 ? u0 + part * kPart : ue0;
  const int64_t ue = ub + kPart < ue0 ? ub + kPart : ue0;
  const T* __restrict__ cf = reinterpret_cast<const T*>(a.cf) + size_t(sys) * 4 * a.K;
  T* lds_t = reinterpret_cast<T*>(lds_cf);
  for (int i = threadIdx.x; i < 4 * a.K; i += blockDim.x) {
    const int which = i / a.K, idx = i - which * a.K;
    lds_t[4 * idx + which] = cf[i];
  }
  __syncthreads();
  const LdsPtr<T> src = (LdsPtr<T>)(lds_t);
  for (int64_t i = ub + threadIdx.x; i < ue; i += blockDim.x) {
    const Sph<T> s = sph<T, kBasisHO>(a.x[i], a.y[i], a.z[i]);
    const ForceOut<T> o = synth_point<T, LB, ACC, kBasisHO, LdsPtr<T>, true>(s, src, a.K, a.nmax, a.lmax);
    force_store<T, ACC>(a, i, o.pot, o.gx, o.gy, o.gz);
  }
}

size_t force_prep_bytes(int nmax, int lmax, int prec) {
  return size_t(4) * coeff_count(nmax, lmax) * (prec == ETICS_FP64 ? 8 : 4);
}

namespace {

struct BatchInfo {
  const int64_t* offsets;
  const int* ustart;
  const int* usys;
  int nsys, unit, split;
};

// the whole 160 KiB of a CU may be requested as dynamic LDS (the largest cutoffs' FP64
// coefficients take 80 KiB); hipFuncSetAttribute once per kernel (failures surface at
// the launch)
void set_lds_limit(const void* kfn) {
  (void)hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

template <typename T, bool ACC, int LBV>
void launch_force_kernel(const ForceArgs& a, int basis, int grid, const BatchInfo* bi,
                         hipStream_t st) {
  if (bi) {
    const size_t lds = size_t(4) * a.K * sizeof(T);
    if (lds) set_lds_limit(reinterpret_cast<const void*>(scf_force_batched_kernel<T, LBV, ACC>));
    hipLaunchKernelGGL((scf_force_batched_kernel<T, LBV, ACC>), dim3(grid), dim3(256), lds, st, a,
                       bi->offsets, bi->ustart, bi->usys, bi->nsys, bi->unit, bi->split);
  } else if constexpr (sizeof(T) == 8) {
    // a few workgroups per CU, each with the coefficients in LDS
    const size_t lds = size_t(4) * a.K * sizeof(double);
    const int g = grid < 1024 ? grid : 1024;
    if (basis == kBasisCB) {
      set_lds_limit(reinterpret_cast<const void*>(scf_force_lds_kernel<LBV, ACC, kBasisCB>));
      hipLaunchKernelGGL((scf_force_lds_kernel<LBV, ACC, kBasisCB>), dim3(g), dim3(256), lds, st, a);
    } else {
      set_lds_limit(reinterpret_cast<const void*>(scf_force_lds_kernel<LBV, ACC, kBasisHO>));
      hipLaunchKernelGGL((scf_force_lds_kernel<LBV, ACC, kBasisHO>), dim3(g), dim3(256), lds, st, a);
    }
  } else if (basis == kBasisCB)
    hipLaunchKernelGGL((scf_force_kernel<T, LBV, ACC, kBasisCB>), dim3(grid), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((scf_force_kernel<T, LBV, ACC, kBasisHO>), dim3(grid), dim3(256), 0, st, a);
}

template <typename T, bool ACC>
int launch_force_lb(int lb, const ForceArgs& a, int basis, int grid, const BatchInfo* bi,
                    hipStream_t st) {
  switch (lb) {
    case 2: launch_force_kernel<T, ACC, 2>(a, basis, grid, bi, st); break;
    case 4: launch_force_kernel<T, ACC, 4>(a, basis, grid, bi, st); break;
    case 6: launch_force_kernel<T, ACC, 6>(a, basis, grid, bi, st); break;
    case 8: launch_force_kernel<T, ACC, 8>(a, basis, grid, bi, st); break;
    case 10: launch_force_kernel<T, ACC, 10>(a, basis, grid, bi, st); break;
    case 12: launch_force_kernel<T, ACC, 12>(a, basis, grid, bi, st); break;
    case 14: launch_force_kernel<T, ACC, 14>(a, basis, grid, bi, st); break;
    default:
      set_error("internal: no force kernel bucket");
      return ETICS_EUNSUPPORTED;
  }
  return hip_fail(hipGetLastError(), "scf_force_kernel launch");
}

int launch_prep(const double* A, const double* B, int nmax, int lmax, int nsys, int prec, int basis,
                void* ws, hipStream_t st) {
  const int K = coeff_count(nmax, lmax);
  const int pb = int((int64_t(nsys) * K + 255) / 256);
  if (prec == ETICS_FP64)
    hipLaunchKernelGGL(scf_force_prep_kernel<double>, dim3(pb), dim3(256), 0, st, A, B, nmax, lmax,
                       nsys, basis, reinterpret_cast<double*>(ws));
  else
    hipLaunchKernelGGL(scf_force_prep_kernel<float>, dim3(pb), dim3(256), 0, st, A, B, nmax, lmax,
                       nsys, basis, reinterpret_cast<float*>(ws));
  return hip_fail(hipGetLastError(), "scf_force_prep_kernel launch");
}

int launch_force_any(const ForceArgs& a, int prec, int outputs, int basis, int grid,
                     const BatchInfo* bi, hipStream_t st) {
  const int lb = a.lmax <= 2 ? 2 : (a.lmax + 1) / 2 * 2;
  const bool acc = (outputs & ETICS_ACC) != 0;
  int rc = hook_before(st);
  if (rc) return rc;
  if (prec == ETICS_FP64)
    rc = acc ? launch_force_lb<double, true>(lb, a, basis, grid, bi, st)
             : launch_force_lb<double, false>(lb, a, basis, grid, bi, st);
  else
    rc = acc ? launch_force_lb<float, true>(lb, a, basis, grid, bi, st)
             : launch_force_lb<float, false>(lb, a, basis, grid, bi, st);
  return rc ? rc : hook_after(st);
}

ForceArgs make_force_args(const double* x, const double* y, const double* z, int64_t n, int nmax,
                          int lmax, int outputs, double* pot, double* ax, double* ay, double* az,
                          const void* cf) {
  ForceArgs a{};
  a.x = x;
  a.y = y;
  a.z = z;
  a.n = n;
  a.cf = cf;
  a.pot = pot;
  a.ax = ax;
  a.ay = ay;
  a.az = az;
  a.K = coeff_count(nmax, lmax);
  a.nmax = nmax;
  a.lmax = lmax;
  a.want_pot = (outputs & ETICS_POT) ? 1 : 0;
  return a;
}

}  // namespace

int launch_scf_force(const double* x, const double* y, const double* z, int64_t n, int nmax,
                     int lmax, const double* A, const double* B, int prec, int outputs,
                     double* pot, double* ax, double* ay, double* az, void* ws, hipStream_t st,
                     int basis) {
  int rc = launch_prep(A, B, nmax, lmax, 1, prec, basis, ws, st);
  if (rc || n == 0) return rc;
  const ForceArgs a = make_force_args(x, y, z, n, nmax, lmax, outputs, pot, ax, ay, az, ws);
  int64_t grid = (n + 255) / 256;
  if (grid > 65536) grid = 65536;
  return launch_force_any(a, prec, outputs, basis, int(grid), nullptr, st);
}

int launch_scf_force_batched(const CoeffPlan& plan, const double* x, const double* y,
                             const double* z, const int64_t* offsets, const int* ustart,
                             const int* usys, int nsys, int64_t ntotal, const double* A,
                             const double* B, int outputs, double* pot, double* ax, double* ay,
                             double* az, void* prep, hipStream_t st, const LfUpdate* lf) {
  const int nmax = plan.nmax, lmax = plan.lmax, prec = plan.prec;
  int rc = launch_prep(A, B, nmax, lmax, nsys, prec, kBasisHO, prep, st);
  if (rc || ntotal == 0) return rc;
  ForceArgs a = make_force_args(x, y, z, ntotal, nmax, lmax, outputs, pot, ax, ay, az, prep);
  if (lf) a.lf = *lf;
  const BatchInfo bi{offsets, ustart, usys, nsys, plan.unit, plan.split};
  return launch_force_any(a, prec, outputs, kBasisHO, max_units(ntotal, nsys, plan.unit) * plan.split,
                          &bi, st);
}

}  // namespace etics
