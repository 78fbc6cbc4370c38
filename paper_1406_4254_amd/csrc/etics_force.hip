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
#include "etics_internal.hpp"

namespace etics {

__constant__ BasisTables<float> g_tab32 = make_tables<float>();
__constant__ BasisTables<double> g_tab64 = make_tables<double>();

template <typename T>
__device__ __forceinline__ const BasisTables<T>& tab();
template <>
__device__ __forceinline__ const BasisTables<float>& tab<float>() { return g_tab32; }
template <>
__device__ __forceinline__ const BasisTables<double>& tab<double>() { return g_tab64; }

// ------------------------------------------------------------------ force prep
// Coefficients rescaled for the force kernel, four arrays of K in compute precision:
//   [0,K)   -sqrt(4pi) k_n A          (potential / radial part, with monic C_n)
//   [K,2K)  -sqrt(4pi) k_n B
//   [2K,3K) -sqrt(4pi) 4 a_l k'_{n-1} A  (d/dr part: dC_n/dr = 4 a_l u^2 C_{n-1}^(a_l+1))
//   [3K,4K) -sqrt(4pi) 4 a_l k'_{n-1} B
template <typename T>
__global__ __launch_bounds__(256) void scf_force_prep_kernel(const double* __restrict__ A,
                                                            const double* __restrict__ B,
                                                            int nmax, int lmax, int nsys,
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
  const double al = 2.0 * l + 1.5;
  const double s4 = -2.0 * sqrt(kPi);
  const double su = s4 * gegen_k(n, al);
  const double sw = n >= 1 ? s4 * 4.0 * al * gegen_k(n - 1, al + 1.0) : 0.0;
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

// potential / acceleration of point i from one system's prepared coefficients cf
template <typename T, int LB, bool ACC>
__device__ __forceinline__ void force_point(const ForceArgs& a, const T* __restrict__ cf,
                                            int64_t i) {
  const BasisTables<T>& tb = tab<T>();
  const int K = a.K;
  const int L2 = (a.lmax + 1) * (a.lmax + 2) / 2;
  const int lmax = a.lmax;
  const int nmax = a.nmax;
  {
    const Sph<T> s = sph<T>(a.x[i], a.y[i], a.z[i]);
    const T tu = s.t * s.u, u2 = s.u * s.u;

    // cos/sin(m phi) by rotation
    T cm[LB + 1], sm[LB + 1];
    cm[0] = T(1);
    sm[0] = T(0);
#pragma unroll
    for (int m = 1; m <= LB; ++m) {
      cm[m] = cm[m - 1] * s.cp - sm[m - 1] * s.sp;
      sm[m] = sm[m - 1] * s.cp + cm[m - 1] * s.sp;
    }

    // Legendre rows; row l+1 is needed for m Ybar_lm / sin(theta)
    T Y[LB + 2][LB + 2];
    Y[0][0] = T(kTab.c1[0][0]);
    auto legendre_row = [&](auto rc) {
      constexpr int r = decltype(rc)::value;
      Y[r][r] = T(kTab.c1[r][r]) * s.st * Y[r - 1][r - 1];
      Y[r][r - 1] = T(kTab.c1[r][r - 1]) * s.ct * Y[r - 1][r - 1];
      static_for<(r >= 2 ? r - 1 : 0)>([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        Y[r][m] = (T(kTab.c1[r][m]) * s.ct) * Y[r - 1][m] - T(kTab.c2[r][m]) * Y[r - 2][m];
      });
    };

    T accP = T(0), accR = T(0), accT = T(0), accF = T(0);
    T Rl = s.u;      // t^l u^(l+1)
    T Rprev = T(0);  // t^(l-1) u^l
    static_for<LB + 1>([&](auto lc) {
      constexpr int l = decltype(lc)::value;
      if (l > lmax) return;
      if constexpr (ACC) {
        legendre_row(std::integral_constant<int, l + 1>{});
      } else if constexpr (l >= 1) {
        legendre_row(std::integral_constant<int, l>{});
      }

      // radial sums over n: U,V (potential), W,X (radial derivative).  Order 0 is taken
      // in closed form (Chat_0 = 1; it adds nothing to W, X since Ehat_{-1} = 0), the
      // loop starts at order 1.
      // the prepared coefficients are read-only here: through the constant address
      // space their wave-uniform loads become scalar loads into SGPR operands (for FP64
      // as well, where the generic pointer left the compiler with per-lane loads)
      const __attribute__((address_space(4))) T* cfl =
          (const __attribute__((address_space(4))) T*)(cf) + l * (l + 1) / 2;
      T U[l + 1], V[l + 1], W[l + 1], X[l + 1];
#pragma unroll
      for (int m = 0; m <= l; ++m) {
        U[m] = cfl[m];
        V[m] = m > 0 ? cfl[K + m] : T(0);
        W[m] = T(0);
        X[m] = T(0);
      }
      T c2 = T(0), c1 = T(1);  // Chat_{n-2}, Chat_{n-1} for n = 1 (Chat_{-1} enters times 0)
      T e2 = T(0), e1 = T(1);  // Ehat_{n-2}, Ehat_{n-1} (parameter a_l + 1)
      const T* ql = tb.q[l];
      const T* qdl = tb.qd[l];
      // one radial order: c <- Chat_nn, accumulate, advance Ehat
      auto step = [&](int nn, T& cA, T& cB, T& eA, T& eB) {
        // on entry cA = Chat_{nn-2}, cB = Chat_{nn-1}; on exit cA = Chat_nn
        cA = s.xi * cB - ql[nn] * cA;
        const auto* cn = cfl + nn * L2;
#pragma unroll
        for (int m = 0; m <= l; ++m) {
          U[m] = fma_(cA, cn[m], U[m]);
          if (m > 0) V[m] = fma_(cA, cn[K + m], V[m]);
        }
        if constexpr (ACC) {
          // eB = Ehat_{nn-1} is used, then eA <- Ehat_nn
#pragma unroll
          for (int m = 0; m <= l; ++m) {
            W[m] = fma_(eB, cn[2 * K + m], W[m]);
            if (m > 0) X[m] = fma_(eB, cn[3 * K + m], X[m]);
          }
          eA = s.xi * eB - qdl[nn] * eA;
        }
      };
      if constexpr (sizeof(T) == 4) {
        // two orders per trip: the recurrence registers swap roles instead of moving
        int nn = 1;
        for (; nn + 1 <= nmax; nn += 2) {
          step(nn, c2, c1, e2, e1);      // c2 <- Chat_nn, e2 <- Ehat_nn
          step(nn + 1, c1, c2, e1, e2);  // c1 <- Chat_{nn+1}, e1 <- Ehat_{nn+1}
        }
        if (nn <= nmax) step(nn, c2, c1, e2, e1);
      } else {
        // FP64 coefficients take two SGPRs each: one order per trip keeps them in SGPRs
        for (int nn = 1; nn <= nmax; ++nn) {
          step(nn, c2, c1, e2, e1);
          const T tc = c2, te = e2;
          c2 = c1;
          c1 = tc;
          e2 = e1;
          e1 = te;
        }
      }

      // angular synthesis for this l
      T Pl = T(0), Gl = T(0), Tl = T(0), Fl = T(0);
      static_for<l + 1>([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        const T ec = U[m] * cm[m] + V[m] * sm[m];
        Pl = fma_(Y[l][m], ec, Pl);
        if constexpr (ACC) {
          const T gc = W[m] * cm[m] + X[m] * sm[m];
          Gl = fma_(Y[l][m], gc, Gl);
          if constexpr (l >= 1) {
            T dY;
            if constexpr (m == 0) {
              dY = T(kTab.e1[l][0]) * Y[l][1];
            } else if constexpr (m + 1 <= l) {
              dY = T(kTab.e1[l][m]) * Y[l][m + 1] - T(kTab.e2[l][m]) * Y[l][m - 1];
            } else {
              dY = -T(kTab.e2[l][m]) * Y[l][m - 1];
            }
            Tl = fma_(dY, ec, Tl);
            if constexpr (m >= 1) {
              const T fc = V[m] * cm[m] - U[m] * sm[m];
              const T mYs = -(T(kTab.f1[l][m]) * Y[l + 1][m + 1] + T(kTab.f2[l][m]) * Y[l + 1][m - 1]);
              Fl = fma_(mYs, fc, Fl);
            }
          }
        }
      });
      accP = fma_(Rl, Pl, accP);
      if constexpr (ACC) {
        const T Ql = Rprev * u2;                             // t^(l-1) u^(l+2) = (t^l u^(l+1))/r
        const T dRl = T(l) * Ql - T(2 * l + 1) * Rl * s.u;   // d/dr (t^l u^(l+1))
        T ar = dRl * Pl + Rl * u2 * Gl;
        if constexpr (l == 0) {
          if (!(s.r > T(0))) ar = T(0);  // no direction at the origin
        }
        accR -= ar;
        if constexpr (l >= 1) {
          accT -= Ql * Tl;
          accF -= Ql * Fl;
        }
      }
      Rprev = Rl;
      Rl = Rl * tu;
    });
    if (a.want_pot) a.pot[i] = double(accP);
    if constexpr (ACC) {
      const T gx = s.st * s.cp * accR + s.ct * s.cp * accT - s.sp * accF;
      const T gy = s.st * s.sp * accR + s.ct * s.sp * accT + s.cp * accF;
      const T gz = s.ct * accR - s.st * accT;
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
}

template <typename T, int LB, bool ACC>
__global__ __launch_bounds__(256) void scf_force_kernel(const ForceArgs a) {
  const T* __restrict__ cf = reinterpret_cast<const T*>(a.cf);
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n;
       i += int64_t(gridDim.x) * blockDim.x)
    force_point<T, LB, ACC>(a, cf, i);
}

// batched systems: kForceSplit workgroups per unit of one system (each a contiguous
// part of it), so the coefficient pointer (and with it every coefficient operand) is
// uniform across the workgroup; splitting the coefficient kernel's units gives the
// force pass more workgroups
constexpr int kForceSplit = 4;

template <typename T, int LB, bool ACC>
__global__ __launch_bounds__(256) void scf_force_batched_kernel(const ForceArgs a,
                                                                const int64_t* __restrict__ offsets,
                                                                const int* __restrict__ ustart,
                                                                const int* __restrict__ usys,
                                                                int nsys) {
  const int u = blockIdx.x / kForceSplit;
  const int part = blockIdx.x % kForceSplit;
  if (u >= ustart[nsys]) return;
  const int sys = usys[u];
  int64_t b = offsets[sys], e = offsets[sys + 1];
  b = b < 0 ? 0 : (b > a.n ? a.n : b);
  e = e < b ? b : (e > a.n ? a.n : e);
  constexpr int64_t kPart = kUnitParticles / kForceSplit;
  const int64_t u0 = b + int64_t(u - ustart[sys]) * kUnitParticles;
  const int64_t ue0 = u0 + kUnitParticles < e ? u0 + kUnitParticles : e;
  const int64_t ub = u0 + part * kPart < ue0 ? u0 + part * kPart : ue0;
  const int64_t ue = ub + kPart < ue0 ? ub + kPart : ue0;
  const T* __restrict__ cf = reinterpret_cast<const T*>(a.cf) + size_t(sys) * 4 * a.K;
  for (int64_t i = ub + threadIdx.x; i < ue; i += blockDim.x) force_point<T, LB, ACC>(a, cf, i);
}

size_t force_prep_bytes(int nmax, int lmax, int prec) {
  return size_t(4) * coeff_count(nmax, lmax) * (prec == ETICS_FP64 ? 8 : 4);
}

namespace {

struct BatchInfo {
  const int64_t* offsets;
  const int* ustart;
  const int* usys;
  int nsys;
};

template <typename T, bool ACC, int LBV>
void launch_force_kernel(const ForceArgs& a, int grid, const BatchInfo* bi, hipStream_t st) {
  if (bi)
    hipLaunchKernelGGL((scf_force_batched_kernel<T, LBV, ACC>), dim3(grid), dim3(256), 0, st, a,
                       bi->offsets, bi->ustart, bi->usys, bi->nsys);
  else
    hipLaunchKernelGGL((scf_force_kernel<T, LBV, ACC>), dim3(grid), dim3(256), 0, st, a);
}

template <typename T, bool ACC>
int launch_force_lb(int lb, const ForceArgs& a, int grid, const BatchInfo* bi, hipStream_t st) {
  switch (lb) {
    case 2: launch_force_kernel<T, ACC, 2>(a, grid, bi, st); break;
    case 4: launch_force_kernel<T, ACC, 4>(a, grid, bi, st); break;
    case 6: launch_force_kernel<T, ACC, 6>(a, grid, bi, st); break;
    case 8: launch_force_kernel<T, ACC, 8>(a, grid, bi, st); break;
    case 10: launch_force_kernel<T, ACC, 10>(a, grid, bi, st); break;
    case 12: launch_force_kernel<T, ACC, 12>(a, grid, bi, st); break;
    case 14: launch_force_kernel<T, ACC, 14>(a, grid, bi, st); break;
    default:
      set_error("internal: no force kernel bucket");
      return ETICS_EUNSUPPORTED;
  }
  return hip_fail(hipGetLastError(), "scf_force_kernel launch");
}

int launch_prep(const double* A, const double* B, int nmax, int lmax, int nsys, int prec, void* ws,
                hipStream_t st) {
  const int K = coeff_count(nmax, lmax);
  const int pb = int((int64_t(nsys) * K + 255) / 256);
  if (prec == ETICS_FP64)
    hipLaunchKernelGGL(scf_force_prep_kernel<double>, dim3(pb), dim3(256), 0, st, A, B, nmax, lmax,
                       nsys, reinterpret_cast<double*>(ws));
  else
    hipLaunchKernelGGL(scf_force_prep_kernel<float>, dim3(pb), dim3(256), 0, st, A, B, nmax, lmax,
                       nsys, reinterpret_cast<float*>(ws));
  return hip_fail(hipGetLastError(), "scf_force_prep_kernel launch");
}

int launch_force_any(const ForceArgs& a, int prec, int outputs, int grid, const BatchInfo* bi,
                     hipStream_t st) {
  const int lb = a.lmax <= 2 ? 2 : (a.lmax + 1) / 2 * 2;
  const bool acc = (outputs & ETICS_ACC) != 0;
  int rc = hook_before(st);
  if (rc) return rc;
  if (prec == ETICS_FP64)
    rc = acc ? launch_force_lb<double, true>(lb, a, grid, bi, st)
             : launch_force_lb<double, false>(lb, a, grid, bi, st);
  else
    rc = acc ? launch_force_lb<float, true>(lb, a, grid, bi, st)
             : launch_force_lb<float, false>(lb, a, grid, bi, st);
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
                     double* pot, double* ax, double* ay, double* az, void* ws, hipStream_t st) {
  int rc = launch_prep(A, B, nmax, lmax, 1, prec, ws, st);
  if (rc || n == 0) return rc;
  const ForceArgs a = make_force_args(x, y, z, n, nmax, lmax, outputs, pot, ax, ay, az, ws);
  int64_t grid = (n + 255) / 256;
  if (grid > 65536) grid = 65536;
  return launch_force_any(a, prec, outputs, int(grid), nullptr, st);
}

int launch_scf_force_batched(const double* x, const double* y, const double* z,
                             const int64_t* offsets, const int* ustart, const int* usys, int nsys,
                             int64_t ntotal, int nmax, int lmax, const double* A, const double* B,
                             int prec, int outputs, double* pot, double* ax, double* ay,
                             double* az, void* prep, hipStream_t st, const LfUpdate* lf) {
  int rc = launch_prep(A, B, nmax, lmax, nsys, prec, prep, st);
  if (rc || ntotal == 0) return rc;
  ForceArgs a = make_force_args(x, y, z, ntotal, nmax, lmax, outputs, pot, ax, ay, az, prep);
  if (lf) a.lf = *lf;
  const BatchInfo bi{offsets, ustart, usys, nsys};
  return launch_force_any(a, prec, outputs, max_units(ntotal, nsys) * kForceSplit, &bi, st);
}

}  // namespace etics
