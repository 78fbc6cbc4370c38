// etics_force.hip -- SCF potential and acceleration on gfx950 (MI355X).
//
// The second part of an SCF force calculation (paper Section 3.3): every particle's
// potential and acceleration from the coefficients A, B.  One particle per lane.
// For each l the two radial recurrences (Gegenbauer in monic form, for the
// potential and for d/dr) run over n while the coefficients, the same for every
// lane, stream through the scalar cache into SGPR operands of the FMAs; the l and m
// loops are compile-time, so the recurrence and derivative constants are instruction
// literals.  The angular synthesis uses division-free identities for dYbar/dtheta
// and m Ybar/sin(theta), and the result is rotated to Cartesian components.  No MFMA:
// the work is basis evaluation and short reductions with ragged shapes.
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
                                                            int nmax, int lmax, T* __restrict__ cf) {
  const int K = (nmax + 1) * (lmax + 1) * (lmax + 2) / 2;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const int L2 = (lmax + 1) * (lmax + 2) / 2;
  const int n = k / L2;
  const int lm = k - n * L2;
  int l = 0;
  while ((l + 1) * (l + 2) / 2 <= lm) ++l;
  const double al = 2.0 * l + 1.5;
  const double s4 = -2.0 * sqrt(kPi);
  const double su = s4 * gegen_k(n, al);
  const double sw = n >= 1 ? s4 * 4.0 * al * gegen_k(n - 1, al + 1.0) : 0.0;
  cf[k] = T(su * A[k]);
  cf[K + k] = T(su * B[k]);
  cf[2 * K + k] = T(sw * A[k]);
  cf[3 * K + k] = T(sw * B[k]);
}

// ------------------------------------------------------------------------ force
struct ForceArgs {
  const double *x, *y, *z;
  int64_t n;
  const void* cf;  // 4K prepared coefficients (T)
  double *pot, *ax, *ay, *az;
  int K, nmax, lmax;
  int want_pot;
};

template <typename T, int LB, bool ACC>
__global__ __launch_bounds__(256) void scf_force_kernel(const ForceArgs a) {
  const BasisTables<T>& tb = tab<T>();
  const T* __restrict__ cf = reinterpret_cast<const T*>(a.cf);
  const int K = a.K;
  const int L2 = (a.lmax + 1) * (a.lmax + 2) / 2;
  const int lmax = a.lmax;
  const int nmax = a.nmax;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n;
       i += int64_t(gridDim.x) * blockDim.x) {
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

      // radial sums over n: U,V (potential), W,X (radial derivative)
      T U[l + 1], V[l + 1], W[l + 1], X[l + 1];
#pragma unroll
      for (int m = 0; m <= l; ++m) {
        U[m] = T(0);
        V[m] = T(0);
        W[m] = T(0);
        X[m] = T(0);
      }
      T c2 = T(1), c1 = T(0);  // Chat_{n-2}, Chat_{n-1}
      T e2 = T(1), e1 = T(0);  // Ehat_{n-2}, Ehat_{n-1} (parameter a_l + 1)
      const T* cfl = cf + l * (l + 1) / 2;
      const T* ql = tb.q[l];
      const T* qdl = tb.qd[l];
      // one radial order: c <- Chat_nn, accumulate, advance Ehat
      auto step = [&](int nn, T& cA, T& cB, T& eA, T& eB) {
        // on entry cA = Chat_{nn-2}, cB = Chat_{nn-1}; on exit cA = Chat_nn
        cA = s.xi * cB - ql[nn] * cA;
        const T* cn = cfl + nn * L2;
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
        int nn = 0;
        for (; nn + 1 <= nmax; nn += 2) {
          step(nn, c2, c1, e2, e1);      // c2 <- Chat_nn, e2 <- Ehat_nn
          step(nn + 1, c1, c2, e1, e2);  // c1 <- Chat_{nn+1}, e1 <- Ehat_{nn+1}
        }
        if (nn <= nmax) step(nn, c2, c1, e2, e1);
      } else {
        // FP64 coefficients take two SGPRs each: one order per trip keeps them in SGPRs
        for (int nn = 0; nn <= nmax; ++nn) {
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
      a.ax[i] = double(gx);
      a.ay[i] = double(gy);
      a.az[i] = double(gz);
    }
  }
}

size_t force_prep_bytes(int nmax, int lmax, int prec) {
  return size_t(4) * coeff_count(nmax, lmax) * (prec == ETICS_FP64 ? 8 : 4);
}

namespace {
template <typename T, bool ACC>
int launch_force_lb(int lb, const ForceArgs& a, int grid, hipStream_t st) {
#define ETICS_FORCE_CASE(LBV)                                                         \
  case LBV:                                                                           \
    hipLaunchKernelGGL((scf_force_kernel<T, LBV, ACC>), dim3(grid), dim3(256), 0, st, a); \
    break;
  switch (lb) {
    ETICS_FORCE_CASE(2)
    ETICS_FORCE_CASE(4)
    ETICS_FORCE_CASE(6)
    ETICS_FORCE_CASE(8)
    ETICS_FORCE_CASE(10)
    ETICS_FORCE_CASE(12)
    ETICS_FORCE_CASE(14)
    default:
      set_error("internal: no force kernel bucket");
      return ETICS_EUNSUPPORTED;
  }
#undef ETICS_FORCE_CASE
  return hip_fail(hipGetLastError(), "scf_force_kernel launch");
}
}  // namespace

int launch_scf_force(const double* x, const double* y, const double* z, int64_t n, int nmax,
                     int lmax, const double* A, const double* B, int prec, int outputs,
                     double* pot, double* ax, double* ay, double* az, void* ws, hipStream_t st) {
  const int K = coeff_count(nmax, lmax);
  const bool f64 = prec == ETICS_FP64;
  const int pb = (K + 255) / 256;
  if (f64)
    hipLaunchKernelGGL(scf_force_prep_kernel<double>, dim3(pb), dim3(256), 0, st, A, B, nmax, lmax,
                       reinterpret_cast<double*>(ws));
  else
    hipLaunchKernelGGL(scf_force_prep_kernel<float>, dim3(pb), dim3(256), 0, st, A, B, nmax, lmax,
                       reinterpret_cast<float*>(ws));
  int rc = hip_fail(hipGetLastError(), "scf_force_prep_kernel launch");
  if (rc || n == 0) return rc;
  ForceArgs a{};
  a.x = x;
  a.y = y;
  a.z = z;
  a.n = n;
  a.cf = ws;
  a.pot = pot;
  a.ax = ax;
  a.ay = ay;
  a.az = az;
  a.K = K;
  a.nmax = nmax;
  a.lmax = lmax;
  a.want_pot = (outputs & ETICS_POT) ? 1 : 0;
  const int lb = lmax <= 2 ? 2 : (lmax + 1) / 2 * 2;
  int64_t grid = (n + 255) / 256;
  if (grid > 65536) grid = 65536;
  const bool acc = (outputs & ETICS_ACC) != 0;
  if (f64)
    return acc ? launch_force_lb<double, true>(lb, a, int(grid), st)
               : launch_force_lb<double, false>(lb, a, int(grid), st);
  return acc ? launch_force_lb<float, true>(lb, a, int(grid), st)
             : launch_force_lb<float, false>(lb, a, int(grid), st);
}

}  // namespace etics
