// etics_force_synth.hpp -- the per-point synthesis of the SCF potential and
// acceleration from prepared coefficients, shared by the force kernels
// (etics_force.hip) and the jerk kernels (etics_jerk.hip).
//
// For each l the two radial recurrences (Gegenbauer in monic form, for the potential
// and for d/dr) run over n while the coefficients, the same for every lane, stream
// through the scalar cache into SGPR operands of the FMAs; the l and m loops are
// compile-time, so the recurrence and derivative constants are instruction literals.
// The angular synthesis uses division-free identities for dYbar/dtheta and
// m Ybar/sin(theta), and the result is rotated to Cartesian components.  The compute
// type may carry time derivatives (Dual), which turns the same code into the jerk.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "etics_device.hpp"
#include "etics_internal.hpp"

namespace etics {

static __constant__ BasisTables<float> g_tab32 = make_tables<float>();
static __constant__ BasisTables<double> g_tab64 = make_tables<double>();

template <typename T>
__device__ __forceinline__ const BasisTables<T>& tab();
template <>
__device__ __forceinline__ const BasisTables<float>& tab<float>() { return g_tab32; }
template <>
__device__ __forceinline__ const BasisTables<double>& tab<double>() { return g_tab64; }

// A prepared coefficient read through the constant address space (wave-uniform, so a
// scalar load into SGPR operands); a Dual one member by member
template <typename T>
__device__ __forceinline__ T cload(const __attribute__((address_space(4))) T* p) {
  return *p;
}
template <typename S>
__device__ __forceinline__ Dual<S> cload(const __attribute__((address_space(4))) Dual<S>* p) {
  return Dual<S>(p->v, p->d);
}
// ... or from a workgroup's copy in LDS: every lane reads the same address (a broadcast)
// into VGPR operands (FP64 and Dual, where each coefficient would take two SGPRs)
template <typename T>
__device__ __forceinline__ T cload(const __attribute__((address_space(3))) T* p) {
  return *p;
}
template <typename S>
__device__ __forceinline__ Dual<S> cload(const __attribute__((address_space(3))) Dual<S>* p) {
  return Dual<S>(p->v, p->d);
}
template <typename T>
using ConstPtr = const __attribute__((address_space(4))) T*;
template <typename T>
using LdsPtr = const __attribute__((address_space(3))) T*;

// Potential and acceleration (-grad Phi, Cartesian) at a point with spherical
// coordinates s, from one system's prepared coefficients cf.  T is the compute type,
// or Dual<S> to carry every quantity's time derivative along the motion (the jerk).
template <typename T>
struct ForceOut {
  T pot, gx, gy, gz;
};

// cf: the coefficients' four arrays, through the constant address space (ConstPtr) or
// in LDS (LdsPtr); laid out [4][K], or with QUAD [K][4] (the four values of a
// coefficient side by side, two 16-byte reads in FP64)
template <typename T, int LB, bool ACC, int BASIS, typename P = ConstPtr<T>, bool QUAD = false>
__device__ __forceinline__ ForceOut<T> synth_point(const Sph<T>& s, P cf, int K, int nmax, int lmax) {
  const int WK = QUAD ? 1 : K;      // offset from one array to the next
  constexpr int IS = QUAD ? 4 : 1;  // offset from one coefficient to the next
  using S = typename ScalarOf<T>::type;
  const BasisTables<S>& tb = tab<S>();
  const int L2 = (lmax + 1) * (lmax + 2) / 2;
  ForceOut<T> out{};
  {
    const T tu = s.t * s.u, u2 = s.u * s.u;
    // d/dr of the prefactor t^l u^(l+1) is l (t^l u^(l+1))/r - (2l+1) t^l u^(l+1) h, and
    // dxi/dr carries g (its constant is in the prepared coefficients):
    //   Hernquist-Ostriker h = u, g = u^2;  Clutton-Brock h = t u, g = t u^3
    const T hfac = BASIS == kBasisCB ? tu : s.u;
    const T gfac = BASIS == kBasisCB ? tu * u2 : u2;

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
      const P cfl = cf + l * (l + 1) / 2 * IS;
      T U[l + 1], V[l + 1], W[l + 1], X[l + 1];
#pragma unroll
      for (int m = 0; m <= l; ++m) {
        U[m] = cload(cfl + m * IS);
        V[m] = m > 0 ? cload(cfl + WK + m * IS) : T(0);
        W[m] = T(0);
        X[m] = T(0);
      }
      T c2 = T(0), c1 = T(1);  // Chat_{n-2}, Chat_{n-1} for n = 1 (Chat_{-1} enters times 0)
      T e2 = T(0), e1 = T(1);  // Ehat_{n-2}, Ehat_{n-1} (parameter a_l + 1)
      const S* ql = BASIS == kBasisCB ? tb.qcb[l] : tb.q[l];
      const S* qdl = BASIS == kBasisCB ? tb.qdcb[l] : tb.qd[l];
      // one radial order: c <- Chat_nn, accumulate, advance Ehat
      auto step = [&](int nn, T& cA, T& cB, T& eA, T& eB) {
        // on entry cA = Chat_{nn-2}, cB = Chat_{nn-1}; on exit cA = Chat_nn
        cA = s.xi * cB - ql[nn] * cA;
        const auto* cn = cfl + nn * L2 * IS;
#pragma unroll
        for (int m = 0; m <= l; ++m) {
          U[m] = fma_(cA, cload(cn + m * IS), U[m]);
          if (m > 0) V[m] = fma_(cA, cload(cn + WK + m * IS), V[m]);
        }
        if constexpr (ACC) {
          // eB = Ehat_{nn-1} is used, then eA <- Ehat_nn
#pragma unroll
          for (int m = 0; m <= l; ++m) {
            W[m] = fma_(eB, cload(cn + 2 * WK + m * IS), W[m]);
            if (m > 0) X[m] = fma_(eB, cload(cn + 3 * WK + m * IS), X[m]);
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
        const T dRl = T(l) * Ql - T(2 * l + 1) * Rl * hfac;  // d/dr (t^l u^(l+1))
        T ar = dRl * Pl + Rl * gfac * Gl;
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
    out.pot = accP;
    if constexpr (ACC) {
      out.gx = s.st * s.cp * accR + s.ct * s.cp * accT - s.sp * accF;
      out.gy = s.st * s.sp * accR + s.ct * s.sp * accT + s.cp * accF;
      out.gz = s.ct * accR - s.st * accT;
    }
  }
  return out;
}

}  // namespace etics
