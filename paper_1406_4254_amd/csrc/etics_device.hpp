// etics_device.hpp -- device helpers shared by the SCF kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>

#include "etics_tables.hpp"

namespace etics {

// FP64 tables as compile-time constants: with compile-time (n, l, m) indices they
// become instruction literals.
constexpr BasisTables<double> kTab = make_tables<double>();

__device__ __forceinline__ float rcp_(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double rcp_(double v) { return 1.0 / v; }
// FP32: the hardware square root (about 1 ulp), without the correctly-rounded fix-up
__device__ __forceinline__ float sqrt_(float v) { return __builtin_amdgcn_sqrtf(v); }
__device__ __forceinline__ double sqrt_(double v) { return __builtin_sqrt(v); }
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

// compile-time loop: f(std::integral_constant<int, I>) for I = 0..N-1
template <typename F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

__device__ __forceinline__ float rsqrt_(float v) { return __builtin_amdgcn_rsqf(v); }
__device__ __forceinline__ double rsqrt_(double v) { return 1.0 / __builtin_sqrt(v); }

// Forward-mode derivative along the motion: a value v and its time derivative d.  The
// jerk kernels run the same basis and synthesis code on these instead of plain numbers,
// so every quantity carries its exact time derivative (product, chain and quotient
// rules below).  Comparisons look at the value only.
template <typename S>
struct Dual {
  S v, d;
  __device__ __forceinline__ Dual() = default;
  __device__ __forceinline__ constexpr Dual(S value, S deriv) : v(value), d(deriv) {}
  __device__ __forceinline__ constexpr explicit Dual(double c) : v(S(c)), d(S(0)) {}
  __device__ __forceinline__ constexpr explicit Dual(float c) : v(S(c)), d(S(0)) {}
  __device__ __forceinline__ constexpr explicit Dual(int c) : v(S(c)), d(S(0)) {}
};
template <typename S>
__device__ __forceinline__ Dual<S> operator+(Dual<S> a, Dual<S> b) { return {a.v + b.v, a.d + b.d}; }
template <typename S>
__device__ __forceinline__ Dual<S> operator-(Dual<S> a, Dual<S> b) { return {a.v - b.v, a.d - b.d}; }
template <typename S>
__device__ __forceinline__ Dual<S> operator-(Dual<S> a) { return {-a.v, -a.d}; }
template <typename S>
__device__ __forceinline__ Dual<S> operator*(Dual<S> a, Dual<S> b) {
  return {a.v * b.v, fma_(a.v, b.d, a.d * b.v)};
}
template <typename S>
__device__ __forceinline__ Dual<S> operator*(S c, Dual<S> a) { return {c * a.v, c * a.d}; }
template <typename S>
__device__ __forceinline__ Dual<S> operator*(Dual<S> a, S c) { return {a.v * c, a.d * c}; }
template <typename S>
__device__ __forceinline__ Dual<S>& operator+=(Dual<S>& a, Dual<S> b) { return a = a + b; }
template <typename S>
__device__ __forceinline__ Dual<S>& operator-=(Dual<S>& a, Dual<S> b) { return a = a - b; }
template <typename S>
__device__ __forceinline__ bool operator>(Dual<S> a, Dual<S> b) { return a.v > b.v; }
template <typename S>
__device__ __forceinline__ Dual<S> fma_(Dual<S> a, Dual<S> b, Dual<S> c) {
  return {fma_(a.v, b.v, c.v), fma_(a.v, b.d, fma_(a.d, b.v, c.d))};
}
template <typename S>
__device__ __forceinline__ Dual<S> rcp_(Dual<S> a) {
  const S q = rcp_(a.v);
  return {q, -a.d * q * q};
}
// at a zero value the derivative is taken as 0 (the direction of the motion there is
// not a property of the point)
template <typename S>
__device__ __forceinline__ Dual<S> sqrt_(Dual<S> a) {
  const S q = sqrt_(a.v);
  return {q, a.v > S(0) ? S(0.5) * a.d * rcp_(q) : S(0)};
}
template <typename S>
__device__ __forceinline__ Dual<S> rsqrt_(Dual<S> a) {
  const S q = rsqrt_(a.v);
  return {q, S(-0.5) * a.d * q * q * q};
}

template <typename T>
struct ScalarOf {
  using type = T;
};
template <typename S>
struct ScalarOf<Dual<S>> {
  using type = S;
};

// Spherical coordinates of a point (expansion centre at the origin), with the
// radial variables u, t = r u and xi of radial basis BASIS:
//   Hernquist-Ostriker: u = 1/(1+r), xi = t - u;  Clutton-Brock: u = 1/sqrt(1+r^2),
//   xi = t^2 - u^2.
// r = 0 -> theta = 0; R = sqrt(x^2 + y^2) = 0 -> phi = 0.
template <typename T>
struct Sph {
  T r, ct, st, cp, sp, u, t, xi;
};

template <typename V, int BASIS = kBasisHO>
__device__ __forceinline__ Sph<V> sph_v(V x, V y, V z) {
  Sph<V> s;
  V R2 = x * x + y * y;
  V r2 = R2 + z * z;
  V R = sqrt_(R2);
  s.r = sqrt_(r2);
  V ir = s.r > V(0) ? rcp_(s.r) : V(0);
  V iR = R > V(0) ? rcp_(R) : V(0);
  s.ct = s.r > V(0) ? z * ir : V(1);
  s.st = R * ir;
  s.cp = R > V(0) ? x * iR : V(1);
  s.sp = y * iR;
  if constexpr (BASIS == kBasisCB) {
    s.u = rsqrt_(V(1) + r2);
    s.t = s.r * s.u;
    s.xi = (s.t - s.u) * (s.t + s.u);
  } else {
    s.u = rcp_(V(1) + s.r);
    s.t = s.r * s.u;
    s.xi = s.t - s.u;
  }
  return s;
}

template <typename T, int BASIS = kBasisHO>
__device__ __forceinline__ Sph<T> sph(double xd, double yd, double zd) {
  return sph_v<T, BASIS>(T(xd), T(yd), T(zd));
}

// the same with the time derivatives along the velocity (vx, vy, vz)
template <typename S, int BASIS = kBasisHO>
__device__ __forceinline__ Sph<Dual<S>> sph_dual(double xd, double yd, double zd, double vxd,
                                                 double vyd, double vzd) {
  return sph_v<Dual<S>, BASIS>(Dual<S>(S(xd), S(vxd)), Dual<S>(S(yd), S(vyd)), Dual<S>(S(zd), S(vzd)));
}

}  // namespace etics
