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

// Spherical coordinates of a point (expansion centre at the origin), with the
// radial variables of the Hernquist-Ostriker basis.
// r = 0 -> theta = 0; R = sqrt(x^2 + y^2) = 0 -> phi = 0.
template <typename T>
struct Sph {
  T r, ct, st, cp, sp, u, t, xi;
};

template <typename T>
__device__ __forceinline__ Sph<T> sph(double xd, double yd, double zd) {
  Sph<T> s;
  T x = T(xd), y = T(yd), z = T(zd);
  T R2 = x * x + y * y;
  T r2 = R2 + z * z;
  T R = sqrt_(R2);
  s.r = sqrt_(r2);
  T ir = s.r > T(0) ? rcp_(s.r) : T(0);
  T iR = R > T(0) ? rcp_(R) : T(0);
  s.ct = s.r > T(0) ? z * ir : T(1);
  s.st = R * ir;
  s.cp = R > T(0) ? x * iR : T(1);
  s.sp = y * iR;
  s.u = rcp_(T(1) + s.r);
  s.t = s.r * s.u;
  s.xi = s.t - s.u;
  return s;
}

}  // namespace etics
