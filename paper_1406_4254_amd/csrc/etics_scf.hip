// etics_scf.hip -- SCF coefficient and force kernels for gfx950 (MI355X).
//
// The SCF force calculation (paper Section 3.3) has two parts: (1) the expansion
// coefficients, a sum over all particles of basis-function products, and (2) the
// potential and acceleration of every particle from those coefficients.
//
// (1) scf_coeff_kernel: each workgroup (4 wavefronts) walks tiles of `tp`
//     particles.  Phase 1 evaluates each particle's basis once, one particle per
//     lane, with the basis split into independent jobs shared out between the four
//     wavefronts (a radial job is the Gegenbauer column of one l, an angular job the
//     Legendre column of one m); the values go to LDS.  Phase 2 is an outer-product
//     accumulation over the tile: every lane owns an nb x bs register block of
//     coefficients (radial orders x angular slots of one l) and accumulates the
//     products of the LDS-staged radial and angular values.  FP32 partial sums are
//     folded into FP64 (or compensated double-float) accumulators every few tiles.
//     At the end the lanes that own the same block (one per "stream") are combined in
//     a fixed order and the workgroup writes one partial coefficient vector.
//     scf_reduce_kernel sums the partials over workgroups in a fixed order and
//     applies the normalisation (2 - delta_m0) Atilde_nl and the basis constants.
//     The result does not depend on how the hardware schedules workgroups.
// (2) scf_force_kernel: one particle per lane.  For each l the radial recurrences
//     run over n while the coefficients, identical for every lane, stream through
//     the scalar cache into SGPR operands of the FMAs; the angular synthesis and
//     the spherical-to-Cartesian transform follow.  No MFMA: the work is basis
//     evaluation and reductions with ragged shapes, not a dense contraction.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

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

__device__ __forceinline__ float rcp_(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double rcp_(double v) { return 1.0 / v; }
__device__ __forceinline__ float sqrt_(float v) { return __builtin_sqrtf(v); }
__device__ __forceinline__ double sqrt_(double v) { return __builtin_sqrt(v); }

// Spherical coordinates of a point (expansion centre at the origin).
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

// ------------------------------------------------------------------ coefficients
struct CoeffArgs {
  const double *x, *y, *z, *m;
  int64_t n;
  void* partials;  // [grid][2K] FP64 (or double-float pairs)
  int K, nmax, lmax, tp, nrow, spg, spz, nblocks, streams, flush_tiles, ntiles, nchunks;
  int zoff[LCAP + 2];
  int njobs[4];
  unsigned char jobs[4][kMaxJobs];  // bit 7 set: radial job for l; else angular job for m
};

// angular slot of (m, cos|sin) inside one l: m=0 cos -> 0, (m,cos) -> 2m-1, (m,sin) -> 2m
__device__ __forceinline__ int slot_cos(int m) { return m == 0 ? 0 : 2 * m - 1; }

// wide accumulator: MODE 0 -> FP64; MODE 1 -> compensated FP32 pair (hi, lo)
template <typename T, int MODE>
struct Wide;
template <>
struct Wide<float, 0> {
  double v = 0.0;
  __device__ void add(float a) { v += double(a); }
};
template <>
struct Wide<float, 1> {
  float hi = 0.f, lo = 0.f;
  __device__ void add(float a) {  // Knuth TwoSum, error carried in lo
    float s = hi + a;
    float bb = s - hi;
    float err = (hi - (s - bb)) + (a - bb);
    hi = s;
    lo += err;
  }
};
template <>
struct Wide<double, 0> {
  double v = 0.0;
  __device__ void add(double a) { v += a; }
};

// partial entry type and combination for the fixed-order stream merge
template <int MODE>
struct PartialT;
template <>
struct PartialT<0> {
  using type = double;
};
template <>
struct PartialT<1> {
  using type = float2;
};

__device__ __forceinline__ double wide_value(const Wide<float, 0>& w) { return w.v; }
__device__ __forceinline__ double wide_value(const Wide<double, 0>& w) { return w.v; }
__device__ __forceinline__ float2 wide_value(const Wide<float, 1>& w) { return make_float2(w.hi, w.lo); }

__device__ __forceinline__ double merge(double a, double b) { return a + b; }
__device__ __forceinline__ float2 merge(float2 a, float2 b) {  // double-float addition
  float s = a.x + b.x;
  float bb = s - a.x;
  float err = (a.x - (s - bb)) + (b.x - bb);
  err += a.y + b.y;
  float hi = s + err;
  float lo = err - (hi - s);
  return make_float2(hi, lo);
}

template <typename T, int NB, int BS, int MODE>
__global__ __launch_bounds__(kCoeffThreads, 2) void scf_coeff_kernel(const CoeffArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* G = reinterpret_cast<T*>(lds_raw);  // [tp][spg]   radial values, rows of nrow per l
  T* Z = G + a.tp * a.spg;               // [tp][spz]   angular values x mass x radial prefactor
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const BasisTables<T>& tb = tab<T>();

  // register block owned by this thread
  const int my_stream = tid / a.nblocks;
  const int my_block = tid - my_stream * a.nblocks;
  const bool active = my_stream < a.streams;
  int bl = 0, n0 = 0, s0 = 0;
  {
    int b = my_block;
    for (int l = 0; l <= a.lmax; ++l) {
      int nsc = (a.zoff[l + 1] - a.zoff[l]) / BS;
      int cnt = a.nchunks * nsc;
      if (b < cnt) {
        bl = l;
        n0 = (b / nsc) * NB;
        s0 = (b % nsc) * BS;
        break;
      }
      b -= cnt;
    }
  }

  T acc[NB][BS];
  Wide<T, MODE> wide[NB][BS];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < BS; ++j) acc[i][j] = T(0);

  // angular padding slots are never written by phase 1 and must read as zero
  for (int i = tid; i < a.tp * a.spz; i += kCoeffThreads) Z[i] = T(0);
  __syncthreads();

  int tcount = 0;
  for (int tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    // ---------------- phase 1: basis of the tile's particles (one per lane)
    if (lane < a.tp) {
      const int64_t pi = int64_t(tile) * a.tp + lane;
      const bool valid = pi < a.n;
      const double xd = valid ? a.x[pi] : 0.0, yd = valid ? a.y[pi] : 0.0;
      const double zd = valid ? a.z[pi] : 0.0, md = valid ? a.m[pi] : 0.0;
      const Sph<T> s = sph<T>(xd, yd, zd);
      const T tu = s.t * s.u, ctu = s.ct * tu, tu2 = tu * tu, stu = s.st * tu;
      T* Gp = G + lane * a.spg;
      T* Zp = Z + lane * a.spz;
      // angular-job state: diagonal value mass u (tu)^m Ybar_mm and (cos, sin)(m phi)
      int mcur = 0;
      T Pd = T(md) * s.u * tb.c1[0][0];
      T cmc = T(1), smc = T(0);
      const int nj = a.njobs[wave];
      for (int j = 0; j < nj; ++j) {
        const int job = a.jobs[wave][j];
        if (job & 0x80) {
          // radial job: monic Gegenbauer Chat_n^(2l+3/2)(xi), n = 0..nrow-1 (0 past nmax)
          const int l = job & 0x7f;
          T p2 = T(1), p1 = T(0);
          T* row = Gp + l * a.nrow;
          for (int nb4 = 0; nb4 < a.nrow; nb4 += 4) {
            T v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int nn = nb4 + q;
              const int nc = nn <= a.nmax ? nn : 0;
              T c = s.xi * p1 - tb.q[l][nc] * p2;
              c = nn <= a.nmax ? c : T(0);
              p2 = p1;
              p1 = c;
              v[q] = c;
            }
            if constexpr (sizeof(T) == 4) {
              *reinterpret_cast<float4*>(row + nb4) = make_float4(v[0], v[1], v[2], v[3]);
            } else {
              *reinterpret_cast<double2*>(row + nb4) = make_double2(v[0], v[1]);
              *reinterpret_cast<double2*>(row + nb4 + 2) = make_double2(v[2], v[3]);
            }
          }
        } else {
          // angular job: column m of mass u (tu)^l Ybar_lm (cos, sin)(m phi), l = m..lmax
          const int mm = job;
          while (mcur < mm) {
            ++mcur;
            Pd = tb.c1[mcur][mcur] * stu * Pd;
            const T c2 = cmc * s.cp - smc * s.sp;
            smc = smc * s.cp + cmc * s.sp;
            cmc = c2;
          }
          T P2 = T(0), P1 = Pd;
          const int sc = slot_cos(mm);
          Zp[a.zoff[mm] + sc] = P1 * cmc;
          if (mm > 0) Zp[a.zoff[mm] + sc + 1] = P1 * smc;
          for (int l = mm + 1; l <= a.lmax; ++l) {
            const T P = (tb.c1[l][mm] * ctu) * P1 - (tb.c2[l][mm] * tu2) * P2;
            P2 = P1;
            P1 = P;
            Zp[a.zoff[l] + sc] = P * cmc;
            if (mm > 0) Zp[a.zoff[l] + sc + 1] = P * smc;
          }
        }
      }
    }
    __syncthreads();

    // ---------------- phase 2: outer-product accumulation over the tile
    if (active) {
      const T* gbase = G + bl * a.nrow + n0;
      const T* zbase = Z + a.zoff[bl] + s0;
      for (int p = my_stream; p < a.tp; p += a.streams) {
        const T* g = gbase + p * a.spg;
        const T* zz = zbase + p * a.spz;
        T gv[(NB + 3) / 4 * 4];
        if constexpr (sizeof(T) == 4) {
#pragma unroll
          for (int q = 0; q < (NB + 3) / 4; ++q) {
            const float4 f = reinterpret_cast<const float4*>(g)[q];
            gv[4 * q] = f.x;
            gv[4 * q + 1] = f.y;
            gv[4 * q + 2] = f.z;
            gv[4 * q + 3] = f.w;
          }
        } else {
#pragma unroll
          for (int q = 0; q < (NB + 1) / 2; ++q) {
            const double2 f = reinterpret_cast<const double2*>(g)[q];
            gv[2 * q] = f.x;
            gv[2 * q + 1] = f.y;
          }
        }
        T zv[BS];
#pragma unroll
        for (int j = 0; j < BS; ++j) zv[j] = zz[j];
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
          for (int j = 0; j < BS; ++j) acc[i][j] = __builtin_fma(gv[i], zv[j], acc[i][j]);
      }
    }
    if (++tcount == a.flush_tiles) {
      tcount = 0;
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < BS; ++j) {
          wide[i][j].add(acc[i][j]);
          acc[i][j] = T(0);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < BS; ++j) wide[i][j].add(acc[i][j]);

  // ---------------- merge the streams in a fixed order through LDS
  using PT = typename PartialT<(sizeof(T) == 4 && MODE == 1) ? 1 : 0>::type;
  PT* out = reinterpret_cast<PT*>(lds_raw);
  for (int s = 0; s < a.streams; ++s) {
    if (active && my_stream == s) {
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < BS; ++j) {
          const int e = (my_block * NB + i) * BS + j;
          const PT v = wide_value(wide[i][j]);
          out[e] = (s == 0) ? v : merge(out[e], v);
        }
    }
    __syncthreads();
  }

  // ---------------- write this workgroup's partial sums, coefficient layout
  PT* part = reinterpret_cast<PT*>(a.partials) + size_t(blockIdx.x) * 2 * a.K;
  const int L2 = (a.lmax + 1) * (a.lmax + 2) / 2;
  const int nent = a.nblocks * NB * BS;
  for (int e = tid; e < nent; e += kCoeffThreads) {
    const int j = e % BS;
    const int i = (e / BS) % NB;
    int b = e / (NB * BS);
    int l = 0, nc = 0, sb = 0;
    for (int ll = 0; ll <= a.lmax; ++ll) {
      int nsc = (a.zoff[ll + 1] - a.zoff[ll]) / BS;
      int cnt = a.nchunks * nsc;
      if (b < cnt) {
        l = ll;
        nc = b / nsc;
        sb = b % nsc;
        break;
      }
      b -= cnt;
    }
    const int nn = nc * NB + i;
    const int slot = sb * BS + j;
    if (nn > a.nmax || slot > 2 * l) continue;
    const int m = (slot + 1) / 2;
    const bool is_sin = slot > 0 && (slot & 1) == 0;
    const int k = nn * L2 + l * (l + 1) / 2 + m;
    part[(is_sin ? a.K : 0) + k] = out[e];
  }
}

// ------------------------------------------------------------ fixed-order reduce
struct ReduceArgs {
  const void* partials;
  double* A;
  double* B;
  int grid, K, nmax, lmax;
  double scale[(NCAP + 1) * (LCAP + 1)];  // -sqrt(4 pi) Atilde_nl k_n, index n*(lmax+1)+l
};

template <int MODE>
__global__ __launch_bounds__(256) void scf_reduce_kernel(const ReduceArgs a) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= 2 * a.K) return;
  const int k = c < a.K ? c : c - a.K;
  const int L2 = (a.lmax + 1) * (a.lmax + 2) / 2;
  const int n = k / L2;
  const int lm = k - n * L2;
  int l = 0;
  while ((l + 1) * (l + 2) / 2 <= lm) ++l;
  const int m = lm - l * (l + 1) / 2;
  const bool is_sin = c >= a.K;
  if (is_sin && m == 0) {
    a.B[k] = 0.0;
    return;
  }
  double sum;
  if constexpr (MODE == 0) {
    const double* p = reinterpret_cast<const double*>(a.partials) + c;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;  // fixed interleave, fixed merge order
    int g = 0;
    for (; g + 4 <= a.grid; g += 4) {
      s0 += p[size_t(g) * 2 * a.K];
      s1 += p[size_t(g + 1) * 2 * a.K];
      s2 += p[size_t(g + 2) * 2 * a.K];
      s3 += p[size_t(g + 3) * 2 * a.K];
    }
    for (; g < a.grid; ++g) s0 += p[size_t(g) * 2 * a.K];
    sum = (s0 + s1) + (s2 + s3);
  } else {
    const float2* p = reinterpret_cast<const float2*>(a.partials) + c;
    float2 s = make_float2(0.f, 0.f);
    for (int g = 0; g < a.grid; ++g) s = merge(s, p[size_t(g) * 2 * a.K]);
    sum = double(s.x) + double(s.y);
  }
  const double f = (m == 0 ? 1.0 : 2.0) * a.scale[n * (a.lmax + 1) + l];
  (is_sin ? a.B : a.A)[k] = f * sum;
}

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

    // Legendre rows (row l+1 is needed for m Ybar_lm / sin(theta))
    T Y[LB + 2][LB + 2];
    Y[0][0] = tb.c1[0][0];

    T accP = T(0), accR = T(0), accT = T(0), accF = T(0);
    T Rl = s.u;     // t^l u^(l+1)
    T Rprev = T(0); // t^(l-1) u^l
#pragma unroll
    for (int l = 0; l <= LB; ++l) {
      if (l <= lmax) {
      // Legendre row l (l >= 1) and, for the force, row l+1
#pragma unroll
      for (int rr = (l == 0 ? 1 : l + (ACC ? 1 : 0)); rr <= l + (ACC ? 1 : 0); ++rr) {
        if (rr == 0) continue;
        Y[rr][rr] = tb.c1[rr][rr] * s.st * Y[rr - 1][rr - 1];
        Y[rr][rr - 1] = tb.c1[rr][rr - 1] * s.ct * Y[rr - 1][rr - 1];
#pragma unroll
        for (int m = 0; m + 2 <= rr; ++m)
          Y[rr][m] = tb.c1[rr][m] * s.ct * Y[rr - 1][m] - tb.c2[rr][m] * Y[rr - 2][m];
      }
      if (l == 0 && !ACC) {
        // nothing else needed for row 0
      }

      // radial sums over n: U,V (potential), W,X (radial derivative)
      T U[LB + 1], V[LB + 1], W[LB + 1], X[LB + 1];
#pragma unroll
      for (int m = 0; m <= l; ++m) {
        U[m] = T(0);
        V[m] = T(0);
        W[m] = T(0);
        X[m] = T(0);
      }
      T c2 = T(1), c1 = T(0);   // Chat_{n-2}, Chat_{n-1}
      T e2 = T(1), e1 = T(0);   // Ehat_{n-2}, Ehat_{n-1} (parameter a_l + 1)
      const T* cfl = cf + l * (l + 1) / 2;
      for (int nn = 0; nn <= a.nmax; ++nn) {
        const T c = s.xi * c1 - tb.q[l][nn] * c2;
        c2 = c1;
        c1 = c;
        const T* cn = cfl + nn * L2;
#pragma unroll
        for (int m = 0; m <= l; ++m) {
          U[m] = __builtin_fma(c, cn[m], U[m]);
          if (m > 0) V[m] = __builtin_fma(c, cn[K + m], V[m]);
        }
        if constexpr (ACC) {
          const T e = e1;  // Ehat_{nn-1}
#pragma unroll
          for (int m = 0; m <= l; ++m) {
            W[m] = __builtin_fma(e, cn[2 * K + m], W[m]);
            if (m > 0) X[m] = __builtin_fma(e, cn[3 * K + m], X[m]);
          }
          const T en = s.xi * e1 - tb.qd[l][nn] * e2;
          e2 = e1;
          e1 = en;
        }
      }

      // angular synthesis for this l
      T Pl = T(0), Gl = T(0), Tl = T(0), Fl = T(0);
#pragma unroll
      for (int m = 0; m <= l; ++m) {
        const T ec = U[m] * cm[m] + V[m] * sm[m];
        Pl = __builtin_fma(Y[l][m], ec, Pl);
        if constexpr (ACC) {
          const T gc = W[m] * cm[m] + X[m] * sm[m];
          Gl = __builtin_fma(Y[l][m], gc, Gl);
          if (l >= 1) {
            // dYbar/dtheta
            T dY = T(0);
            if (m + 1 <= l) dY = tb.e1[l][m] * Y[l][m + 1];
            if (m >= 1) dY = dY - tb.e2[l][m] * Y[l][m - 1];
            Tl = __builtin_fma(dY, ec, Tl);
            if (m >= 1) {
              const T fc = V[m] * cm[m] - U[m] * sm[m];
              const T mYs = -(tb.f1[l][m] * Y[l + 1][m + 1] + tb.f2[l][m] * Y[l + 1][m - 1]);
              Fl = __builtin_fma(mYs, fc, Fl);
            }
          }
        }
      }
      accP = __builtin_fma(Rl, Pl, accP);
      if constexpr (ACC) {
        const T Ql = Rprev * u2;                         // t^(l-1) u^(l+2) = (t^l u^(l+1))/r
        const T dRl = T(l) * Ql - T(2 * l + 1) * Rl * s.u;  // d/dr (t^l u^(l+1))
        T ar = dRl * Pl + Rl * u2 * Gl;
        if (l == 0 && !(s.r > T(0))) ar = T(0);          // no direction at the origin
        accR -= ar;
        if (l >= 1) {
          accT -= Ql * Tl;
          accF -= Ql * Fl;
        }
      }
      Rprev = Rl;
      Rl = Rl * tu;
      }
    }
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

// zero fill by a kernel (kept out of hipMemsetAsync so the call stays graph-safe)
__global__ __launch_bounds__(256) void fill_zero_kernel(double* __restrict__ p, int64_t count) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = 0.0;
}

// ================================================================ host launchers
int launch_fill_zero(double* p, int64_t count, hipStream_t st) {
  if (count <= 0) return ETICS_OK;
  int64_t grid = (count + 255) / 256;
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(int(grid)), dim3(256), 0, st, p, count);
  return hip_fail(hipGetLastError(), "fill_zero_kernel launch");
}

namespace {

// Hernquist-Ostriker normalisation Atilde_nl = 1/I_nl in FP64 (lgamma on the host):
//   I_nl = -(4 pi K_nl / 2^(8l+6)) Gamma(n+4l+3) / (n! (n+2l+3/2) Gamma(2l+3/2)^2),
//   K_nl = n(n+4l+3)/2 + (l+1)(2l+1).
double anl_tilde(int n, int l) {
  const double Knl = 0.5 * n * (n + 4.0 * l + 3.0) + (l + 1.0) * (2.0 * l + 1.0);
  const double logI = std::log(4.0 * kPi * Knl) - (8.0 * l + 6.0) * std::log(2.0) +
                      std::lgamma(n + 4.0 * l + 3.0) - std::lgamma(n + 1.0) -
                      std::log(n + 2.0 * l + 1.5) - 2.0 * std::lgamma(2.0 * l + 1.5);
  return -std::exp(-logI);
}

// greedy (longest job first) split of the basis jobs between the four wavefronts
void assign_jobs(const CoeffPlan& p, CoeffArgs* a) {
  struct Job {
    int code, cost;
  };
  Job jobs[2 * (LCAP + 1)];
  int nj = 0;
  for (int l = 0; l <= p.lmax; ++l) jobs[nj++] = {0x80 | l, 2 * p.nrow + p.nrow / 4 + 4};
  for (int m = 0; m <= p.lmax; ++m) jobs[nj++] = {m, (p.lmax - m + 1) * (m > 0 ? 8 : 5) + 6};
  for (int i = 1; i < nj; ++i)  // insertion sort, descending cost (stable)
    for (int j = i; j > 0 && jobs[j].cost > jobs[j - 1].cost; --j) {
      Job t = jobs[j];
      jobs[j] = jobs[j - 1];
      jobs[j - 1] = t;
    }
  int load[4] = {0, 0, 0, 0};
  int cnt[4] = {0, 0, 0, 0};
  int list[4][kMaxJobs];
  for (int i = 0; i < nj; ++i) {
    int w = 0;
    for (int k = 1; k < 4; ++k)
      if (load[k] < load[w]) w = k;
    load[w] += jobs[i].cost;
    list[w][cnt[w]++] = jobs[i].code;
  }
  for (int w = 0; w < 4; ++w) {
    // angular jobs first in increasing m (the diagonal walk only moves up), then radial
    int k = 0;
    for (int m = 0; m <= p.lmax; ++m)
      for (int i = 0; i < cnt[w]; ++i)
        if (list[w][i] == m) a->jobs[w][k++] = (unsigned char)m;
    for (int i = 0; i < cnt[w]; ++i)
      if (list[w][i] & 0x80) a->jobs[w][k++] = (unsigned char)list[w][i];
    a->njobs[w] = k;
  }
}

template <typename T, int NB, int BS, int MODE>
int launch_coeff_t(const CoeffPlan& p, const CoeffArgs& a, hipStream_t st) {
  auto kfn = scf_coeff_kernel<T, NB, BS, MODE>;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kfn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(scf_coeff)");
    attr_set = true;
  }
  hipLaunchKernelGGL(kfn, dim3(p.grid), dim3(kCoeffThreads), p.lds_bytes, st, a);
  return hip_fail(hipGetLastError(), "scf_coeff_kernel launch");
}

}  // namespace

// ------------------------------------------------------------------ planning
bool make_coeff_plan(int64_t n, int nmax, int lmax, int prec, CoeffPlan* p) {
  CoeffPlan q{};
  q.nmax = nmax;
  q.lmax = lmax;
  q.prec = prec;
  const bool f32 = prec != ETICS_FP64;
  const size_t esz = f32 ? 4 : 8;
  // register block: radial orders x angular slots
  if (nmax + 1 <= 9) {
    q.nb = 9;
  } else if (nmax + 1 <= 11) {
    q.nb = 11;
  } else {
    q.nb = 12;
  }
  q.bs = 4;
  q.nchunks = (nmax + 1 + q.nb - 1) / q.nb;
  q.nrow = (q.nchunks * q.nb + 3) / 4 * 4;
  q.zoff[0] = 0;
  for (int l = 0; l <= lmax; ++l) q.zoff[l + 1] = q.zoff[l] + (2 * l + 1 + q.bs - 1) / q.bs * q.bs;
  for (int l = lmax + 1; l <= LCAP; ++l) q.zoff[l + 1] = q.zoff[l];
  q.spg = (lmax + 1) * q.nrow;
  while (q.spg % 8 != 4) q.spg += 4;  // b128 phase-1 writes fall on distinct banks
  q.spz = q.zoff[lmax + 1] | 1;       // odd: b32 writes of consecutive lanes on distinct banks
  q.nblocks = 0;
  for (int l = 0; l <= lmax; ++l) q.nblocks += q.nchunks * (q.zoff[l + 1] - q.zoff[l]) / q.bs;
  if (q.nblocks > kCoeffThreads) return false;
  q.streams = kCoeffThreads / q.nblocks;
  if (q.streams > kMaxStreams) q.streams = kMaxStreams;
  // particles per tile: as many lanes as fit the LDS budget (<= 64, one per lane)
  const size_t budget = f32 ? 76 * 1024 : 150 * 1024;
  q.tp = 64;
  while (q.tp > 8 && size_t(q.tp) * (q.spg + q.spz) * esz > budget) q.tp -= 8;
  q.lds_bytes = size_t(q.tp) * (q.spg + q.spz) * esz;
  const size_t merge_bytes = size_t(q.nblocks) * q.nb * q.bs * 8;
  if (merge_bytes > q.lds_bytes) q.lds_bytes = merge_bytes;
  if (q.lds_bytes > 160 * 1024) return false;
  q.flush_tiles = 4;
  const int64_t ntiles = (n + q.tp - 1) / q.tp;
  const int wg_per_cu = q.lds_bytes <= 80 * 1024 ? 2 : 1;
  int64_t grid = int64_t(256) * wg_per_cu;
  if (grid > ntiles) grid = ntiles;
  if (grid < 1) grid = 1;
  q.grid = int(grid);
  *p = q;
  return true;
}

size_t coeff_partials_bytes(const CoeffPlan& p) {
  const int K = coeff_count(p.nmax, p.lmax);
  return size_t(p.grid) * 2 * K * 8;  // FP64 or a double-float pair: 8 bytes per entry
}

size_t force_prep_bytes(int nmax, int lmax, int prec) {
  return size_t(4) * coeff_count(nmax, lmax) * (prec == ETICS_FP64 ? 8 : 4);
}

int launch_scf_coeffs(const CoeffPlan& p, const double* x, const double* y, const double* z,
                      const double* m, int64_t n, double* A, double* B, void* ws,
                      hipStream_t st) {
  const int K = coeff_count(p.nmax, p.lmax);
  CoeffArgs a{};
  a.x = x;
  a.y = y;
  a.z = z;
  a.m = m;
  a.n = n;
  a.partials = ws;
  a.K = K;
  a.nmax = p.nmax;
  a.lmax = p.lmax;
  a.tp = p.tp;
  a.nrow = p.nrow;
  a.spg = p.spg;
  a.spz = p.spz;
  a.nblocks = p.nblocks;
  a.streams = p.streams;
  a.flush_tiles = p.flush_tiles;
  a.ntiles = int((n + p.tp - 1) / p.tp);
  a.nchunks = p.nchunks;
  for (int l = 0; l <= LCAP + 1; ++l) a.zoff[l] = p.zoff[l];
  assign_jobs(p, &a);

  int rc;
  const int mode = p.prec == ETICS_FP64 ? 0 : (p.prec == ETICS_MIXED_FP64ACC ? 1 : 2);
  if (p.nb == 9) {
    rc = mode == 0 ? launch_coeff_t<double, 9, 4, 0>(p, a, st)
       : mode == 1 ? launch_coeff_t<float, 9, 4, 0>(p, a, st)
                   : launch_coeff_t<float, 9, 4, 1>(p, a, st);
  } else if (p.nb == 11) {
    rc = mode == 0 ? launch_coeff_t<double, 11, 4, 0>(p, a, st)
       : mode == 1 ? launch_coeff_t<float, 11, 4, 0>(p, a, st)
                   : launch_coeff_t<float, 11, 4, 1>(p, a, st);
  } else {
    rc = mode == 0 ? launch_coeff_t<double, 12, 4, 0>(p, a, st)
       : mode == 1 ? launch_coeff_t<float, 12, 4, 0>(p, a, st)
                   : launch_coeff_t<float, 12, 4, 1>(p, a, st);
  }
  if (rc) return rc;

  ReduceArgs r{};
  r.partials = ws;
  r.A = A;
  r.B = B;
  r.grid = p.grid;
  r.K = K;
  r.nmax = p.nmax;
  r.lmax = p.lmax;
  for (int nn = 0; nn <= p.nmax; ++nn)
    for (int l = 0; l <= p.lmax; ++l)
      r.scale[nn * (p.lmax + 1) + l] =
          -2.0 * std::sqrt(kPi) * anl_tilde(nn, l) * gegen_k(nn, 2.0 * l + 1.5);
  const int rb = (2 * K + 255) / 256;
  if (mode == 2)
    hipLaunchKernelGGL(scf_reduce_kernel<1>, dim3(rb), dim3(256), 0, st, r);
  else
    hipLaunchKernelGGL(scf_reduce_kernel<0>, dim3(rb), dim3(256), 0, st, r);
  return hip_fail(hipGetLastError(), "scf_reduce_kernel launch");
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
