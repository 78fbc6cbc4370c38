// etics_coeff.hip -- SCF expansion coefficients on gfx950 (MI355X).
//
// The first part of an SCF force calculation (paper Section 3.3) is the sum over all
// particles k of m_k PhiT_nl(r_k) Ybar_lm(theta_k) (cos, sin)(m phi_k) for every
// (n, l, m) (eq. scf-phi with the Hernquist-Ostriker basis of Section 2.5).
//
// scf_coeff_kernel: each workgroup (4 wavefronts) walks tiles of `tp` particles.
//   Phase 1 evaluates each particle's basis once, one particle per lane.  The basis
//   is split into independent jobs -- the Gegenbauer row of one l (radial job) and
//   the Legendre column of one m times (cos, sin)(m phi) and the radial prefactor
//   (angular job) -- and a compile-time plan gives each job to one wavefront, so the
//   four wavefronts share the work of the same 64 particles.  The values go to LDS
//   at compile-time offsets.
//   Phase 2 is an outer-product accumulation over the tile: every lane owns an
//   nb x bs register block of coefficients (radial orders x angular slots of one l)
//   and accumulates the products of the LDS-staged radial and angular values.  The
//   lanes are grouped in "streams": each stream owns one copy of every block and
//   takes every streams-th particle of the tile.  FP32 partial sums are folded into
//   FP64 (or compensated double-float) accumulators every few tiles.
//   At the end the streams are merged in a fixed order through LDS and the
//   workgroup writes one partial coefficient vector.
// scf_reduce_kernel sums the partial vectors over workgroups in a fixed order and
//   applies (2 - delta_m0) Atilde_nl and the basis constants, so the result does not
//   depend on how the hardware schedules workgroups.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "etics_device.hpp"
#include "etics_internal.hpp"

namespace etics {

struct CoeffArgs {
  const double *x, *y, *z, *m;
  int64_t n;
  void* partials;  // [grid][2K] FP64 (or double-float pairs)
  int K, nmax, lmax, tp, nblocks, streams, flush_tiles, ntiles, nchunks;
};

// ------------------------------------------------------------ phase-1 job plan
// Greedy longest-job-first split of the basis jobs of a cutoff bucket between the
// four wavefronts.  Angular job m costs ~6 operations per l in [m, lb]; radial job l
// ~2 operations per padded radial order.
template <int LB, int NRP>
struct JobPlan {
  int ownerZ[LB + 1];
  int ownerG[LB + 1];
  int maxm[4];
};

template <int LB, int NRP>
constexpr JobPlan<LB, NRP> make_job_plan() {
  JobPlan<LB, NRP> p{};
  int code[2 * (LB + 1)] = {};
  int cost[2 * (LB + 1)] = {};
  int nj = 0;
  for (int m = 0; m <= LB; ++m) {
    code[nj] = m;
    cost[nj++] = 6 * (LB - m + 1) + 8;
  }
  for (int l = 0; l <= LB; ++l) {
    code[nj] = 0x80 | l;
    cost[nj++] = 2 * NRP + NRP / 4 + 2;
  }
  for (int i = 1; i < nj; ++i)
    for (int j = i; j > 0 && cost[j] > cost[j - 1]; --j) {
      int c = cost[j];
      cost[j] = cost[j - 1];
      cost[j - 1] = c;
      c = code[j];
      code[j] = code[j - 1];
      code[j - 1] = c;
    }
  int load[4] = {0, 0, 0, 0};
  for (int w = 0; w < 4; ++w) p.maxm[w] = -1;
  for (int i = 0; i < nj; ++i) {
    int w = 0;
    for (int k = 1; k < 4; ++k)
      if (load[k] < load[w]) w = k;
    load[w] += cost[i];
    if (code[i] & 0x80) {
      p.ownerG[code[i] & 0x7f] = w;
    } else {
      p.ownerZ[code[i]] = w;
      if (code[i] > p.maxm[w]) p.maxm[w] = code[i];
    }
  }
  return p;
}

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

// decode register block b of a cutoff (lmax, nchunks) into (l, n0, s0)
template <int NB, int BS>
__device__ __forceinline__ void decode_block(int b, int lmax, int nchunks, int& bl, int& n0,
                                             int& s0) {
  bl = 0;
  n0 = 0;
  s0 = 0;
  for (int l = 0; l <= lmax; ++l) {
    const int nsc = slot_pad(l, BS) / BS;
    const int cnt = nchunks * nsc;
    if (b < cnt) {
      bl = l;
      n0 = (b / nsc) * NB;
      s0 = (b % nsc) * BS;
      return;
    }
    b -= cnt;
  }
}

template <typename T, int LB, int NB, int BS, int MODE>
__global__ __launch_bounds__(kCoeffThreads, sizeof(T) == 4 ? 2 : 1) void scf_coeff_kernel(
    const CoeffArgs a) {
  constexpr int NRP = nrp_for_nb(NB);
  constexpr int SPG = g_stride(LB, NRP);
  constexpr int SPZ = z_stride(LB, BS);
  constexpr JobPlan<LB, NRP> kJP = make_job_plan<LB, NRP>();

  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* G = reinterpret_cast<T*>(lds_raw);  // [tp][SPG]  radial values, rows of NRP per l
  T* Z = G + a.tp * SPG;                 // [tp][SPZ]  angular values x mass x radial prefactor
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lmax = a.lmax, nmax = a.nmax;

  // largest angular column owned by this wavefront (the diagonal walk stops there)
  int maxm_w = -1;
  static_for<4>([&](auto wc) {
    if (wave == decltype(wc)::value) maxm_w = kJP.maxm[decltype(wc)::value];
  });

  // register block owned by this thread
  const int my_stream = tid / a.nblocks;
  const int my_block = tid - my_stream * a.nblocks;
  const bool active = my_stream < a.streams;
  int bl, n0, s0;
  decode_block<NB, BS>(my_block, lmax, a.nchunks, bl, n0, s0);

  T acc[NB][BS];
  Wide<T, MODE> wide[NB][BS];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < BS; ++j) acc[i][j] = T(0);

  // angular padding slots are never written by phase 1; keep them finite
  for (int i = tid; i < a.tp * SPZ; i += kCoeffThreads) Z[i] = T(0);
  __syncthreads();

  // particle data of the first tile (later tiles are prefetched during phase 2)
  double xd = 0.0, yd = 0.0, zd = 0.0, md = 0.0;
  auto load_particle = [&](int tile) {
    const int64_t pi = int64_t(tile) * a.tp + lane;
    const bool valid = tile < a.ntiles && lane < a.tp && pi < a.n;
    xd = valid ? a.x[pi] : 0.0;
    yd = valid ? a.y[pi] : 0.0;
    zd = valid ? a.z[pi] : 0.0;
    md = valid ? a.m[pi] : 0.0;
  };
  load_particle(blockIdx.x);

  int tcount = 0;
  for (int tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    // ---------------- phase 1: basis of the tile's particles (one per lane)
    if (lane < a.tp) {
      const Sph<T> s = sph<T>(xd, yd, zd);
      const T tu = s.t * s.u, ctu = s.ct * tu, tu2 = tu * tu, stu = s.st * tu;
      T* Gp = G + lane * SPG;
      T* Zp = Z + lane * SPZ;
      // angular jobs: column m of mass u (tu)^l Ybar_lm (cos, sin)(m phi), l = m..lmax.
      // The diagonal value mass u (tu)^m Ybar_mm and (cos, sin)(m phi) are walked up
      // to the largest column this wavefront owns.
      T Pd = T(md) * s.u * T(kTab.c1[0][0]);
      T cmc = T(1), smc = T(0);
      static_for<LB + 1>([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        if constexpr (m > 0) {
          if (m <= maxm_w) {
            Pd = (T(kTab.c1[m][m]) * stu) * Pd;
            const T c2 = cmc * s.cp - smc * s.sp;
            smc = smc * s.cp + cmc * s.sp;
            cmc = c2;
          }
        }
        if (wave == kJP.ownerZ[m] && m <= lmax) {
          constexpr int sc = m == 0 ? 0 : 2 * m - 1;
          T P2 = T(0), P1 = Pd;
          Zp[zoff(m, BS) + sc] = P1 * cmc;
          if constexpr (m > 0) Zp[zoff(m, BS) + sc + 1] = P1 * smc;
          static_for<LB - m>([&](auto kc) {
            constexpr int l = m + 1 + decltype(kc)::value;
            if (l <= lmax) {
              const T P = (T(kTab.c1[l][m]) * ctu) * P1 - (T(kTab.c2[l][m]) * tu2) * P2;
              P2 = P1;
              P1 = P;
              Zp[zoff(l, BS) + sc] = P * cmc;
              if constexpr (m > 0) Zp[zoff(l, BS) + sc + 1] = P * smc;
            }
          });
        }
      });
      // radial jobs: monic Gegenbauer Chat_n^(2l+3/2)(xi), n = 0..NRP-1.  Entries past
      // nmax only feed coefficients that are never written out; they stay finite.
      static_for<LB + 1>([&](auto lc) {
        constexpr int l = decltype(lc)::value;
        if (wave == kJP.ownerG[l] && l <= lmax) {
          T p2 = T(1), p1 = T(0);
          static_for<NRP / 4>([&](auto qc) {
            constexpr int nb4 = 4 * decltype(qc)::value;
            T v[4];
            static_for<4>([&](auto jc) {
              constexpr int nn = nb4 + decltype(jc)::value;
              const T c = s.xi * p1 - T(kTab.q[l][nn]) * p2;
              p2 = p1;
              p1 = c;
              v[decltype(jc)::value] = c;
            });
            T* row = Gp + l * NRP + nb4;
            if constexpr (sizeof(T) == 4) {
              *reinterpret_cast<float4*>(row) = make_float4(v[0], v[1], v[2], v[3]);
            } else {
              *reinterpret_cast<double2*>(row) = make_double2(v[0], v[1]);
              *reinterpret_cast<double2*>(row + 2) = make_double2(v[2], v[3]);
            }
          });
        }
      });
    }
    __syncthreads();
    // next tile's particles load while phase 2 runs
    load_particle(tile + gridDim.x);

    // ---------------- phase 2: outer-product accumulation over the tile
    if (active) {
      const T* gbase = G + bl * NRP + n0;
      const T* zbase = Z + zoff_rt<BS>(bl) + s0;
      constexpr int NG = (NB + 3) / 4 * 4;
      T gv[2][NG], zv[2][BS];
      auto fetch = [&](int p, int buf) {
        const T* g = gbase + p * SPG;
        const T* zz = zbase + p * SPZ;
        if constexpr (sizeof(T) == 4) {
#pragma unroll
          for (int q = 0; q < NG / 4; ++q) {
            const float4 f = reinterpret_cast<const float4*>(g)[q];
            gv[buf][4 * q] = f.x;
            gv[buf][4 * q + 1] = f.y;
            gv[buf][4 * q + 2] = f.z;
            gv[buf][4 * q + 3] = f.w;
          }
        } else {
#pragma unroll
          for (int q = 0; q < (NB + 1) / 2; ++q) {
            const double2 f = reinterpret_cast<const double2*>(g)[q];
            gv[buf][2 * q] = f.x;
            gv[buf][2 * q + 1] = f.y;
          }
        }
#pragma unroll
        for (int j = 0; j < BS; ++j) zv[buf][j] = zz[j];
      };
      auto madd = [&](int buf) {
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
          for (int j = 0; j < BS; ++j) acc[i][j] = fma_(gv[buf][i], zv[buf][j], acc[i][j]);
      };
      // two particles per trip, each one's LDS reads issued before the other's FMAs
      int p = my_stream;
      if (p < a.tp) fetch(p, 0);
      for (; p + a.streams < a.tp; p += 2 * a.streams) {
        fetch(p + a.streams, 1);
        madd(0);
        if (p + 2 * a.streams < a.tp) fetch(p + 2 * a.streams, 0);
        madd(1);
      }
      if (p < a.tp) madd(0);
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
  const int L2 = (lmax + 1) * (lmax + 2) / 2;
  const int nent = a.nblocks * NB * BS;
  for (int e = tid; e < nent; e += kCoeffThreads) {
    const int j = e % BS;
    const int i = (e / BS) % NB;
    int l, nb0, sb0;
    decode_block<NB, BS>(e / (NB * BS), lmax, a.nchunks, l, nb0, sb0);
    const int nn = nb0 + i;
    const int slot = sb0 + j;
    if (nn > nmax || slot > 2 * l) continue;
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

// Each workgroup sums 32 coefficient columns over all partials: 8 slices of rows
// (slice s takes rows s, s+8, ...) are summed in row order, then the 8 slice sums
// are added in slice order.  The order is fixed, so the result is reproducible.
constexpr int kRedCols = 32, kRedSlices = 8;

template <int MODE>
__global__ __launch_bounds__(256) void scf_reduce_kernel(const ReduceArgs a) {
  using PT = typename PartialT<MODE>::type;
  __shared__ PT red[kRedSlices][kRedCols];
  const int col = threadIdx.x % kRedCols, slice = threadIdx.x / kRedCols;
  const int c = blockIdx.x * kRedCols + col;
  const size_t stride = size_t(2) * a.K;
  PT s{};
  if (c < 2 * a.K) {
    const PT* p = reinterpret_cast<const PT*>(a.partials) + c;
    if constexpr (MODE == 0) {
      double s0 = 0.0, s1 = 0.0;
      int g = slice;
      for (; g + kRedSlices < a.grid; g += 2 * kRedSlices) {
        s0 += p[size_t(g) * stride];
        s1 += p[size_t(g + kRedSlices) * stride];
      }
      if (g < a.grid) s0 += p[size_t(g) * stride];
      s = s0 + s1;
    } else {
      s = make_float2(0.f, 0.f);
      for (int g = slice; g < a.grid; g += kRedSlices) s = merge(s, p[size_t(g) * stride]);
    }
  }
  red[slice][col] = s;
  __syncthreads();
  if (slice != 0 || c >= 2 * a.K) return;
  PT sum = red[0][col];
  for (int q = 1; q < kRedSlices; ++q) sum = merge(sum, red[q][col]);
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
  double v;
  if constexpr (MODE == 0) {
    v = sum;
  } else {
    v = double(sum.x) + double(sum.y);
  }
  const double f = (m == 0 ? 1.0 : 2.0) * a.scale[n * (a.lmax + 1) + l];
  (is_sin ? a.B : a.A)[k] = f * v;
}

// zero fill by a kernel (kept out of hipMemsetAsync so the call stays graph-safe)
__global__ __launch_bounds__(256) void fill_zero_kernel(double* __restrict__ p, int64_t count) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = 0.0;
}

// ================================================================ host side
int launch_fill_zero(double* p, int64_t count, hipStream_t st) {
  if (count <= 0) return ETICS_OK;
  int64_t grid = (count + 255) / 256;
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(int(grid)), dim3(256), 0, st, p, count);
  return hip_fail(hipGetLastError(), "fill_zero_kernel launch");
}

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

namespace {

template <typename T, int LB, int NB, int BS, int MODE>
int launch_coeff_t(const CoeffPlan& p, const CoeffArgs& a, hipStream_t st) {
  auto kfn = scf_coeff_kernel<T, LB, NB, BS, MODE>;
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

template <typename T, int MODE, int LB>
int launch_coeff_nb(const CoeffPlan& p, const CoeffArgs& a, hipStream_t st) {
  switch (p.nb) {
    case 9: return launch_coeff_t<T, LB, 9, 4, MODE>(p, a, st);
    case 11: return launch_coeff_t<T, LB, 11, 4, MODE>(p, a, st);
    default: return launch_coeff_t<T, LB, 12, 4, MODE>(p, a, st);
  }
}

template <typename T, int MODE>
int launch_coeff_lb(const CoeffPlan& p, const CoeffArgs& a, hipStream_t st) {
  switch (p.lb) {
    case 2: return launch_coeff_nb<T, MODE, 2>(p, a, st);
    case 6: return launch_coeff_nb<T, MODE, 6>(p, a, st);
    case 10: return launch_coeff_nb<T, MODE, 10>(p, a, st);
    default: return launch_coeff_nb<T, MODE, 14>(p, a, st);
  }
}

}  // namespace

// ------------------------------------------------------------------ planning
bool make_coeff_plan(int64_t n, int nmax, int lmax, int prec, CoeffPlan* p) {
  CoeffPlan q{};
  q.nmax = nmax;
  q.lmax = lmax;
  q.prec = prec;
  const size_t esz = prec == ETICS_FP64 ? 8 : 4;
  q.lb = lmax <= 2 ? 2 : lmax <= 6 ? 6 : lmax <= 10 ? 10 : 14;
  q.nb = nmax + 1 <= 9 ? 9 : nmax + 1 <= 11 ? 11 : 12;
  q.bs = 4;
  q.nchunks = (nmax + 1 + q.nb - 1) / q.nb;
  const int nrp = nrp_for_nb(q.nb);
  if (q.nchunks * q.nb > nrp) return false;
  q.spg = g_stride(q.lb, nrp);
  q.spz = z_stride(q.lb, q.bs);
  q.nblocks = 0;
  for (int l = 0; l <= lmax; ++l) q.nblocks += q.nchunks * slot_pad(l, q.bs) / q.bs;
  if (q.nblocks > kCoeffThreads) return false;
  q.streams = kCoeffThreads / q.nblocks;
  if (q.streams > kMaxStreams) q.streams = kMaxStreams;
  // particles per tile: one per lane of a wavefront, a multiple of the stream count
  // (every stream takes the same number), within the LDS budget
  const size_t budget = esz == 4 ? 76 * 1024 : 150 * 1024;
  const size_t per_particle = size_t(q.spg + q.spz) * esz;
  int tp = 64;
  if (size_t(tp) * per_particle > budget) tp = int(budget / per_particle);
  if (q.streams <= tp) tp = tp / q.streams * q.streams;
  if (tp < 1) return false;
  q.tp = tp;
  q.lds_bytes = size_t(q.tp) * per_particle;
  const size_t merge_bytes = size_t(q.nblocks) * q.nb * q.bs * 8;
  if (merge_bytes > q.lds_bytes) q.lds_bytes = merge_bytes;
  if (q.lds_bytes > 160 * 1024) return false;
  q.flush_tiles = 8;
  const int64_t ntiles = (n + q.tp - 1) / q.tp;
  const int wg_per_cu = (esz == 4 && q.lds_bytes <= 80 * 1024) ? 2 : 1;
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
  a.nblocks = p.nblocks;
  a.streams = p.streams;
  a.flush_tiles = p.flush_tiles;
  a.ntiles = int((n + p.tp - 1) / p.tp);
  a.nchunks = p.nchunks;

  int rc;
  const int mode = p.prec == ETICS_FP64 ? 0 : (p.prec == ETICS_MIXED_FP64ACC ? 1 : 2);
  if (mode == 0)
    rc = launch_coeff_lb<double, 0>(p, a, st);
  else if (mode == 1)
    rc = launch_coeff_lb<float, 0>(p, a, st);
  else
    rc = launch_coeff_lb<float, 1>(p, a, st);
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
  const int rb = (2 * K + kRedCols - 1) / kRedCols;
  if (mode == 2)
    hipLaunchKernelGGL(scf_reduce_kernel<1>, dim3(rb), dim3(256), 0, st, r);
  else
    hipLaunchKernelGGL(scf_reduce_kernel<0>, dim3(rb), dim3(256), 0, st, r);
  return hip_fail(hipGetLastError(), "scf_reduce_kernel launch");
}

}  // namespace etics
