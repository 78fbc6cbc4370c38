// etics_coeff.hip -- SCF expansion coefficients on gfx950 (MI355X): host side.
//
// The coefficient kernels themselves are in etics_coeff_wg.hpp.  This file holds the
// fixed-order reductions that sum the per-workgroup (or per-unit) partial vectors and
// apply (2 - delta_m0) Atilde_nl and the basis constants, the tile plans (fixed rules
// and tuned overrides), and the launches of the coefficient sums of one system, of
// batched systems and of the allocation-free entry point.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdint>
#include <mutex>

#include "etics_coeff_wg.hpp"
#include "etics_device.hpp"
#include "etics_internal.hpp"

namespace etics {

// ------------------------------------------------------------ fixed-order reduce
struct ReduceArgs {
  const void* partials;
  double* A;
  double* B;
  int grid, K, nmax, lmax;
  double scale[(NCAP + 1) * (LCAP + 1)];  // -sqrt(4 pi) Atilde_nl k_n, index n*(lmax+1)+l
};

// Each workgroup sums 8 coefficient columns over all partials: 32 slices of rows
// (slice s takes rows s, s+32, ...) are summed in row order, then the 32 slice sums
// are added in slice order.  The order is fixed, so the result is reproducible.
constexpr int kRedCols = 8, kRedSlices = 32;

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

// Normalisation Atilde_nl = 1/I_nl, I_nl = integral of rhoT_nl PhiT_nl r^2 dr, in FP64
// (lgamma on the host).
// Hernquist-Ostriker:
//   I_nl = -(4 pi K_nl / 2^(8l+6)) Gamma(n+4l+3) / (n! (n+2l+3/2) Gamma(2l+3/2)^2),
//   K_nl = n(n+4l+3)/2 + (l+1)(2l+1).
// Clutton-Brock:
//   I_nl = -pi K_nl 2^(-4l-4) Gamma(n+2l+2) / (n! (n+l+1) (l!)^2),
//   K_nl = 4n(n+2l+2) + (2l+1)(2l+3).
double anl_tilde(int n, int l, int basis) {
  double logI;
  if (basis == kBasisCB) {
    const double Knl = 4.0 * n * (n + 2.0 * l + 2.0) + (2.0 * l + 1.0) * (2.0 * l + 3.0);
    logI = std::log(kPi * Knl) - (4.0 * l + 4.0) * std::log(2.0) + std::lgamma(n + 2.0 * l + 2.0) -
           std::lgamma(n + 1.0) - std::log(n + l + 1.0) - 2.0 * std::lgamma(l + 1.0);
  } else {
    const double Knl = 0.5 * n * (n + 4.0 * l + 3.0) + (l + 1.0) * (2.0 * l + 1.0);
    logI = std::log(4.0 * kPi * Knl) - (8.0 * l + 6.0) * std::log(2.0) + std::lgamma(n + 4.0 * l + 3.0) -
           std::lgamma(n + 1.0) - std::log(n + 2.0 * l + 1.5) - 2.0 * std::lgamma(2.0 * l + 1.5);
  }
  return -std::exp(-logI);
}

namespace {
void fill_scale(double* scale, int nmax, int lmax, int basis) {
  for (int nn = 0; nn <= nmax; ++nn)
    for (int l = 0; l <= lmax; ++l)
      scale[nn * (lmax + 1) + l] =
          -2.0 * std::sqrt(kPi) * anl_tilde(nn, l, basis) * gegen_k(nn, basis_alpha(basis, l));
}

}  // namespace

// ------------------------------------------------------------------ planning
namespace {

// LDS bytes per particle of a tile, and the element size, of a plan's cutoff bucket
size_t plan_per_particle(const CoeffPlan& q) {
  return size_t(q.spg + q.spz) * (q.prec == ETICS_FP64 ? 8 : 4);
}

// Complete a plan from its tile shape (nw particle groups, tp particles, streams, outer
// products on the matrix cores or not); false if the shape breaks a limit of the
// kernel: phase 1 has one lane per particle in each of 4/nw groups of 64; the VALU
// phase 2 needs streams x nblocks lanes and an LDS stream merge, the matrix phase 2 an
// FP32 mode; everything must fit the LDS.
bool finish_plan(CoeffPlan& q, int nw, int tp, int streams, bool mfma) {
  if (!(nw == 4 || ((nw == 1 || nw == 2) && q.lb <= 6))) return false;
  if (streams < 1 || streams > kMaxStreams || streams * q.nblocks > kCoeffThreads) return false;
  if (tp < 1 || tp > 64 * (4 / nw)) return false;
  if (mfma && q.prec == ETICS_FP64) return false;
  const size_t lds = size_t(tp) * plan_per_particle(q);
  const size_t merge_bytes = mfma ? 0 : size_t(q.nblocks) * q.nb * q.bs * 8;
  q.nw = nw;
  q.tp = tp;
  q.streams = streams;
  q.mfma = mfma;
  q.lds_bytes = lds > merge_bytes ? lds : merge_bytes;
  if (q.lds_bytes > 160 * 1024) return false;
  // FP32 runs of about 72 particles per lane (VALU) or per output entry (matrix cores)
  // before each fold
  const int per_tile = mfma ? q.tp : (q.tp / q.streams > 0 ? q.tp / q.streams : 1);
  q.flush_tiles = 72 / per_tile > 0 ? 72 / per_tile : 1;
  return true;
}

}  // namespace

int coeff_grid(const CoeffPlan& p, int64_t work_items) {
  int64_t grid = int64_t(256) * p.grid_mult;
  if (grid > work_items) grid = work_items;
  if (grid < 1) grid = 1;
  return int(grid);
}

bool make_coeff_plan(int64_t n, int nmax, int lmax, int prec, CoeffPlan* p, int basis, bool batched) {
  CoeffPlan q{};
  q.nmax = nmax;
  q.lmax = lmax;
  q.prec = prec;
  q.basis = basis;
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
  // Fixed rules.  Streams: as many copies of the register blocks as the workgroup's
  // lanes hold.  Particles per tile: one per lane of a wavefront in each particle group
  // (1, 2 or 4 groups of 64, the four wavefronts splitting the basis jobs 4, 2 or 1
  // ways), a multiple of the stream count (every stream takes the same number), within
  // the LDS budget; more groups when they fit (small cutoffs), so a tile does more work
  // per barrier.  Two workgroups per CU when the LDS allows it in FP32.
  int streams = kCoeffThreads / q.nblocks;
  if (streams > kMaxStreams) streams = kMaxStreams;
  const size_t budget = esz == 4 ? 76 * 1024 : 150 * 1024;
  const size_t per_particle = plan_per_particle(q);
  int nw = 4, tp = 64;
  if (q.lb <= 6) {
    for (int w = 1; w <= 2; w *= 2) {
      const int tmax = 64 * (4 / w);
      if (size_t(tmax) * per_particle <= budget && streams <= tmax) {
        nw = w;
        tp = tmax;
        break;
      }
    }
  }
  if (size_t(tp) * per_particle > budget) tp = int(budget / per_particle);
  // Phase 2 on the VALU: the matrix-core variant needs two 32-bit LDS reads per lane per
  // 256 products (and more for the ragged edges), so on this kernel it is bound by LDS
  // traffic and latency rather than by the matrix cores, and measured slower at the
  // larger cutoffs; the tuner takes it where it wins.
  const bool mfma = false;
  if (streams <= tp) tp = tp / streams * streams;
  if (!finish_plan(q, nw, tp, streams, mfma)) return false;
  q.grid_mult = (esz == 4 && q.lds_bytes <= 80 * 1024) ? 2 : 1;
  q.unit = kUnitParticles;
  q.split = kForceSplit;
  q.tuned = false;
  // a plan measured faster by the tuner, if one is known and valid for this kernel
  TunedParams t;
  if (tuned_lookup(batched ? 1 : 0, nmax, lmax, prec, basis, n, &t)) {
    CoeffPlan r = q;
    bool ok = finish_plan(r, t.nw > 0 ? t.nw : q.nw, t.tp > 0 ? t.tp : q.tp,
                          t.streams > 0 ? t.streams : q.streams,
                          t.phase2 > 0 ? t.phase2 == 2 : q.mfma);
    if (t.grid_mult > 0) r.grid_mult = t.grid_mult;
    if (t.unit > 0) r.unit = t.unit;
    if (t.split > 0) r.split = t.split;
    ok = ok && r.grid_mult >= 1 && r.grid_mult <= 2 && r.unit >= kMinUnitParticles &&
         r.unit <= kMaxUnitParticles && r.split >= 1 && r.split <= 16 && r.unit / r.split >= 64;
    if (ok) {
      r.tuned = true;
      q = r;
    }
  }
  const int64_t ntiles = (n + q.tp - 1) / q.tp;
  q.grid = coeff_grid(q, ntiles);
  *p = q;
  return true;
}

size_t coeff_partials_bytes(const CoeffPlan& p) {
  const int K = coeff_count(p.nmax, p.lmax);
  return size_t(p.grid) * 2 * K * 8;  // FP64 or a double-float pair: 8 bytes per entry
}

int launch_coeff_reduce(const CoeffPlan& p, const void* partials, int grid, double* A, double* B,
                        hipStream_t st) {
  const int K = coeff_count(p.nmax, p.lmax);
  ReduceArgs r{};
  r.partials = partials;
  r.A = A;
  r.B = B;
  r.grid = grid;
  r.K = K;
  r.nmax = p.nmax;
  r.lmax = p.lmax;
  fill_scale(r.scale, p.nmax, p.lmax, p.basis);
  const int rb = (2 * K + kRedCols - 1) / kRedCols;
  if (p.prec == ETICS_MIXED_COMP32)
    hipLaunchKernelGGL(scf_reduce_kernel<1>, dim3(rb), dim3(256), 0, st, r);
  else
    hipLaunchKernelGGL(scf_reduce_kernel<0>, dim3(rb), dim3(256), 0, st, r);
  return hip_fail(hipGetLastError(), "scf_reduce_kernel launch");
}

CoeffArgs coeff_args(const CoeffPlan& p, const double* x, const double* y, const double* z,
                     const double* m, int64_t n, int tile_particles, void* ws) {
  CoeffArgs a{};
  a.x = x;
  a.y = y;
  a.z = z;
  a.m = m;
  a.n = n;
  a.partials = ws;
  a.K = coeff_count(p.nmax, p.lmax);
  a.nmax = p.nmax;
  a.lmax = p.lmax;
  a.tp = p.tp;
  a.nblocks = p.nblocks;
  a.streams = p.streams;
  a.flush_tiles = p.flush_tiles;
  a.ntiles = int((n + tile_particles - 1) / tile_particles);
  a.nchunks = p.nchunks;
  return a;
}

int launch_scf_coeffs(const CoeffPlan& p, const double* x, const double* y, const double* z,
                      const double* m, int64_t n, double* A, double* B, void* ws,
                      hipStream_t st) {
  const CoeffArgs a = coeff_args(p, x, y, z, m, n, p.tp, ws);
  int rc = launch_coeff_any<false, false>(p, a, p.grid, st);
  if (rc) return rc;
  return launch_coeff_reduce(p, ws, p.grid, A, B, st);
}

bool dot_plan(const CoeffPlan& p, int64_t n, CoeffPlan* out) {
  CoeffPlan q = p;
  // two rows per particle: an even number of rows
  int tp = p.tp / 2 * 2;
  if (!p.mfma && tp < p.streams) tp = (p.streams + 1) / 2 * 2;
  if (!finish_plan(q, p.nw, tp, p.streams, p.mfma)) return false;
  q.grid = coeff_grid(q, (n + q.tp / 2 - 1) / (q.tp / 2));
  *out = q;
  return true;
}

// ------------------------------------------------------- allocation-free variant
// Per-workgroup partial vectors of etics_scf_coeffs_noalloc: a file-scope device array
// instead of a caller workspace.  Every device the library runs on holds its own copy
// until the process ends.  In host code `scratch` names a host-side stand-in, never
// the device memory: its device address is looked up once per device and only that
// address is passed to kernels.  Every call on a device shares that device's array,
// so calls that overlap in time on one device race.  The coefficient kernel writes
// every partial entry the reduction reads, so nothing needs clearing between calls.
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_dev[kMaxDevices] = {};
}  // namespace

int noalloc_scratch(void** out) {
  int dev = 0;
  int rc = hip_fail(hipGetDevice(&dev), "hipGetDevice");
  if (rc) return rc;
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("etics_scf_coeffs_noalloc: device index beyond 63");
    return ETICS_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    rc = hip_fail(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (rc) return rc;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return ETICS_OK;
}

// ------------------------------------------------------------ batched reduce
struct BatchedReduceArgs {
  const void* partials;  // [units][2K]
  const int* ustart;     // [nsys+1]
  double* A;             // [nsys*K]
  double* B;
  int nsys, K, nmax, lmax;
  double scale[(NCAP + 1) * (LCAP + 1)];
};

// a system's units' partials summed in unit order: workgroup (s, j) takes entries
// [64 j, 64 j + 64) of system s, one per lane, the loads of several units in flight
constexpr int kReduceLanes = 64;
template <int MODE>
__global__ __launch_bounds__(kReduceLanes) void scf_reduce_batched_kernel(const BatchedReduceArgs a) {
  using PT = typename PartialT<MODE>::type;
  const int s = blockIdx.x;
  const int u0 = a.ustart[s], u1 = a.ustart[s + 1];
  const size_t stride = size_t(2) * a.K;
  const int L2 = (a.lmax + 1) * (a.lmax + 2) / 2;
  const int c = blockIdx.y * kReduceLanes + threadIdx.x;
  if (c < 2 * a.K) {
    const int k = c < a.K ? c : c - a.K;
    const int n = k / L2;
    const int lm = k - n * L2;
    int l = 0;
    while ((l + 1) * (l + 2) / 2 <= lm) ++l;
    const int m = lm - l * (l + 1) / 2;
    const bool is_sin = c >= a.K;
    double* dst = (is_sin ? a.B : a.A) + size_t(s) * a.K + k;
    if (is_sin && m == 0) {
      *dst = 0.0;
      return;
    }
    const PT* p = reinterpret_cast<const PT*>(a.partials) + c;
    double v;
    if constexpr (MODE == 0) {
      double acc = 0.0;
#pragma unroll 8
      for (int u = u0; u < u1; ++u) acc += p[size_t(u) * stride];
      v = acc;
    } else {
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll 8
      for (int u = u0; u < u1; ++u) acc = merge(acc, p[size_t(u) * stride]);
      v = double(acc.x) + double(acc.y);
    }
    *dst = (m == 0 ? 1.0 : 2.0) * a.scale[n * (a.lmax + 1) + l] * v;
  }
}

int max_units(int64_t ntotal, int nsys, int unit) {
  return nsys + int((ntotal + unit - 1) / unit);
}

int launch_coeff_reduce_batched(const CoeffPlan& p, const void* partials, const int* ustart, int nsys,
                                double* A, double* B, hipStream_t st) {
  BatchedReduceArgs r{};
  r.partials = partials;
  r.ustart = ustart;
  r.A = A;
  r.B = B;
  r.nsys = nsys;
  r.K = coeff_count(p.nmax, p.lmax);
  r.nmax = p.nmax;
  r.lmax = p.lmax;
  fill_scale(r.scale, p.nmax, p.lmax, kBasisHO);
  const dim3 grid(nsys, (2 * r.K + kReduceLanes - 1) / kReduceLanes);
  if (p.prec == ETICS_MIXED_COMP32)
    hipLaunchKernelGGL(scf_reduce_batched_kernel<1>, grid, dim3(kReduceLanes), 0, st, r);
  else
    hipLaunchKernelGGL(scf_reduce_batched_kernel<0>, grid, dim3(kReduceLanes), 0, st, r);
  return hip_fail(hipGetLastError(), "scf_reduce_batched_kernel launch");
}

BatchedCoeffArgs batched_coeff_args(const CoeffPlan& p, const double* x, const double* y,
                                    const double* z, const double* m, const int64_t* offsets,
                                    const int* ustart, const int* usys, int nsys, int64_t ntotal,
                                    void* partials) {
  BatchedCoeffArgs a{};
  a.x = x;
  a.y = y;
  a.z = z;
  a.m = m;
  a.offsets = offsets;
  a.ustart = ustart;
  a.usys = usys;
  a.ntotal = ntotal;
  a.partials = partials;
  a.nsys = nsys;
  a.K = coeff_count(p.nmax, p.lmax);
  a.nmax = p.nmax;
  a.lmax = p.lmax;
  a.tp = p.tp;
  a.nblocks = p.nblocks;
  a.streams = p.streams;
  a.nchunks = p.nchunks;
  a.flush_tiles = p.flush_tiles;
  a.unit = p.unit;
  return a;
}

int launch_scf_coeffs_batched(const CoeffPlan& p, const double* x, const double* y, const double* z,
                              const double* m, const int64_t* offsets, const int* ustart,
                              const int* usys, int nsys, int64_t ntotal, double* A, double* B,
                              void* partials, hipStream_t st) {
  const BatchedCoeffArgs a = batched_coeff_args(p, x, y, z, m, offsets, ustart, usys, nsys, ntotal, partials);
  const int grid = coeff_grid(p, max_units(ntotal, nsys, p.unit));
  int rc = launch_coeff_any<true, false>(p, a, grid, st);
  if (rc) return rc;
  return launch_coeff_reduce_batched(p, partials, ustart, nsys, A, B, st);
}

}  // namespace etics
