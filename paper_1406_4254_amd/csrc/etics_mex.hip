// etics_mex.hip -- multipole expansion (MEX) potential and force on gfx950 (MI355X).
//
// The paper's MEX (Section 2.4, eqs. mex-phi, mex-qlm, mex-plm; implementation in
// Section 3.2) expands the Green's function: for particle i, the inward moments
//   q_lm(i) = sum over particles j before i of m_j r_j^l Ybar_lm(j) (cos, sin)(m phi_j)
// and the outward moments
//   p_lm(i) = sum over particles j after i of m_j r_j^-(l+1) Ybar_lm(j) (cos, sin)(m phi_j)
// are exclusive prefix / suffix sums over particles ordered by radius, and
//   Phi_i = -sum_l 4pi/(2l+1) sum_{m>=0} (2-delta_m0) Ybar_lm(i)
//           [(q^c r^-(l+1) + p^c r^l) cos m phi_i + (q^s r^-(l+1) + p^s r^l) sin m phi_i].
// The force is -grad Phi with q and p held fixed.
//
// Steps (all on the caller's stream):
//   1. mex_keys: FP64 key (x*x + y*y) + z*z, each operation rounded, as its IEEE bit
//      pattern (order-preserving for non-negative values), with the particle index.
//   2. LSD radix sort of (key, index), 8 bits per pass: per-block digit histograms,
//      one exclusive scan of the histograms, a stable scatter whose in-block ranks come
//      from wavefront ballots.  Stable, so equal keys stay in index order.
//   3. mex_tile_sums: per tile of sorted particles, the sums of the inward and outward
//      summands (FP64).
//   4. mex_tile_scan: exclusive prefix (inward) and suffix (outward) over tiles.
//   5. mex_force: per tile, the summands again, exclusive scans inside the tile in LDS,
//      plus the tile offsets, give q and p of every particle; then the synthesis and
//      the Cartesian force, scattered back to the caller's order.
// Radial powers, moments, scans and synthesis accumulations are FP64 in every mode;
// the MIXED modes evaluate Ybar_lm, its derivatives and (cos, sin)(m phi) in FP32.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "etics_device.hpp"
#include "etics_internal.hpp"

namespace etics {

constexpr int kMexTile = 256;       // sorted particles per tile (one per thread)
constexpr int kSortSeg = 4096;      // keys per radix block
constexpr int kSortThreads = 256;

// ------------------------------------------------------------------ keys
__global__ __launch_bounds__(256) void mex_keys_kernel(const double* __restrict__ x,
                                                       const double* __restrict__ y,
                                                       const double* __restrict__ z, int64_t n,
                                                       uint64_t* __restrict__ key,
                                                       uint32_t* __restrict__ idx) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double xx = __dmul_rn(x[i], x[i]);
  const double yy = __dmul_rn(y[i], y[i]);
  const double zz = __dmul_rn(z[i], z[i]);
  const double k = __dadd_rn(__dadd_rn(xx, yy), zz);
  key[i] = __double_as_longlong(k);
  idx[i] = uint32_t(i);
}

// ------------------------------------------------------------------ radix sort
// hist[d * nblk + b] = number of keys of block b with digit d
__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(const uint64_t* __restrict__ key,
                                                                  int64_t n, int shift, int nblk,
                                                                  uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t b0 = int64_t(blockIdx.x) * kSortSeg;
  const int64_t b1 = b0 + kSortSeg < n ? b0 + kSortSeg : n;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += kSortThreads)
    atomicAdd(&h[(key[i] >> shift) & 0xff], 1u);
  __syncthreads();
  hist[size_t(threadIdx.x) * nblk + blockIdx.x] = h[threadIdx.x];
}

// exclusive scan of hist (256 * nblk entries, digit-major) in one workgroup
__global__ __launch_bounds__(1024) void radix_scan_kernel(uint32_t* __restrict__ hist, int total) {
  __shared__ uint32_t part[1024];
  const int t = threadIdx.x;
  const int per = (total + 1023) / 1024;
  const int a = t * per, b = (a + per < total) ? a + per : total;
  uint32_t s = 0;
  for (int i = a; i < b; ++i) s += hist[i];
  part[t] = s;
  __syncthreads();
  // exclusive scan of the 1024 partial sums (Hillis-Steele on inclusive, then shift)
  for (int off = 1; off < 1024; off <<= 1) {
    const uint32_t v = t >= off ? part[t - off] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t run = t > 0 ? part[t - 1] : 0u;
  for (int i = a; i < b; ++i) {
    const uint32_t v = hist[i];
    hist[i] = run;
    run += v;
  }
}

// Stable scatter.  The block walks its segment in chunks of 256 keys (one per
// thread, in order); a key's rank among equal digits is (keys of that digit in
// earlier chunks) + (in earlier wavefronts of this chunk) + (in earlier lanes of its
// wavefront, from 8 ballots).
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint64_t* __restrict__ kout,
    uint32_t* __restrict__ vout, int64_t n, int shift, int nblk, const uint32_t* __restrict__ hist) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcnt[4][256];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  base[t] = hist[size_t(t) * nblk + blockIdx.x];
  const int64_t b0 = int64_t(blockIdx.x) * kSortSeg;
  const int64_t b1 = b0 + kSortSeg < n ? b0 + kSortSeg : n;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int64_t c0 = b0; c0 < b1; c0 += kSortThreads) {
    for (int q = 0; q < 4; ++q) wcnt[q][t] = 0;
    __syncthreads();
    const int64_t i = c0 + t;
    const bool valid = i < b1;
    const uint64_t k = valid ? kin[i] : 0ull;
    const uint32_t v = valid ? vin[i] : 0u;
    const uint32_t d = uint32_t(k >> shift) & 0xffu;
    uint64_t same = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const uint64_t bb = __ballot((d >> bit) & 1u);
      same &= ((d >> bit) & 1u) ? bb : ~bb;
    }
    const uint32_t below = uint32_t(__popcll(same & lt_mask));
    const uint32_t cnt = uint32_t(__popcll(same));
    // the lowest lane of each digit group publishes the wavefront's count
    if (valid && below == 0) wcnt[w][d] = cnt;
    __syncthreads();
    if (valid) {
      uint32_t r = base[d] + below;
      for (int q = 0; q < w; ++q) r += wcnt[q][d];
      kout[r] = k;
      vout[r] = v;
    }
    __syncthreads();
    base[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
    __syncthreads();
  }
}

// ------------------------------------------------------------------ basis
template <typename T>
struct MexParticle {
  double r, rinv;  // FP64 radial variables
  T ct, st, cp, sp;
  double mass;
  bool at_origin;
};

template <typename T>
__device__ __forceinline__ MexParticle<T> mex_particle(double x, double y, double z, double m) {
  MexParticle<T> p;
  const double R2 = x * x + y * y;
  p.r = sqrt(R2 + z * z);
  p.at_origin = !(p.r > 0.0);
  p.rinv = p.at_origin ? 0.0 : 1.0 / p.r;
  const double R = sqrt(R2);
  p.ct = T(p.at_origin ? 1.0 : z * p.rinv);
  p.st = T(R * p.rinv);
  const double iR = R > 0.0 ? 1.0 / R : 0.0;
  p.cp = T(R > 0.0 ? x * iR : 1.0);
  p.sp = T(y * iR);
  p.mass = m;
  return p;
}

// component slots of one l: 0 = (m=0, cos), 2m-1 = (m, cos), 2m = (m, sin); 2l+1 per side
template <int LB>
struct MexArgs {
  const double *x, *y, *z, *m;
  int64_t n;
  const uint32_t* perm;      // sorted position -> particle index
  double* tsum;              // [ntiles][2][(LB+1)^2]  tile sums: inward, outward
  double* toff;              // [ntiles][2][(LB+1)^2]  exclusive tile prefix / suffix
  double *pot, *ax, *ay, *az;
  int lmax, ntiles, want_pot, want_acc;
};

constexpr int mex_nc(int lb) { return (lb + 1) * (lb + 1); }
constexpr int mex_coff(int l) { return l * l; }  // first component of l (2l+1 per l)

// Per l: each thread writes its 2(2l+1) summands to LDS, then every column is summed
// (tile sums) or scanned (force).  Column c of the LDS block is component c with rows
// = threads (sorted order).
template <typename T, int LB, int l>
__device__ __forceinline__ void mex_summands_row(const MexParticle<T>& p, const T (&Y)[LB + 2][LB + 2],
                                                 const T* cm, const T* sm, double rl, double rm,
                                                 double* row) {
  // row[0 .. 2l]: inward (m r^l Ybar trig), row[2l+1 .. 4l+1]: outward (m r^-(l+1) Ybar trig)
  const double wi = p.mass * rl;
  const double wo = p.at_origin ? 0.0 : p.mass * rm;
  static_for<l + 1>([&](auto mc) {
    constexpr int m = decltype(mc)::value;
    constexpr int sc = m == 0 ? 0 : 2 * m - 1;
    const double yc = double(Y[l][m] * cm[m]);
    row[sc] = wi * yc;
    row[2 * l + 1 + sc] = wo * yc;
    if constexpr (m > 0) {
      const double ys = double(Y[l][m] * sm[m]);
      row[sc + 1] = wi * ys;
      row[2 * l + 1 + sc + 1] = wo * ys;
    }
  });
}

template <typename T, int LB, int r>
__device__ __forceinline__ void mex_legendre_row(T (&Y)[LB + 2][LB + 2], T ct, T st) {
  Y[r][r] = T(kTab.c1[r][r]) * st * Y[r - 1][r - 1];
  Y[r][r - 1] = T(kTab.c1[r][r - 1]) * ct * Y[r - 1][r - 1];
  static_for<(r >= 2 ? r - 1 : 0)>([&](auto mc) {
    constexpr int m = decltype(mc)::value;
    Y[r][m] = (T(kTab.c1[r][m]) * ct) * Y[r - 1][m] - T(kTab.c2[r][m]) * Y[r - 2][m];
  });
}

// tile sums of inward / outward summands
template <typename T, int LB>
__global__ __launch_bounds__(kMexTile) void mex_tile_sums_kernel(const MexArgs<LB> a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double* S = reinterpret_cast<double*>(lds_raw);  // [kMexTile][4l+2 (+1)]
  constexpr int NC = mex_nc(LB);
  const int t = threadIdx.x;
  const int64_t k = int64_t(blockIdx.x) * kMexTile + t;
  const bool valid = k < a.n;
  double px = 0, py = 0, pz = 0, pm = 0;
  if (valid) {
    const uint32_t i = a.perm[k];
    px = a.x[i];
    py = a.y[i];
    pz = a.z[i];
    pm = a.m[i];
  }
  const MexParticle<T> p = mex_particle<T>(px, py, pz, pm);
  T cm[LB + 1], sm[LB + 1];
  cm[0] = T(1);
  sm[0] = T(0);
#pragma unroll
  for (int m = 1; m <= LB; ++m) {
    cm[m] = cm[m - 1] * p.cp - sm[m - 1] * p.sp;
    sm[m] = sm[m - 1] * p.cp + cm[m - 1] * p.sp;
  }
  T Y[LB + 2][LB + 2];
  Y[0][0] = T(kTab.c1[0][0]);
  double rl = 1.0, rm = p.rinv;  // r^l, r^-(l+1)
  double* out = a.tsum + size_t(blockIdx.x) * 2 * NC;
  static_for<LB + 1>([&](auto lc) {
    constexpr int l = decltype(lc)::value;
    if (l > a.lmax) return;
    if constexpr (l >= 1) mex_legendre_row<T, LB, l>(Y, p.ct, p.st);
    constexpr int W = 2 * (2 * l + 1);
    constexpr int RS = W | 1;  // odd row stride (doubles)
    double* row = S + t * RS;
    if (valid) {
      mex_summands_row<T, LB, l>(p, Y, cm, sm, rl, rm, row);
    } else {
#pragma unroll
      for (int c = 0; c < W; ++c) row[c] = 0.0;
    }
    __syncthreads();
    // column sums: 4 threads per column, each over 64 rows in order, then in order
    constexpr int Q = 4;
    double part = 0.0;
    const int col = t / Q, seg = t % Q;
    if (col < W) {
      for (int rr = seg * (kMexTile / Q); rr < (seg + 1) * (kMexTile / Q); ++rr) part += S[rr * RS + col];
    }
    __syncthreads();
    if (col < W) S[seg * RS + col] = part;  // rows 0..Q-1 reused for the partials
    __syncthreads();
    if (t < W) {
      double s = 0.0;
      for (int q = 0; q < Q; ++q) s += S[q * RS + t];
      const int side = t < 2 * l + 1 ? 0 : 1;
      const int c = side == 0 ? t : t - (2 * l + 1);
      out[side * NC + mex_coff(l) + c] = s;
    }
    __syncthreads();
    rl *= p.r;
    rm *= p.rinv;
  });
}

// exclusive prefix (inward side) and suffix (outward side) over tiles; one thread per
// component column, serial in tile order
template <int LB>
__global__ __launch_bounds__(256) void mex_tile_scan_kernel(const MexArgs<LB> a) {
  constexpr int NC = mex_nc(LB);
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int nc = (a.lmax + 1) * (a.lmax + 1);
  if (c >= 2 * nc) return;
  const int side = c < nc ? 0 : 1;
  const int comp = side == 0 ? c : c - nc;
  double run = 0.0;
  if (side == 0) {
    for (int tl = 0; tl < a.ntiles; ++tl) {
      const size_t o = (size_t(tl) * 2 + 0) * NC + comp;
      const double v = a.tsum[o];
      a.toff[o] = run;
      run += v;
    }
  } else {
    for (int tl = a.ntiles - 1; tl >= 0; --tl) {
      const size_t o = (size_t(tl) * 2 + 1) * NC + comp;
      const double v = a.tsum[o];
      a.toff[o] = run;
      run += v;
    }
  }
}

// per-particle synthesis
template <typename T, int LB>
__global__ __launch_bounds__(kMexTile) void mex_force_kernel(const MexArgs<LB> a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double* S = reinterpret_cast<double*>(lds_raw);
  __shared__ double segtot[4][64];
  constexpr int NC = mex_nc(LB);
  const int t = threadIdx.x;
  const int64_t k = int64_t(blockIdx.x) * kMexTile + t;
  const bool valid = k < a.n;
  uint32_t pidx = 0;
  double px = 0, py = 0, pz = 0, pm = 0;
  if (valid) {
    pidx = a.perm[k];
    px = a.x[pidx];
    py = a.y[pidx];
    pz = a.z[pidx];
    pm = a.m[pidx];
  }
  const MexParticle<T> p = mex_particle<T>(px, py, pz, pm);
  T cm[LB + 1], sm[LB + 1];
  cm[0] = T(1);
  sm[0] = T(0);
#pragma unroll
  for (int m = 1; m <= LB; ++m) {
    cm[m] = cm[m - 1] * p.cp - sm[m - 1] * p.sp;
    sm[m] = sm[m - 1] * p.cp + cm[m - 1] * p.sp;
  }
  T Y[LB + 2][LB + 2];
  Y[0][0] = T(kTab.c1[0][0]);
  mex_legendre_row<T, LB, 1>(Y, p.ct, p.st);
  double rl = 1.0, rm = p.rinv;                      // r^l, r^-(l+1)
  double rlm1 = 0.0;                                 // r^(l-1)  (0 for l = 0)
  double Phi = 0.0, ar = 0.0, at = 0.0, ap = 0.0;
  const double* offs = a.toff + size_t(blockIdx.x) * 2 * NC;
  static_for<LB + 1>([&](auto lc) {
    constexpr int l = decltype(lc)::value;
    if (l > a.lmax) return;
    // Legendre row l+1 (for m Ybar / sin)
    mex_legendre_row<T, LB, l + 1>(Y, p.ct, p.st);
    constexpr int W = 2 * (2 * l + 1);
    constexpr int RS = W | 1;
    double* row = S + t * RS;
    if (valid) {
      mex_summands_row<T, LB, l>(p, Y, cm, sm, rl, rm, row);
    } else {
#pragma unroll
      for (int c = 0; c < W; ++c) row[c] = 0.0;
    }
    __syncthreads();
    // exclusive scans of every column inside the tile: 4 segments of 64 rows per
    // column; inward columns run forward, outward columns backward
    constexpr int Q = 4, SEGL = kMexTile / Q;
    const int col = t / Q, seg = t % Q;
    const bool fwd = col < 2 * l + 1;
    if (col < W) {
      double run = 0.0;
      if (fwd) {
        for (int rr = seg * SEGL; rr < (seg + 1) * SEGL; ++rr) {
          const double v = S[rr * RS + col];
          S[rr * RS + col] = run;
          run += v;
        }
      } else {
        for (int rr = (seg + 1) * SEGL - 1; rr >= seg * SEGL; --rr) {
          const double v = S[rr * RS + col];
          S[rr * RS + col] = run;
          run += v;
        }
      }
      segtot[seg][col] = run;
    }
    __syncthreads();
    if (col < W) {
      const int side = fwd ? 0 : 1;
      const int c = fwd ? col : col - (2 * l + 1);
      double off = offs[side * NC + mex_coff(l) + c];
      if (fwd) {
        for (int q = 0; q < seg; ++q) off += segtot[q][col];
      } else {
        for (int q = Q - 1; q > seg; --q) off += segtot[q][col];
      }
      for (int rr = seg * SEGL; rr < (seg + 1) * SEGL; ++rr) S[rr * RS + col] += off;
    }
    __syncthreads();
    // synthesis of this l from the particle's own q (row[0..2l]) and p (row[2l+1..])
    {
      const double g = 4.0 * kPi / (2.0 * l + 1.0);
      static_for<l + 1>([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        constexpr int sc = m == 0 ? 0 : 2 * m - 1;
        const double w = (m == 0 ? 1.0 : 2.0) * g;
        const double qc = row[sc], pc = row[2 * l + 1 + sc];
        const double qs = m > 0 ? row[sc + 1] : 0.0;
        const double ps = m > 0 ? row[2 * l + 1 + sc + 1] : 0.0;
        const double c = double(cm[m]), s = double(sm[m]);
        // radial factors: inward q r^-(l+1), outward p r^l; the inward part is absent
        // for a particle at the origin
        const double fq = p.at_origin ? 0.0 : rm;
        const double e = (qc * c + qs * s) * fq + (pc * c + ps * s) * rl;
        const double dr = p.at_origin ? (l >= 1 ? double(l) * rlm1 * (pc * c + ps * s) : 0.0)
                                      : (-(l + 1.0) * rm * p.rinv * (qc * c + qs * s) +
                                         double(l) * rlm1 * (pc * c + ps * s));
        // (1/r) x radial factor: q r^-(l+2), p r^(l-1)
        const double eo = p.at_origin ? (pc * c + ps * s) * rlm1
                                      : (qc * c + qs * s) * rm * p.rinv + (pc * c + ps * s) * rlm1;
        const double f = p.at_origin ? (ps * c - pc * s) * rlm1
                                     : (qs * c - qc * s) * rm * p.rinv + (ps * c - pc * s) * rlm1;
        const double y = double(Y[l][m]);
        Phi -= w * y * e;
        ar += w * y * dr;
        if constexpr (l >= 1) {
          T dY;
          if constexpr (m == 0) {
            dY = T(kTab.e1[l][0]) * Y[l][1];
          } else if constexpr (m + 1 <= l) {
            dY = T(kTab.e1[l][m]) * Y[l][m + 1] - T(kTab.e2[l][m]) * Y[l][m - 1];
          } else {
            dY = -T(kTab.e2[l][m]) * Y[l][m - 1];
          }
          at += w * double(dY) * eo;
          if constexpr (m >= 1) {
            const T mYs = -(T(kTab.f1[l][m]) * Y[l + 1][m + 1] + T(kTab.f2[l][m]) * Y[l + 1][m - 1]);
            ap += w * double(mYs) * f;
          }
        }
      });
    }
    __syncthreads();
    rlm1 = rl;
    rl *= p.r;
    rm *= p.rinv;
  });
  if (!valid) return;
  if (a.want_pot) a.pot[pidx] = Phi;
  if (a.want_acc) {
    const double st = double(p.st), ct = double(p.ct), cp = double(p.cp), sp = double(p.sp);
    a.ax[pidx] = st * cp * ar + ct * cp * at - sp * ap;
    a.ay[pidx] = st * sp * ar + ct * sp * at + cp * ap;
    a.az[pidx] = ct * ar - st * at;
  }
}

// ================================================================ host side
namespace {

struct MexLayout {
  size_t off_key0, off_key1, off_idx0, off_idx1, off_hist, off_tsum, off_toff, total;
  int nblk, ntiles, lb;
};

MexLayout mex_layout(int64_t n, int lmax) {
  MexLayout L{};
  L.lb = lmax <= 2 ? 2 : lmax <= 6 ? 6 : lmax <= 10 ? 10 : 14;
  L.nblk = int((n + kSortSeg - 1) / kSortSeg);
  if (L.nblk < 1) L.nblk = 1;
  L.ntiles = int((n + kMexTile - 1) / kMexTile);
  if (L.ntiles < 1) L.ntiles = 1;
  const size_t NC = size_t(mex_nc(L.lb));
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  const size_t nn = size_t(n > 0 ? n : 1);
  L.off_key0 = take(nn * 8);
  L.off_key1 = take(nn * 8);
  L.off_idx0 = take(nn * 4);
  L.off_idx1 = take(nn * 4);
  L.off_hist = take(size_t(256) * L.nblk * 4);
  L.off_tsum = take(size_t(L.ntiles) * 2 * NC * 8);
  L.off_toff = take(size_t(L.ntiles) * 2 * NC * 8);
  L.total = o;
  return L;
}

template <typename T, int LB>
int launch_mex_lb(const MexArgs<LB>& a, int ntiles, hipStream_t st) {
  // largest LDS block: 256 rows x (2(2l+1) | 1) doubles at l = LB
  const size_t lds = size_t(kMexTile) * ((2 * (2 * LB + 1)) | 1) * 8;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(mex_tile_sums_kernel<T, LB>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e == hipSuccess)
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(mex_force_kernel<T, LB>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(mex)");
    attr_set = true;
  }
  hipLaunchKernelGGL((mex_tile_sums_kernel<T, LB>), dim3(ntiles), dim3(kMexTile), lds, st, a);
  int rc = hip_fail(hipGetLastError(), "mex_tile_sums_kernel launch");
  if (rc) return rc;
  const int ncol = 2 * (a.lmax + 1) * (a.lmax + 1);
  hipLaunchKernelGGL((mex_tile_scan_kernel<LB>), dim3((ncol + 255) / 256), dim3(256), 0, st, a);
  rc = hip_fail(hipGetLastError(), "mex_tile_scan_kernel launch");
  if (rc) return rc;
  rc = hook_before(st);
  if (rc) return rc;
  hipLaunchKernelGGL((mex_force_kernel<T, LB>), dim3(ntiles), dim3(kMexTile), lds, st, a);
  rc = hip_fail(hipGetLastError(), "mex_force_kernel launch");
  return rc ? rc : hook_after(st);
}

template <typename T>
int launch_mex_t(int lb, const double* x, const double* y, const double* z, const double* m,
                 int64_t n, int lmax, const uint32_t* perm, double* tsum, double* toff, int ntiles,
                 int outputs, double* pot, double* ax, double* ay, double* az, hipStream_t st) {
  auto fill = [&](auto& a) {
    a.x = x;
    a.y = y;
    a.z = z;
    a.m = m;
    a.n = n;
    a.perm = perm;
    a.tsum = tsum;
    a.toff = toff;
    a.pot = pot;
    a.ax = ax;
    a.ay = ay;
    a.az = az;
    a.lmax = lmax;
    a.ntiles = ntiles;
    a.want_pot = (outputs & ETICS_POT) ? 1 : 0;
    a.want_acc = (outputs & ETICS_ACC) ? 1 : 0;
  };
  switch (lb) {
    case 2: { MexArgs<2> a{}; fill(a); return launch_mex_lb<T, 2>(a, ntiles, st); }
    case 6: { MexArgs<6> a{}; fill(a); return launch_mex_lb<T, 6>(a, ntiles, st); }
    case 10: { MexArgs<10> a{}; fill(a); return launch_mex_lb<T, 10>(a, ntiles, st); }
    default: { MexArgs<14> a{}; fill(a); return launch_mex_lb<T, 14>(a, ntiles, st); }
  }
}

}  // namespace

size_t mex_ws_bytes(int64_t n, int lmax) { return mex_layout(n, lmax).total; }

int launch_mex_force(const double* x, const double* y, const double* z, const double* m, int64_t n,
                     int lmax, int prec, int outputs, double* pot, double* ax, double* ay,
                     double* az, void* ws, hipStream_t st) {
  const MexLayout L = mex_layout(n, lmax);
  char* base = reinterpret_cast<char*>(ws);
  uint64_t* k0 = reinterpret_cast<uint64_t*>(base + L.off_key0);
  uint64_t* k1 = reinterpret_cast<uint64_t*>(base + L.off_key1);
  uint32_t* i0 = reinterpret_cast<uint32_t*>(base + L.off_idx0);
  uint32_t* i1 = reinterpret_cast<uint32_t*>(base + L.off_idx1);
  uint32_t* hist = reinterpret_cast<uint32_t*>(base + L.off_hist);
  double* tsum = reinterpret_cast<double*>(base + L.off_tsum);
  double* toff = reinterpret_cast<double*>(base + L.off_toff);

  hipLaunchKernelGGL(mex_keys_kernel, dim3(int((n + 255) / 256)), dim3(256), 0, st, x, y, z, n, k0, i0);
  int rc = hip_fail(hipGetLastError(), "mex_keys_kernel launch");
  if (rc) return rc;
  for (int pass = 0; pass < 8; ++pass) {
    const int shift = 8 * pass;
    hipLaunchKernelGGL(radix_hist_kernel, dim3(L.nblk), dim3(kSortThreads), 0, st, k0, n, shift,
                       L.nblk, hist);
    hipLaunchKernelGGL(radix_scan_kernel, dim3(1), dim3(1024), 0, st, hist, 256 * L.nblk);
    hipLaunchKernelGGL(radix_scatter_kernel, dim3(L.nblk), dim3(kSortThreads), 0, st, k0, i0, k1, i1,
                       n, shift, L.nblk, hist);
    rc = hip_fail(hipGetLastError(), "radix sort launch");
    if (rc) return rc;
    uint64_t* tk = k0;
    k0 = k1;
    k1 = tk;
    uint32_t* ti = i0;
    i0 = i1;
    i1 = ti;
  }
  // after an even number of passes the sorted order is back in (k0, i0)
  if (prec == ETICS_FP64)
    return launch_mex_t<double>(L.lb, x, y, z, m, n, lmax, i0, tsum, toff, L.ntiles, outputs, pot,
                                ax, ay, az, st);
  return launch_mex_t<float>(L.lb, x, y, z, m, n, lmax, i0, tsum, toff, L.ntiles, outputs, pot, ax,
                             ay, az, st);
}

}  // namespace etics
