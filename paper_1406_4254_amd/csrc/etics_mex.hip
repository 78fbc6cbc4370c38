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
//   2. LSD radix sort of (key, index), 8 bits per pass, three kernels per pass: the
//      digit counts of every tile of keys, a scan of each digit's counts over the tiles,
//      then every tile ranks its keys stably in LDS and writes them as runs of equal
//      digit.  Stable, so equal keys stay in index order.
//   3. tile sums: per tile of 128 sorted particles, the sums of the inward and outward
//      summands (FP64).  FP32-basis modes (mex_tile_sums_pair_kernel): one wavefront per
//      tile, two particles per lane; the lane pair sums go through the wavefront's own
//      LDS block and each 16-lane DPP row sums one column (4 rows a lane, then a row
//      tree).  FP64 (mex_tile_sums_kernel): one particle per thread, each 16-lane row
//      sums one LDS column, a lane adding 8 consecutive rows before a row tree.
//   4. tile offsets: exclusive prefix (inward) and suffix (outward) over tiles, in
//      three parallel steps (sums of blocks of tiles, a scan over the blocks, then the
//      tiles of every block).
//   5. mex_force: per tile (one wavefront, two particles per lane), the summands again;
//      exclusive scans inside the tile, in registers with DPP lane moves (prefix over
//      the lanes for inward sums, the same tree over the reversed lanes for outward
//      sums), plus the tile offsets, give q and p of every particle; then the synthesis
//      and the Cartesian force, scattered back to the caller's order.  The FP64 mode
//      stages each column in LDS instead (one particle per thread), scanned by one
//      wavefront with the same lane tree.
// Radial powers, moments, scans and synthesis accumulations are FP64 in every mode;
// the MIXED modes evaluate Ybar_lm, its derivatives and (cos, sin)(m phi) in FP32.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "etics_device.hpp"
#include "etics_internal.hpp"

namespace etics {

constexpr int kMexTile = 128;  // sorted particles per tile (tile sums: one per thread; force: two per lane)
// LDS column of a tile in the tile-sum kernel: the rows in 16 groups of 8 (one group per
// lane of a 16-lane DPP row), with 2 doubles of padding after every second group, so
// the four 16-byte reads of a group by 8 neighbouring lanes fall on distinct banks
constexpr int kMexColStride = kMexTile + 2 * (kMexTile / 16);  // 144 doubles
__device__ __forceinline__ int mex_row_pos(int t) { return t + 2 * (t >> 4); }
constexpr int kMexBlockTiles = 16;  // tiles per block of the tile-offset scan
constexpr int kSortThreads = 256;
constexpr int kSortKPT = 8;                         // keys per thread of a radix pass
constexpr int kSortTile = kSortThreads * kSortKPT;  // keys per tile of a radix pass
constexpr int kSortPasses = 8;                      // 8-bit digits of a 64-bit key

// ------------------------------------------------------------------ block scans
// exclusive prefix sum of one value per thread over a workgroup of 256 threads
// (4 wavefronts); `wsum` is 4 words of LDS.  Returns the exclusive prefix; *total gets
// the workgroup sum.
__device__ __forceinline__ uint32_t block_excl_scan_u32(uint32_t v, uint32_t* wsum, uint32_t* total) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  uint32_t incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o);
    if (lane >= o) incl += y;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t s = wsum[q];
    before += q < w ? s : 0u;
    all += s;
  }
  __syncthreads();
  *total = all;
  return before + incl - v;
}

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
// The lanes of a wavefront whose digit equals this lane's (8 ballots; only valid lanes)
__device__ __forceinline__ uint64_t same_digit_lanes(uint32_t d, bool valid) {
  uint64_t same = __ballot(valid);
#pragma unroll
  for (int bit = 0; bit < 8; ++bit) {
    const uint64_t bb = __ballot((d >> bit) & 1u);
    same &= ((d >> bit) & 1u) ? bb : ~bb;
  }
  return same;
}

// counts[d * ntiles + tile] = keys of the tile with digit d.  Lanes with equal digits
// add their number once, so a digit shared by many keys (the exponent bytes) does not
// serialize on one LDS word.
__global__ __launch_bounds__(kSortThreads) void radix_count_kernel(const uint64_t* __restrict__ key,
                                                                   int64_t n, int shift, int ntiles,
                                                                   uint32_t* __restrict__ counts) {
  __shared__ uint32_t h[256];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  h[t] = 0;
  __syncthreads();
  const int64_t t0 = int64_t(blockIdx.x) * kSortTile;
  const int tn = int(n - t0 < kSortTile ? n - t0 : kSortTile);
  constexpr int Q = kSortTile / 4;
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  uint64_t k[kSortKPT];
#pragma unroll
  for (int j = 0; j < kSortKPT; ++j) {
    const int i = w * Q + j * 64 + lane;
    k[j] = i < tn ? key[t0 + i] : 0ull;
  }
#pragma unroll
  for (int j = 0; j < kSortKPT; ++j) {
    const bool valid = w * Q + j * 64 + lane < tn;
    const uint32_t d = uint32_t(k[j] >> shift) & 0xffu;
    const uint64_t same = same_digit_lanes(d, valid);
    if (valid && (same & lt_mask) == 0) atomicAdd(&h[d], uint32_t(__popcll(same)));
  }
  __syncthreads();
  counts[size_t(t) * ntiles + blockIdx.x] = h[t];
}

// counts[d * ntiles + b] -> exclusive prefix over tiles b of digit d (in place);
// totals[d] = keys with digit d.  One workgroup per digit.
__global__ __launch_bounds__(256) void radix_digit_scan_kernel(uint32_t* __restrict__ counts, int ntiles,
                                                               uint32_t* __restrict__ totals) {
  __shared__ uint32_t wsum[4];
  uint32_t* row = counts + size_t(blockIdx.x) * ntiles;
  const int t = threadIdx.x;
  uint32_t carry = 0;
  for (int base = 0; base < ntiles; base += 4 * 256) {
    uint32_t v[4], s = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = base + 4 * t + j;
      v[j] = i < ntiles ? row[i] : 0u;
      s += v[j];
    }
    uint32_t chunk;
    uint32_t run = carry + block_excl_scan_u32(s, wsum, &chunk);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = base + 4 * t + j;
      if (i < ntiles) row[i] = run;
      run += v[j];
    }
    carry += chunk;
  }
  if (t == 0) totals[blockIdx.x] = carry;
}

// Stable scatter of one tile: the keys are ranked in LDS (wavefront w ranks keys
// [w Q, (w+1) Q) of the tile in order, 64 at a time: a key's rank among equal digits of
// its wavefront's range is the running count of the digit plus the equal digits in lower
// lanes; the lowest lane of each digit group advances the count; one wavefront reads and
// writes its own row of counts, in program order, so no barrier is needed), placed in
// digit order in LDS, and written out so that consecutive threads write consecutive
// positions of each digit's run.
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint64_t* __restrict__ kout,
    uint32_t* __restrict__ vout, int64_t n, int shift, int ntiles, const uint32_t* __restrict__ counts,
    const uint32_t* __restrict__ totals) {
  __shared__ uint64_t sk[kSortTile];
  __shared__ uint32_t sv[kSortTile];
  __shared__ uint32_t cnt[4][256];  // per wavefront: running digit counts, then bases
  __shared__ uint32_t gbase[256];
  __shared__ uint32_t wsum[4];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  for (int i = t; i < 4 * 256; i += kSortThreads) (&cnt[0][0])[i] = 0;
  __syncthreads();
  const int tile = blockIdx.x;
  const int64_t t0 = int64_t(tile) * kSortTile;
  const int tn = int(n - t0 < kSortTile ? n - t0 : kSortTile);  // keys of this tile
  constexpr int Q = kSortTile / 4;
  uint64_t k[kSortKPT];
  uint32_t v[kSortKPT], rank[kSortKPT];
#pragma unroll
  for (int j = 0; j < kSortKPT; ++j) {
    const int i = w * Q + j * 64 + lane;
    k[j] = i < tn ? kin[t0 + i] : 0ull;
    v[j] = i < tn ? vin[t0 + i] : 0u;
  }
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int j = 0; j < kSortKPT; ++j) {
    const bool valid = w * Q + j * 64 + lane < tn;
    const uint32_t d = uint32_t(k[j] >> shift) & 0xffu;
    const uint64_t same = same_digit_lanes(d, valid);
    const uint32_t below = uint32_t(__popcll(same & lt_mask));
    uint32_t r = 0;
    if (valid) {
      r = cnt[w][d];
      if (below == 0) cnt[w][d] = r + uint32_t(__popcll(same));
    }
    rank[j] = r + below;
  }
  __syncthreads();

  // thread d: the first position of digit d in the tile's sorted order and of each
  // wavefront's keys of d; where the tile's run of d starts in the output
  const int d = t;
  const uint32_t c0 = cnt[0][d], c1 = cnt[1][d], c2 = cnt[2][d];
  const uint32_t own = c0 + c1 + c2 + cnt[3][d];
  uint32_t total;
  const uint32_t lstart = block_excl_scan_u32(own, wsum, &total);
  const uint32_t dstart = block_excl_scan_u32(totals[d], wsum, &total);
  cnt[0][d] = lstart;
  cnt[1][d] = lstart + c0;
  cnt[2][d] = lstart + c0 + c1;
  cnt[3][d] = lstart + c0 + c1 + c2;
  gbase[d] = dstart + counts[size_t(d) * ntiles + tile] - lstart;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kSortKPT; ++j) {
    if (w * Q + j * 64 + lane < tn) {
      const uint32_t pos = cnt[w][uint32_t(k[j] >> shift) & 0xffu] + rank[j];
      if (pos < uint32_t(kSortTile)) {  // always true; keeps a logic error inside the tile
        sk[pos] = k[j];
        sv[pos] = v[j];
      }
    }
  }
  __syncthreads();
  for (int i = t; i < tn; i += kSortThreads) {
    const uint64_t kk = sk[i];
    const uint32_t pos = gbase[uint32_t(kk >> shift) & 0xffu] + uint32_t(i);
    if (int64_t(pos) < n) {  // always true; keeps a logic error inside the output
      kout[pos] = kk;
      vout[pos] = sv[i];
    }
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
  double* bsum;              // [nblocks][2][(LB+1)^2] sums of blocks of tiles, then their
                             //                        exclusive prefix / suffix
  double *pot, *ax, *ay, *az;
  int lmax, ntiles, nblocks, want_pot, want_acc;
};

constexpr int mex_nc(int lb) { return (lb + 1) * (lb + 1); }
constexpr int mex_coff(int l) { return l * l; }  // first component of l (2l+1 per l)

// Per l and side (0 = inward, 1 = outward): each thread writes its 2l+1 summands of that
// side to LDS, then every column is summed (tile sums) or scanned (force).  The LDS block
// is column-major: component c of the particle in row (sorted position within the tile)
// t is at col0[c * CS], col0 = S + t.  Staging one side at a time halves the LDS of a
// workgroup, so more workgroups share a CU.
template <typename T, int LB, int l, int SIDE, int CS>
__device__ __forceinline__ void mex_summands_col(const MexParticle<T>& p, const T (&Y)[LB + 2][LB + 2],
                                                 const T* cm, const T* sm, double rl, double rm,
                                                 bool valid, double* col0) {
  // inward: m r^l Ybar trig; outward: m r^-(l+1) Ybar trig (0 at the origin, rm = 0)
  const double wgt = valid ? p.mass * (SIDE == 0 ? rl : rm) : 0.0;
  static_for<l + 1>([&](auto mc) {
    constexpr int m = decltype(mc)::value;
    constexpr int sc = m == 0 ? 0 : 2 * m - 1;
    col0[sc * CS] = wgt * double(Y[l][m] * cm[m]);
    if constexpr (m > 0) col0[(sc + 1) * CS] = wgt * double(Y[l][m] * sm[m]);
  });
}

// Wavefront-wide sums of one FP64 value per lane with DPP lane moves (each 32-bit half
// moved separately, zero where the source lane is out of range): a Hillis-Steele scan
// inside each row of 16 lanes, then the row totals carried by the row broadcasts.  The
// tree is fixed, so results do not depend on scheduling.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, int(b & 0xffffffffll), CTRL, ROW_MASK, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, ROW_MASK, 0xf, true);
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              static_cast<long long>(static_cast<unsigned int>(lo)));
}
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppWaveShr1 = 0x138, kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;

// inclusive prefix over lanes 0..lane
__device__ __forceinline__ double wave_incl_prefix(double x) {
  x += dpp_move<kDppRowShr1, 0xf>(x);
  x += dpp_move<kDppRowShr2, 0xf>(x);
  x += dpp_move<kDppRowShr4, 0xf>(x);
  x += dpp_move<kDppRowShr8, 0xf>(x);
  x += dpp_move<kDppRowBcast15, 0xa>(x);  // last lane of rows 0, 2 into rows 1, 3
  x += dpp_move<kDppRowBcast31, 0xc>(x);  // lane 31 into rows 2, 3
  return x;
}
// inclusive prefix inside each row of 16 lanes
__device__ __forceinline__ double row16_incl_prefix(double x) {
  x += dpp_move<kDppRowShr1, 0xf>(x);
  x += dpp_move<kDppRowShr2, 0xf>(x);
  x += dpp_move<kDppRowShr4, 0xf>(x);
  x += dpp_move<kDppRowShr8, 0xf>(x);
  return x;
}
// exclusive prefix over lanes 0..lane-1 (0 in lane 0)
__device__ __forceinline__ double wave_excl_prefix(double x) {
  return dpp_move<kDppWaveShr1, 0xf>(wave_incl_prefix(x));
}
// The 8 rows of group g of a padded column (rows 8g .. 8g+7), four 16-byte reads
__device__ __forceinline__ void mex_group_read(const double* col, int g, double (&v)[8]) {
  const double2* p = reinterpret_cast<const double2*>(col + mex_row_pos(8 * g));
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double2 w = p[i];
    v[2 * i] = w.x;
    v[2 * i + 1] = w.y;
  }
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

// per-particle set-up shared by the tile-sum and force kernels
template <typename T, int LB>
struct MexLane {
  MexParticle<T> p;
  T cm[LB + 1], sm[LB + 1];
  T Y[LB + 2][LB + 2];
  uint32_t pidx;
  bool valid;

  __device__ __forceinline__ void load(const MexArgs<LB>& a, int64_t k) {
    valid = k < a.n;
    pidx = 0;
    double px = 0, py = 0, pz = 0, pm = 0;
    if (valid) {
      pidx = a.perm[k];
      px = a.x[pidx];
      py = a.y[pidx];
      pz = a.z[pidx];
      pm = a.m[pidx];
    }
    p = mex_particle<T>(px, py, pz, pm);
    cm[0] = T(1);
    sm[0] = T(0);
#pragma unroll
    for (int m = 1; m <= LB; ++m) {
      cm[m] = cm[m - 1] * p.cp - sm[m - 1] * p.sp;
      sm[m] = sm[m - 1] * p.cp + cm[m - 1] * p.sp;
    }
    Y[0][0] = T(kTab.c1[0][0]);
  }
};

// tile sums of inward / outward summands.  Each 16-lane row of a wavefront sums one
// column: a lane adds its group of 8 rows in order, then a row tree of the 16 lane
// sums; the last lane of the row holds the total.  The two wavefronts take 8 columns
// per round.
template <typename T, int LB>
__global__ __launch_bounds__(kMexTile) void mex_tile_sums_kernel(const MexArgs<LB> a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double* S = reinterpret_cast<double*>(lds_raw);  // [2l+1][kMexColStride], one side at a time
  constexpr int NC = mex_nc(LB);
  const int t = threadIdx.x, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);  // uniform: scalar addressing
  const int drow = lane >> 4, k = lane & 15;                // DPP row (column), group
  MexLane<T, LB> q;
  q.load(a, int64_t(blockIdx.x) * kMexTile + t);
  double rl = 1.0, rm = q.p.rinv;  // r^l, r^-(l+1)
  double* out = a.tsum + size_t(blockIdx.x) * 2 * NC;
  static_for<LB + 1>([&](auto lc) {
    constexpr int l = decltype(lc)::value;
    if (l > a.lmax) return;
    if constexpr (l >= 1) mex_legendre_row<T, LB, l>(q.Y, q.p.ct, q.p.st);
    constexpr int H = 2 * l + 1;
    static_for<2>([&](auto sidec) {
      constexpr int side = decltype(sidec)::value;
      mex_summands_col<T, LB, l, side, kMexColStride>(q.p, q.Y, q.cm, q.sm, rl, rm, q.valid,
                                                      S + mex_row_pos(t));
      __syncthreads();
      static_for<(H + 7) / 8>([&](auto jc) {
        const int c = 8 * decltype(jc)::value + 4 * wave + drow;
        const int cc = c < H ? c : H - 1;  // rows past the last column read a valid one
        double v[8];
        mex_group_read(S + cc * kMexColStride, k, v);
        double sum = v[0];
#pragma unroll
        for (int i = 1; i < 8; ++i) sum += v[i];
        const double tot = row16_incl_prefix(sum);
        if (k == 15 && c < H) out[side * NC + mex_coff(l) + c] = tot;
      });
      __syncthreads();
    });
    rl *= q.p.r;
    rm *= q.p.rinv;
  });
}

// orders a wavefront's LDS accesses (lanes read what other lanes of it wrote)
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Tile sums with two particles per lane (the FP32-basis modes): every wavefront takes a
// tile of kMexTile sorted particles on its own (lane k: rows 2k and 2k+1).  Per l and
// side the lanes write their pair sums (one row per lane) to the wavefront's own LDS
// block, then each 16-lane DPP row sums one column: a lane adds 4 consecutive rows,
// then a row tree.  Half the LDS traffic of one particle per thread, and no workgroup
// barrier.
constexpr int kMexPairWaves = 2;                    // wavefronts (tiles) per workgroup
constexpr int kMexPairStride = 64 + 2 * (64 / 16);  // doubles per column: 64 rows, padded
// padded position of row r: 2 doubles after every 16 rows, so the 16-byte reads of 8
// neighbouring lanes (4 rows each) fall on distinct banks
__device__ __forceinline__ int mex_pair_pos(int r) { return r + 2 * (r >> 4); }
constexpr size_t mex_pair_lds_bytes(int lb) {
  return size_t(kMexPairWaves) * (2 * lb + 1) * kMexPairStride * 8;
}
static_assert(mex_pair_lds_bytes(14) <= 65536, "MEX tile-sum LDS beyond the default limit");

template <typename T, int LB>
__global__ __launch_bounds__(64 * kMexPairWaves) void mex_tile_sums_pair_kernel(const MexArgs<LB> a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  constexpr int NC = mex_nc(LB);
  constexpr int CS = kMexPairStride;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tile = blockIdx.x * kMexPairWaves + wave;
  if (tile >= a.ntiles) return;  // the whole wavefront
  double* S = reinterpret_cast<double*>(lds_raw) + wave * (2 * LB + 1) * CS;
  const int drow = lane >> 4, k = lane & 15;  // DPP row (column of a group of 4), group
  MexLane<T, LB> q0, q1;
  const int64_t k0 = int64_t(tile) * kMexTile + 2 * lane;
  q0.load(a, k0);
  q1.load(a, k0 + 1);
  double rl0 = 1.0, rm0 = q0.p.rinv, rl1 = 1.0, rm1 = q1.p.rinv;  // r^l, r^-(l+1)
  double* out = a.tsum + size_t(tile) * 2 * NC;
  static_for<LB + 1>([&](auto lc) {
    constexpr int l = decltype(lc)::value;
    if (l > a.lmax) return;
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (l >= 1) {
      mex_legendre_row<T, LB, l>(q0.Y, q0.p.ct, q0.p.st);
      mex_legendre_row<T, LB, l>(q1.Y, q1.p.ct, q1.p.st);
    }
    constexpr int H = 2 * l + 1;
    static_for<2>([&](auto sidec) {
      constexpr int side = decltype(sidec)::value;
      const double w0 = q0.valid ? q0.p.mass * (side == 0 ? rl0 : rm0) : 0.0;
      const double w1 = q1.valid ? q1.p.mass * (side == 0 ? rl1 : rm1) : 0.0;
      static_for<l + 1>([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        constexpr int sc = m == 0 ? 0 : 2 * m - 1;
        S[sc * CS + mex_pair_pos(lane)] =
            w0 * double(q0.Y[l][m] * q0.cm[m]) + w1 * double(q1.Y[l][m] * q1.cm[m]);
        if constexpr (m > 0)
          S[(sc + 1) * CS + mex_pair_pos(lane)] =
              w0 * double(q0.Y[l][m] * q0.sm[m]) + w1 * double(q1.Y[l][m] * q1.sm[m]);
      });
      wave_lds_sync();
      static_for<(H + 3) / 4>([&](auto jc) {
        const int c = 4 * decltype(jc)::value + drow;
        const int cc = c < H ? c : H - 1;  // rows past the last column read a valid one
        const double2* g = reinterpret_cast<const double2*>(S + cc * CS + mex_pair_pos(4 * k));
        const double2 u = g[0], v = g[1];
        const double tot = row16_incl_prefix(((u.x + u.y) + v.x) + v.y);
        if (k == 15 && c < H) out[side * NC + mex_coff(l) + c] = tot;
      });
      wave_lds_sync();  // the next side or l writes the block again
    });
    rl0 *= q0.p.r;
    rm0 *= q0.p.rinv;
    rl1 *= q1.p.r;
    rm1 *= q1.p.rinv;
  });
}

// tile offsets, step 1: sums of blocks of kMexBlockTiles tiles (one workgroup per block)
template <int LB>
__global__ __launch_bounds__(256) void mex_block_sums_kernel(const MexArgs<LB> a) {
  constexpr int NC = mex_nc(LB);
  const int ncu = (a.lmax + 1) * (a.lmax + 1);
  const int b = blockIdx.x;
  const int t0 = b * kMexBlockTiles;
  const int t1 = t0 + kMexBlockTiles < a.ntiles ? t0 + kMexBlockTiles : a.ntiles;
  for (int c = threadIdx.x; c < 2 * ncu; c += blockDim.x) {
    const int side = c < ncu ? 0 : 1;
    const int comp = side == 0 ? c : c - ncu;
    double s = 0.0;
    for (int tl = t0; tl < t1; ++tl) s += a.tsum[(size_t(tl) * 2 + side) * NC + comp];
    a.bsum[(size_t(b) * 2 + side) * NC + comp] = s;
  }
}

// step 2: exclusive prefix (inward) / suffix (outward) over the blocks, in place; one
// wavefront per column: lane k takes a run of consecutive blocks (in scan order: forward
// for inward, backward for outward), then a lane tree gives the runs before it
template <int LB>
__global__ __launch_bounds__(256) void mex_block_scan_kernel(const MexArgs<LB> a) {
  constexpr int NC = mex_nc(LB);
  const int ncu = (a.lmax + 1) * (a.lmax + 1);
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= 2 * ncu) return;  // whole wavefronts leave together
  const int side = c < ncu ? 0 : 1;
  const int comp = side == 0 ? c : c - ncu;
  const int nb = a.nblocks;
  const int run = (nb + 63) / 64;
  auto at = [&](int k) {  // k-th block in scan order
    const int b = side == 0 ? k : nb - 1 - k;
    return a.bsum + (size_t(b) * 2 + side) * NC + comp;
  };
  const int k0 = lane * run;
  double tot = 0.0;
  for (int k = k0; k < k0 + run && k < nb; ++k) tot += *at(k);
  double acc = wave_excl_prefix(tot);
  for (int k = k0; k < k0 + run && k < nb; ++k) {
    double* e = at(k);
    const double v = *e;
    *e = acc;
    acc += v;
  }
}

// step 3: the tiles of every block, starting from the block's offset
template <int LB>
__global__ __launch_bounds__(256) void mex_tile_offsets_kernel(const MexArgs<LB> a) {
  constexpr int NC = mex_nc(LB);
  const int ncu = (a.lmax + 1) * (a.lmax + 1);
  const int b = blockIdx.x;
  const int t0 = b * kMexBlockTiles;
  const int t1 = t0 + kMexBlockTiles < a.ntiles ? t0 + kMexBlockTiles : a.ntiles;
  for (int c = threadIdx.x; c < 2 * ncu; c += blockDim.x) {
    const int side = c < ncu ? 0 : 1;
    const int comp = side == 0 ? c : c - ncu;
    double run = a.bsum[(size_t(b) * 2 + side) * NC + comp];
    for (int k = t0; k < t1; ++k) {
      const int tl = side == 0 ? k : t1 - 1 - (k - t0);
      const size_t o = (size_t(tl) * 2 + side) * NC + comp;
      const double v = a.tsum[o];
      a.toff[o] = run;
      run += v;
    }
  }
}

// the value of lane 63 - lane (one wavefront): the lane order reversed
__device__ __forceinline__ double lane_reverse(double x) {
  const int addr = (63 - int(threadIdx.x & 63)) << 2;
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_ds_bpermute(addr, int(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_ds_bpermute(addr, int(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              static_cast<long long>(static_cast<unsigned int>(lo)));
}
// exclusive suffix over lanes lane+1..63 (0 in lane 63): the prefix tree run on the
// reversed lane order
__device__ __forceinline__ double wave_excl_suffix(double x) {
  return lane_reverse(wave_excl_prefix(lane_reverse(x)));
}

// Moments of one column at the two particles of a lane (sorted rows 2k and 2k+1 of the
// tile): inward = exclusive prefix along the tile's order, outward = exclusive suffix;
// `off` is the tile's offset from the other tiles.  The pair sum is scanned over the
// lanes, then the pair's first row in scan order takes the scan value and the second
// adds the first's summand.
__device__ __forceinline__ void mex_pair_inward(double s0, double s1, double off, double& v0, double& v1) {
  const double base = off + wave_excl_prefix(s0 + s1);
  v0 = base;
  v1 = base + s0;
}
__device__ __forceinline__ void mex_pair_outward(double s0, double s1, double off, double& v0, double& v1) {
  const double base = off + wave_excl_suffix(s1 + s0);
  v1 = base;
  v0 = base + s1;
}

// Angular sums of one l at one particle, over m, from the moments: with
// A = v^c cos m phi + v^s sin m phi and B = v^s cos m phi - v^c sin m phi (v = q inward,
// p outward) and w = (2 - delta_m0) 4 pi / (2l + 1):
//   y = sum w Ybar A,  d = sum w dYbar/dtheta A,  s = sum w (m Ybar / sin theta) B.
// Then Phi -= y_q r^-(l+1) + y_p r^l, a_r += d/dr of the same, a_theta and a_phi take d
// and s with the (1/r) x radial factors.
struct MexLSums {
  double yq = 0.0, yp = 0.0, dq = 0.0, dp = 0.0, sq = 0.0, sp = 0.0;
};
template <typename T, int LB, int l, int m>
__device__ __forceinline__ void mex_lsums_add(const MexLane<T, LB>& q, double qc, double qs, double pc,
                                              double ps, MexLSums& S) {
  const T w = T((m == 0 ? 1.0 : 2.0) * 4.0 * kPi / (2.0 * l + 1.0));
  const double c = double(q.cm[m]), s = double(q.sm[m]);
  const double Aq = m > 0 ? qc * c + qs * s : qc;  // cm[0] = 1, sm[0] = 0
  const double Ap = m > 0 ? pc * c + ps * s : pc;
  const double wy = double(w * q.Y[l][m]);
  S.yq += wy * Aq;
  S.yp += wy * Ap;
  if constexpr (l >= 1) {
    T dY;
    if constexpr (m == 0) {
      dY = T(kTab.e1[l][0]) * q.Y[l][1];
    } else if constexpr (m + 1 <= l) {
      dY = T(kTab.e1[l][m]) * q.Y[l][m + 1] - T(kTab.e2[l][m]) * q.Y[l][m - 1];
    } else {
      dY = -T(kTab.e2[l][m]) * q.Y[l][m - 1];
    }
    const double wd = double(w * dY);
    S.dq += wd * Aq;
    S.dp += wd * Ap;
    if constexpr (m >= 1) {
      const T mYs = -(T(kTab.f1[l][m]) * q.Y[l + 1][m + 1] + T(kTab.f2[l][m]) * q.Y[l + 1][m - 1]);
      const double wm = double(w * mYs);
      S.sq += wm * (qs * c - qc * s);
      S.sp += wm * (ps * c - pc * s);
    }
  }
}
// radial factors of one l: inward r^-(l+1), outward r^l; d/dr; and (1/r) x factor.  At
// the origin rinv = 0 and rm = 0, so every inward factor is 0 there (no inward part)
// without a branch.
template <int l>
__device__ __forceinline__ void mex_lsums_apply(const MexLSums& S, double rl, double rm, double rlm1,
                                                double rinv, double& Phi, double& ar, double& at, double& ap) {
  Phi -= S.yq * rm + S.yp * rl;
  ar += S.yq * (-(l + 1.0) * rm * rinv) + S.yp * (double(l) * rlm1);
  if constexpr (l >= 1) {
    const double oq = rm * rinv, op = rlm1;
    at += S.dq * oq + S.dp * op;
    ap += S.sq * oq + S.sp * op;
  }
}

// Per-particle synthesis.  Every wavefront takes a tile of kMexTile sorted particles on
// its own (lane k: rows 2k and 2k+1), so no LDS and no barrier: each column's moments
// come from lane scans in registers (inward: the prefix tree over the lanes; outward:
// the same tree over the reversed lanes), one l at a time.
constexpr int kMexForceWaves = 4;  // independent wavefronts (tiles) per workgroup
template <typename T, int LB>
__global__ __launch_bounds__(64 * kMexForceWaves, LB <= 10 ? 2 : 1) void mex_force_kernel(
    const MexArgs<LB> a) {
  constexpr int NC = mex_nc(LB);
  const int lane = threadIdx.x & 63;
  const int tile = blockIdx.x * kMexForceWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (tile >= a.ntiles) return;  // the whole wavefront
  MexLane<T, LB> q0, q1;
  const int64_t k0 = int64_t(tile) * kMexTile + 2 * lane;
  q0.load(a, k0);
  q1.load(a, k0 + 1);
  mex_legendre_row<T, LB, 1>(q0.Y, q0.p.ct, q0.p.st);
  mex_legendre_row<T, LB, 1>(q1.Y, q1.p.ct, q1.p.st);
  double rl0 = 1.0, rm0 = q0.p.rinv, rlm10 = 0.0;  // r^l, r^-(l+1), r^(l-1) (0 for l = 0)
  double rl1 = 1.0, rm1 = q1.p.rinv, rlm11 = 0.0;
  double Phi0 = 0.0, ar0 = 0.0, at0 = 0.0, ap0 = 0.0;
  double Phi1 = 0.0, ar1 = 0.0, at1 = 0.0, ap1 = 0.0;
  const double* offs = a.toff + size_t(tile) * 2 * NC;
  static_for<LB + 1>([&](auto lc) {
    constexpr int l = decltype(lc)::value;
    if (l > a.lmax) return;
    // one l at a time: nothing of a later l is computed early, so the live registers
    // (and with them the occupancy) stay bounded
    __builtin_amdgcn_sched_barrier(0);
    mex_legendre_row<T, LB, l + 1>(q0.Y, q0.p.ct, q0.p.st);  // row l+1 (for m Ybar / sin)
    mex_legendre_row<T, LB, l + 1>(q1.Y, q1.p.ct, q1.p.st);
    // summand weights m r^l (inward), m r^-(l+1) (outward); 0 for an invalid row
    const double wi0 = q0.valid ? q0.p.mass * rl0 : 0.0, wo0 = q0.valid ? q0.p.mass * rm0 : 0.0;
    const double wi1 = q1.valid ? q1.p.mass * rl1 : 0.0, wo1 = q1.valid ? q1.p.mass * rm1 : 0.0;
    const double* oin = offs + mex_coff(l);
    const double* oout = offs + NC + mex_coff(l);
    MexLSums S0, S1;
    static_for<l + 1>([&](auto mc) {
      constexpr int m = decltype(mc)::value;
      constexpr int sc = m == 0 ? 0 : 2 * m - 1;
      double qc0, qc1, pc0, pc1, qs0 = 0.0, qs1 = 0.0, ps0 = 0.0, ps1 = 0.0;
      {
        const double b0 = double(q0.Y[l][m] * q0.cm[m]), b1 = double(q1.Y[l][m] * q1.cm[m]);
        mex_pair_inward(wi0 * b0, wi1 * b1, oin[sc], qc0, qc1);
        mex_pair_outward(wo0 * b0, wo1 * b1, oout[sc], pc0, pc1);
      }
      if constexpr (m > 0) {
        const double b0 = double(q0.Y[l][m] * q0.sm[m]), b1 = double(q1.Y[l][m] * q1.sm[m]);
        mex_pair_inward(wi0 * b0, wi1 * b1, oin[sc + 1], qs0, qs1);
        mex_pair_outward(wo0 * b0, wo1 * b1, oout[sc + 1], ps0, ps1);
      }
      mex_lsums_add<T, LB, l, m>(q0, qc0, qs0, pc0, ps0, S0);
      mex_lsums_add<T, LB, l, m>(q1, qc1, qs1, pc1, ps1, S1);
    });
    mex_lsums_apply<l>(S0, rl0, rm0, rlm10, q0.p.rinv, Phi0, ar0, at0, ap0);
    mex_lsums_apply<l>(S1, rl1, rm1, rlm11, q1.p.rinv, Phi1, ar1, at1, ap1);
    rlm10 = rl0;
    rl0 *= q0.p.r;
    rm0 *= q0.p.rinv;
    rlm11 = rl1;
    rl1 *= q1.p.r;
    rm1 *= q1.p.rinv;
  });
  auto store = [&](const MexLane<T, LB>& q, double Phi, double ar, double at, double ap) {
    if (!q.valid) return;
    const uint32_t pidx = q.pidx;
    if (a.want_pot) a.pot[pidx] = Phi;
    if (a.want_acc) {
      const double st = double(q.p.st), ct = double(q.p.ct), cp = double(q.p.cp), sp = double(q.p.sp);
      a.ax[pidx] = st * cp * ar + ct * cp * at - sp * ap;
      a.ay[pidx] = st * sp * ar + ct * sp * at + cp * ap;
      a.az[pidx] = ct * ar - st * at;
    }
  };
  store(q0, Phi0, ar0, at0, ap0);
  store(q1, Phi1, ar1, at1, ap1);
}

// Per-particle synthesis with the summands staged in LDS (the FP64 mode: its basis in
// FP64 does not leave the registers for two particles per lane).  One thread per
// particle, two wavefronts per tile; per l and side, every column is scanned by one
// wavefront.
template <typename T, int LB>
__global__ __launch_bounds__(kMexTile, LB <= 10 ? 3 : 2) void mex_force_staged_kernel(const MexArgs<LB> a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double* S = reinterpret_cast<double*>(lds_raw);  // [2l+1][kMexTile], one side at a time
  constexpr int NC = mex_nc(LB);
  const int t = threadIdx.x, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);  // uniform: scalar addressing
  MexLane<T, LB> q;
  q.load(a, int64_t(blockIdx.x) * kMexTile + t);
  const MexParticle<T>& p = q.p;
  mex_legendre_row<T, LB, 1>(q.Y, p.ct, p.st);
  double rl = 1.0, rm = p.rinv;                      // r^l, r^-(l+1)
  double rlm1 = 0.0;                                 // r^(l-1)  (0 for l = 0)
  double Phi = 0.0, ar = 0.0, at = 0.0, ap = 0.0;
  const double* offs = a.toff + size_t(blockIdx.x) * 2 * NC;
  static_for<LB + 1>([&](auto lc) {
    constexpr int l = decltype(lc)::value;
    if (l > a.lmax) return;
    // one l at a time: nothing of a later l is computed early, so the live registers
    // (and with them the occupancy) stay bounded
    __builtin_amdgcn_sched_barrier(0);
    // Legendre row l+1 (for m Ybar / sin)
    mex_legendre_row<T, LB, l + 1>(q.Y, p.ct, p.st);
    constexpr int H = 2 * l + 1;
    // exclusive scans of every column inside the tile, one side at a time, one
    // wavefront per column: lane k takes two consecutive rows, then a lane tree gives
    // what the lanes before it hold.  Inward columns run forward (lane k: rows 2k, 2k+1);
    // outward columns backward (lane k: rows 126-2k, 127-2k, so the lanes before k hold
    // the later particles).  The tile's offset from the other tiles is added.  The
    // particle keeps its own inward values in registers while the outward side reuses
    // the LDS block.
    double qv[H];
    static_for<2>([&](auto sidec) {
      constexpr int side = decltype(sidec)::value;
      mex_summands_col<T, LB, l, side, kMexTile>(p, q.Y, q.cm, q.sm, rl, rm, q.valid, S + t);
      __syncthreads();
#pragma unroll 3
      for (int j = 0; j < (H + 1) / 2; ++j) {
        const int c = 2 * j + wave;
        if (c < H) {
          double* cp = S + c * kMexTile + (side == 0 ? 2 * lane : kMexTile - 2 - 2 * lane);
          const double2 v = *reinterpret_cast<const double2*>(cp);
          const double off = offs[side * NC + mex_coff(l) + c];
          // within the pair: the first row in scan order gets 0, the second the first
          const double first = side == 0 ? v.x : v.y, second = side == 0 ? v.y : v.x;
          const double base = off + wave_excl_prefix(first + second);
          const double r_first = base, r_second = base + first;
          *reinterpret_cast<double2*>(cp) =
              side == 0 ? make_double2(r_first, r_second) : make_double2(r_second, r_first);
        }
      }
      __syncthreads();
      if constexpr (side == 0) {
#pragma unroll
        for (int c = 0; c < H; ++c) qv[c] = S[c * kMexTile + t];
        __syncthreads();  // every lane has its inward values before the outward side
      }
    });
    // synthesis of this l from the particle's own q (registers) and p (LDS).
    // Radial factors of this l: inward q r^-(l+1), outward p r^l; d/dr; and (1/r) x
    // factor.  At the origin rinv = 0 and rm = 0, so every inward factor is 0 there
    // (no inward part) without a branch.
    {
      const double* row = S + t;
      const double g = 4.0 * kPi / (2.0 * l + 1.0);
      const double fq = rm, fp = rl;                       // potential
      const double dq = -(l + 1.0) * rm * p.rinv;          // d/dr r^-(l+1)
      const double dp = double(l) * rlm1;                  // d/dr r^l
      const double oq = rm * p.rinv, op = rlm1;            // (1/r) x radial factor
      static_for<l + 1>([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        constexpr int sc = m == 0 ? 0 : 2 * m - 1;
        const double w = (m == 0 ? 1.0 : 2.0) * g;
        const double qc = qv[sc], pc = row[sc * kMexTile];
        const double qs = m > 0 ? qv[sc + 1] : 0.0;
        const double ps = m > 0 ? row[(sc + 1) * kMexTile] : 0.0;
        const double c = double(q.cm[m]), s = double(q.sm[m]);
        const double Aq = qc * c + qs * s, Ap = pc * c + ps * s;  // cos-weighted parts
        const double e = Aq * fq + Ap * fp;
        const double dr = Aq * dq + Ap * dp;
        const double wy = w * double(q.Y[l][m]);
        Phi -= wy * e;
        ar += wy * dr;
        if constexpr (l >= 1) {
          const double eo = Aq * oq + Ap * op;
          T dY;
          if constexpr (m == 0) {
            dY = T(kTab.e1[l][0]) * q.Y[l][1];
          } else if constexpr (m + 1 <= l) {
            dY = T(kTab.e1[l][m]) * q.Y[l][m + 1] - T(kTab.e2[l][m]) * q.Y[l][m - 1];
          } else {
            dY = -T(kTab.e2[l][m]) * q.Y[l][m - 1];
          }
          at += w * double(dY) * eo;
          if constexpr (m >= 1) {
            const double f = (qs * c - qc * s) * oq + (ps * c - pc * s) * op;
            const T mYs = -(T(kTab.f1[l][m]) * q.Y[l + 1][m + 1] + T(kTab.f2[l][m]) * q.Y[l + 1][m - 1]);
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
  if (!q.valid) return;
  const uint32_t pidx = q.pidx;
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
  size_t off_key0, off_key1, off_idx0, off_idx1, off_sort, sort_bytes, off_tsum, off_toff, off_bsum,
      total;
  int stiles, ntiles, nblocks, lb;
};

MexLayout mex_layout(int64_t n, int lmax) {
  MexLayout L{};
  L.lb = lmax <= 2 ? 2 : lmax <= 6 ? 6 : lmax <= 10 ? 10 : 14;
  L.stiles = int((n + kSortTile - 1) / kSortTile);
  if (L.stiles < 1) L.stiles = 1;
  L.ntiles = int((n + kMexTile - 1) / kMexTile);
  if (L.ntiles < 1) L.ntiles = 1;
  L.nblocks = (L.ntiles + kMexBlockTiles - 1) / kMexBlockTiles;
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
  // radix sort: digit counts [256][tiles], digit totals [256]
  L.sort_bytes = size_t(256) * L.stiles * 4 + size_t(256) * 4;
  L.off_sort = take(L.sort_bytes);
  L.off_tsum = take(size_t(L.ntiles) * 2 * NC * 8);
  L.off_toff = take(size_t(L.ntiles) * 2 * NC * 8);
  L.off_bsum = take(size_t(L.nblocks) * 2 * NC * 8);
  L.total = o;
  return L;
}

template <typename T, int LB>
int launch_mex_lb(const MexArgs<LB>& a, int ntiles, hipStream_t st) {
  // largest LDS blocks: 2l+1 columns (one side) at l = LB, of kMexColStride (tile sums)
  // or kMexTile (FP64 force) doubles; at most 29 columns of 144 doubles (33.4 KiB):
  // within the default LDS limit.  The FP32-basis force kernel uses no LDS.
  const size_t lds_sums = size_t(kMexColStride) * (2 * LB + 1) * 8;
  if constexpr (sizeof(T) == 4)
    hipLaunchKernelGGL((mex_tile_sums_pair_kernel<T, LB>), dim3((ntiles + kMexPairWaves - 1) / kMexPairWaves),
                       dim3(64 * kMexPairWaves), mex_pair_lds_bytes(LB), st, a);
  else
    hipLaunchKernelGGL((mex_tile_sums_kernel<T, LB>), dim3(ntiles), dim3(kMexTile), lds_sums, st, a);
  int rc = hip_fail(hipGetLastError(), "mex_tile_sums_kernel launch");
  if (rc) return rc;
  hipLaunchKernelGGL((mex_block_sums_kernel<LB>), dim3(a.nblocks), dim3(256), 0, st, a);
  const int ncol = 2 * (a.lmax + 1) * (a.lmax + 1);
  hipLaunchKernelGGL((mex_block_scan_kernel<LB>), dim3((ncol + 3) / 4), dim3(256), 0, st, a);
  hipLaunchKernelGGL((mex_tile_offsets_kernel<LB>), dim3(a.nblocks), dim3(256), 0, st, a);
  rc = hip_fail(hipGetLastError(), "mex tile offset launch");
  if (rc) return rc;
  rc = hook_before(st);
  if (rc) return rc;
  if constexpr (sizeof(T) == 8) {
    const size_t lds = size_t(kMexTile) * (2 * LB + 1) * 8;
    hipLaunchKernelGGL((mex_force_staged_kernel<T, LB>), dim3(ntiles), dim3(kMexTile), lds, st, a);
  } else {
    hipLaunchKernelGGL((mex_force_kernel<T, LB>), dim3((ntiles + kMexForceWaves - 1) / kMexForceWaves),
                       dim3(64 * kMexForceWaves), 0, st, a);
  }
  rc = hip_fail(hipGetLastError(), "mex_force_kernel launch");
  return rc ? rc : hook_after(st);
}

template <typename T>
int launch_mex_t(int lb, const double* x, const double* y, const double* z, const double* m,
                 int64_t n, int lmax, const uint32_t* perm, double* tsum, double* toff, double* bsum,
                 int ntiles, int nblocks, int outputs, double* pot, double* ax, double* ay, double* az,
                 hipStream_t st) {
  auto fill = [&](auto& a) {
    a.x = x;
    a.y = y;
    a.z = z;
    a.m = m;
    a.n = n;
    a.perm = perm;
    a.tsum = tsum;
    a.toff = toff;
    a.bsum = bsum;
    a.nblocks = nblocks;
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
  uint32_t* counts = reinterpret_cast<uint32_t*>(base + L.off_sort);
  uint32_t* totals = counts + size_t(256) * L.stiles;
  double* tsum = reinterpret_cast<double*>(base + L.off_tsum);
  double* toff = reinterpret_cast<double*>(base + L.off_toff);
  double* bsum = reinterpret_cast<double*>(base + L.off_bsum);

  hipLaunchKernelGGL(mex_keys_kernel, dim3(int((n + 255) / 256)), dim3(256), 0, st, x, y, z, n, k0, i0);
  int rc = hip_fail(hipGetLastError(), "mex_keys_kernel launch");
  if (rc) return rc;
  for (int pass = 0; pass < kSortPasses; ++pass) {
    const int shift = 8 * pass;
    hipLaunchKernelGGL(radix_count_kernel, dim3(L.stiles), dim3(kSortThreads), 0, st, k0, n, shift, L.stiles,
                       counts);
    hipLaunchKernelGGL(radix_digit_scan_kernel, dim3(256), dim3(256), 0, st, counts, L.stiles, totals);
    hipLaunchKernelGGL(radix_scatter_kernel, dim3(L.stiles), dim3(kSortThreads), 0, st, k0, i0, k1, i1, n,
                       shift, L.stiles, counts, totals);
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
    return launch_mex_t<double>(L.lb, x, y, z, m, n, lmax, i0, tsum, toff, bsum, L.ntiles, L.nblocks,
                                outputs, pot, ax, ay, az, st);
  return launch_mex_t<float>(L.lb, x, y, z, m, n, lmax, i0, tsum, toff, bsum, L.ntiles, L.nblocks,
                             outputs, pot, ax, ay, az, st);
}

}  // namespace etics
