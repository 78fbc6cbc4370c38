// etics_coeff_wg.hpp -- the workgroup code of the SCF coefficient kernels, shared by the
// coefficient sums (etics_coeff.hip) and their time derivatives (etics_coeff_dot.hip).
//
// The first part of an SCF force calculation (paper Section 3.3) is the sum over all
// particles k of m_k PhiT_nl(r_k) Ybar_lm(theta_k) (cos, sin)(m phi_k) for every
// (n, l, m) (eq. scf-phi with the Hernquist-Ostriker basis of Section 2.5).
//
// scf_coeff_kernel: each workgroup (4 wavefronts) walks a contiguous run of tiles of
//   `tp` particles.
//   Phase 1 evaluates each particle's basis once, one particle per lane.  The basis
//   is split into independent jobs -- the Gegenbauer row of one l (radial job) and
//   the Legendre column of one m times (cos, sin)(m phi) and the radial prefactor
//   (angular job) -- and a compile-time plan gives each job to one wavefront of a
//   particle group: the four wavefronts share the work of the same 64 particles, or
//   (small cutoffs, NW = 2 or 1) form 2 or 4 groups of 64 particles.  The values go to
//   LDS at compile-time offsets.
//   Phase 2 is an outer-product accumulation over the tile: every lane owns an
//   nb x bs register block of coefficients (radial orders x angular slots of one l)
//   and accumulates the products of the LDS-staged radial and angular values.  The
//   lanes are grouped in "streams": each stream owns one copy of every block and
//   takes every streams-th particle of the tile.  FP32 partial sums are folded into
//   FP64 (or compensated double-float) accumulators every few tiles.
//   At the end the streams are merged in a fixed order through LDS and the
//   workgroup writes one partial coefficient vector.
// The time derivatives of the sums along the particles' velocities (for the jerk) run
//   the same kernels with DUAL set: phase 1 evaluates the basis on values that carry
//   their time derivative and writes each particle as two rows, (dG/dt, Z) and
//   (G, dZ/dt), so phase 2's outer products sum d/dt (G Z) = (dG/dt) Z + G dZ/dt.
// scf_reduce_kernel sums the partial vectors over workgroups in a fixed order and
//   applies (2 - delta_m0) Atilde_nl and the basis constants, so the result does not
//   depend on how the hardware schedules workgroups.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>

#include "etics_device.hpp"
#include "etics_internal.hpp"

namespace etics {

struct CoeffArgs {
  const double *x, *y, *z, *m;
  const double *vx, *vy, *vz;  // velocities (time-derivative sums only)
  int64_t n;
  void* partials;  // [grid][2K] FP64 (or double-float pairs)
  int K, nmax, lmax, tp, nblocks, streams, flush_tiles, ntiles, nchunks;
};

// ------------------------------------------------------------ phase-1 job plan
// The basis jobs of a cutoff bucket are split between the NW wavefronts that share a
// group of 64 particles (NW = 4: the whole workgroup; NW = 2 or 1: two or four groups,
// so a tile holds 128 or 256 particles).  Angular job m (the Legendre column of m times
// (cos, sin)(m phi)) costs ~6 operations per l in [m, lb]; before it, a wavefront walks
// the diagonal from m = 0 up to the largest column it owns (~6 operations per step), so
// each wavefront gets a contiguous range of columns and the low columns go together.
// Radial job l (a Gegenbauer row) costs ~2 operations per padded order; a wavefront
// with radial jobs only needs xi alone, not the angles.  The plan is the contiguous
// split (searched over all cut points) with the smallest max + total/4 load, radial
// jobs added greedily to the least loaded wavefront.
template <int LB, int NRP, int NW>
struct JobPlan {
  int ownerZ[LB + 1];
  int ownerG[LB + 1];
  int maxm[NW];
};

template <int LB, int NRP, int NW>
constexpr JobPlan<LB, NRP, NW> make_job_plan() {
  constexpr int kDiag = 6, kSphSave = 25;
  constexpr int kRad = 2 * NRP + NRP / 4 + 2;
  auto zcost = [](int m) { return 6 * (LB - m + 1) + 8; };
  JobPlan<LB, NRP, NW> best{};
  long best_key = -1;
  // k = number of wavefronts with angular columns; cut[i] = first column of range i+1
  for (int k = 1; k <= NW && k <= LB + 1; ++k) {
    int cut[NW + 1] = {};
    for (int i = 0; i < k - 1; ++i) cut[i] = i + 1;  // first combination of k-1 cuts
    while (true) {
      JobPlan<LB, NRP, NW> p{};
      int load[NW] = {};
      for (int w = 0; w < NW; ++w) p.maxm[w] = -1;
      int lo = 0;
      for (int r = 0; r < k; ++r) {
        const int hi = (r < k - 1 ? cut[r] : LB + 1) - 1;
        for (int m = lo; m <= hi; ++m) {
          p.ownerZ[m] = r;
          load[r] += zcost(m);
        }
        load[r] += kDiag * hi;
        p.maxm[r] = hi;
        lo = hi + 1;
      }
      for (int w = k; w < NW; ++w) load[w] = -kSphSave;
      for (int l = 0; l <= LB; ++l) {
        int w = 0;
        for (int q = 1; q < NW; ++q)
          if (load[q] < load[w]) w = q;
        p.ownerG[l] = w;
        load[w] += kRad;
      }
      long mx = load[0], tot = 0;
      for (int w = 0; w < NW; ++w) {
        tot += load[w];
        if (load[w] > mx) mx = load[w];
      }
      const long key = 4 * mx + tot;
      if (best_key < 0 || key < best_key) {
        best_key = key;
        best = p;
      }
      // next combination of k-1 cut points from 1..LB (increasing)
      int i = k - 2;
      while (i >= 0 && cut[i] == LB - (k - 2 - i)) --i;
      if (i < 0) break;
      ++cut[i];
      for (int j = i + 1; j < k - 1; ++j) cut[j] = cut[j - 1] + 1;
    }
  }
  return best;
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

// two adjacent LDS values in one store (the address is 2-element aligned)
__device__ __forceinline__ void store_pair(float* p, float a, float b) {
  *reinterpret_cast<float2*>(p) = make_float2(a, b);
}
__device__ __forceinline__ void store_pair(double* p, double a, double b) {
  *reinterpret_cast<double2*>(p) = make_double2(a, b);
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

// plain vector types for reads through LDS (address space 3) pointers
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) f32x4 LdsF32x4;
typedef __attribute__((address_space(3))) f64x2 LdsF64x2;

// One workgroup's share of the coefficient sums: the LDS tile, the register block
// of each lane, and the three steps (basis -> LDS, accumulate, merge and write).
template <typename T, int LB, int NB, int BS, int MODE, int NW, int BASIS>
struct CoeffWG {
  static_assert(NW == 1 || NW == 2 || NW == 4, "wavefronts per particle group");
  static constexpr int NRP = nrp_for_nb(NB);
  static constexpr int SPG = g_stride(LB, NRP);
  static constexpr int SPZ = z_stride(LB, BS);
  using PT = typename PartialT<(sizeof(T) == 4 && MODE == 1) ? 1 : 0>::type;

  T* G;  // [tp][SPG]  radial values, rows of NRP per l
  T* Z;  // [tp][SPZ]  angular values x mass x radial prefactor
  int tid, lane, wave, rank, pidx, maxm_w, lmax, nmax, tp, streams, nblocks, nchunks;
  int my_stream, my_block, bl, n0, s0;
  int goff, zoff0;  // this lane's block in a particle's radial / angular row
  bool active;
  T acc[NB][BS];
  Wide<T, MODE> wide[NB][BS];

  __device__ __forceinline__ void init(unsigned char* lds, int tp_, int lmax_, int nmax_,
                                       int nblocks_, int streams_, int nchunks_) {
    constexpr JobPlan<LB, NRP, NW> kJP = make_job_plan<LB, NRP, NW>();
    G = reinterpret_cast<T*>(lds);
    Z = G + tp_ * SPG;
    tid = threadIdx.x;
    lane = tid & 63;
    wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    rank = wave % NW;               // job share within the particle group
    pidx = (wave / NW) * 64 + lane;  // this lane's particle in the tile (phase 1)
    tp = tp_;
    lmax = lmax_;
    nmax = nmax_;
    nblocks = nblocks_;
    streams = streams_;
    nchunks = nchunks_;
    // largest angular column owned by this wavefront (the diagonal walk stops there)
    maxm_w = -1;
    static_for<NW>([&](auto wc) {
      if (rank == decltype(wc)::value) maxm_w = kJP.maxm[decltype(wc)::value];
    });
    my_stream = tid / nblocks;
    my_block = tid - my_stream * nblocks;
    active = my_stream < streams;
    decode_block<NB, BS>(my_block, lmax, nchunks, bl, n0, s0);
    goff = bl * NRP + n0;
    zoff0 = zoff_rt<BS>(bl) + s0;
    clear_acc();
    clear_wide();
  }

  __device__ __forceinline__ void clear_acc() {
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int j = 0; j < BS; ++j) acc[i][j] = T(0);
  }
  __device__ __forceinline__ void clear_wide() {
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int j = 0; j < BS; ++j) wide[i][j] = Wide<T, MODE>{};
  }
  // angular padding slots are never written by phase 1; keep them finite
  __device__ __forceinline__ void zero_slots() {
    for (int i = tid; i < tp * SPZ; i += kCoeffThreads) Z[i] = T(0);
  }
  // fold the FP32 run into the wide accumulators
  __device__ __forceinline__ void fold() {
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int j = 0; j < BS; ++j) {
        wide[i][j].add(acc[i][j]);
        acc[i][j] = T(0);
      }
  }

  // phase 1: basis of the particle of this lane (zero mass for an empty lane)
  __device__ __forceinline__ void phase1(double xd, double yd, double zd, double md) {
    if (pidx >= tp) return;
    T* Gp = G + pidx * SPG;
    T* Zp = Z + pidx * SPZ;
    T xi;
    if (maxm_w >= 0) {
      const Sph<T> s = sph<T, BASIS>(xd, yd, zd);
      xi = s.xi;
      angular_jobs(s, md, Zp, Zp);
    } else {  // radial jobs only: xi alone
      xi = xi_only<T>(T(xd), T(yd), T(zd));
    }
    radial_jobs(xi, Gp, Gp);
  }

  // phase 1 of the time-derivative sums: d/dt sum_k m_k G_k Z_k = sum_k (dG_k/dt) Z_k +
  // G_k (dZ_k/dt), so the particle of this lane fills two rows of the tile, which
  // phase 2 then treats as two particles: row 2p holds (dG/dt, Z), row 2p+1 (G, dZ/dt).
  // The basis is evaluated on values that carry their time derivative along the
  // particle's velocity; the tile holds tp/2 particles.
  __device__ __forceinline__ void phase1_dual(double xd, double yd, double zd, double vxd, double vyd,
                                              double vzd, double md) {
    if (2 * pidx + 1 >= tp) return;
    T* Gder = G + (2 * pidx) * SPG;
    T* Gval = Gder + SPG;
    T* Zval = Z + (2 * pidx) * SPZ;
    T* Zder = Zval + SPZ;
    Dual<T> xi;
    if (maxm_w >= 0) {
      const Sph<Dual<T>> s = sph_dual<T, BASIS>(xd, yd, zd, vxd, vyd, vzd);
      xi = s.xi;
      angular_jobs(s, md, Zval, Zder);
    } else {
      xi = xi_only<Dual<T>>(Dual<T>(T(xd), T(vxd)), Dual<T>(T(yd), T(vyd)), Dual<T>(T(zd), T(vzd)));
    }
    radial_jobs(xi, Gval, Gder);
  }

  // xi of the radial basis from the position alone (wavefronts with radial jobs only)
  template <typename V>
  static __device__ __forceinline__ V xi_only(V x, V y, V z) {
    const V r2 = x * x + y * y + z * z;
    if constexpr (BASIS == kBasisCB) {  // (r^2 - 1) / (r^2 + 1)
      return (r2 - V(1)) * rcp_(r2 + V(1));
    } else {  // (r - 1) / (r + 1)
      const V r = sqrt_(r2);
      const V u = rcp_(V(1) + r);
      return r * u - u;
    }
  }

  // LDS stores of basis values: a plain value goes to its row; a value that carries a
  // time derivative goes to the value row, its derivative to the derivative row
  static __device__ __forceinline__ void put1(T* val, T*, int off, T v) { val[off] = v; }
  static __device__ __forceinline__ void put1(T* val, T* der, int off, Dual<T> v) {
    val[off] = v.v;
    der[off] = v.d;
  }
  static __device__ __forceinline__ void put2(T* val, T*, int off, T a, T b) { store_pair(val + off, a, b); }
  static __device__ __forceinline__ void put2(T* val, T* der, int off, Dual<T> a, Dual<T> b) {
    store_pair(val + off, a.v, b.v);
    store_pair(der + off, a.d, b.d);
  }
  static __device__ __forceinline__ void put4row(T* row, T a, T b, T c, T d) {
    if constexpr (sizeof(T) == 4) {
      *reinterpret_cast<float4*>(row) = make_float4(a, b, c, d);
    } else {
      *reinterpret_cast<double2*>(row) = make_double2(a, b);
      *reinterpret_cast<double2*>(row + 2) = make_double2(c, d);
    }
  }
  static __device__ __forceinline__ void put4(T* val, T*, int off, const T (&v)[4]) {
    put4row(val + off, v[0], v[1], v[2], v[3]);
  }
  static __device__ __forceinline__ void put4(T* val, T* der, int off, const Dual<T> (&v)[4]) {
    put4row(val + off, v[0].v, v[1].v, v[2].v, v[3].v);
    put4row(der + off, v[0].d, v[1].d, v[2].d, v[3].d);
  }

  // angular jobs: column m of mass u (tu)^l Ybar_lm (cos, sin)(m phi), l = m..lmax.  The
  // diagonal value mass u (tu)^m Ybar_mm and (cos, sin)(m phi) are walked up to the
  // largest column this wavefront owns.  V is T, or Dual<T> for the time derivatives.
  template <typename V>
  __device__ __forceinline__ void angular_jobs(const Sph<V>& s, double md, T* Zval, T* Zder) {
    constexpr JobPlan<LB, NRP, NW> kJP = make_job_plan<LB, NRP, NW>();
    const V tu = s.t * s.u, ctu = s.ct * tu, tu2 = tu * tu, stu = s.st * tu;
    V Pd = T(md) * s.u * T(kTab.c1[0][0]);
    V cmc = V(1), smc = V(0);
    static_for<LB + 1>([&](auto mc) {
      constexpr int m = decltype(mc)::value;
      if constexpr (m > 0) {
        if (m <= maxm_w) {
          Pd = (T(kTab.c1[m][m]) * stu) * Pd;
          const V c2 = cmc * s.cp - smc * s.sp;
          smc = smc * s.cp + cmc * s.sp;
          cmc = c2;
        }
      }
      if (rank == kJP.ownerZ[m] && m <= lmax) {
        V P2 = V(0), P1 = Pd;  // P2 is first read at l = m + 2
        auto put = [&](auto lc2, V P) {
          constexpr int l = decltype(lc2)::value;
          if constexpr (m == 0) {
            put1(Zval, Zder, zoff(l, BS) + 2 * l, P);
          } else {  // (cos, sin) pair at an even slot of an 8-byte aligned row
            put2(Zval, Zder, zoff(l, BS) + 2 * m - 2, P * cmc, P * smc);
          }
        };
        // the whole column up to the bucket's LB (rows past lmax are never read), so
        // the recurrence runs without a branch per row
        put(std::integral_constant<int, m>{}, P1);
        static_for<LB - m>([&](auto kc) {
          constexpr int l = m + 1 + decltype(kc)::value;
          V P = (T(kTab.c1[l][m]) * ctu) * P1;
          if constexpr (l > m + 1) P -= (T(kTab.c2[l][m]) * tu2) * P2;
          P2 = P1;
          P1 = P;
          put(std::integral_constant<int, l>{}, P);
        });
      }
    });
  }

  // radial jobs: monic Gegenbauer Chat_n^(a_l)(xi), n = 0..NRP-1 (a_l of the basis).
  // Entries past nmax only feed coefficients that are never written out; they stay
  // finite.
  template <typename V>
  __device__ __forceinline__ void radial_jobs(V xi, T* Gval, T* Gder) {
    constexpr JobPlan<LB, NRP, NW> kJP = make_job_plan<LB, NRP, NW>();
    static_for<LB + 1>([&](auto lc) {
      constexpr int l = decltype(lc)::value;
      if (rank == kJP.ownerG[l] && l <= lmax) {
        V p2 = V(1), p1 = V(0);
        static_for<NRP / 4>([&](auto qc) {
          constexpr int nb4 = 4 * decltype(qc)::value;
          V v[4];
          static_for<4>([&](auto jc) {
            constexpr int nn = nb4 + decltype(jc)::value;
            constexpr double qv = BASIS == kBasisCB ? kTab.qcb[l][nn] : kTab.q[l][nn];
            const V c = xi * p1 - T(qv) * p2;
            p2 = p1;
            p1 = c;
            v[decltype(jc)::value] = c;
          });
          put4(Gval, Gder, l * NRP + nb4, v);
        });
      }
    });
  }

  // phase 2: outer-product accumulation over the tile.  LDS positions are 32-bit
  // element offsets from the tile base.
  __device__ __forceinline__ void phase2() {
    if (!active) return;
    using LT = __attribute__((address_space(3))) const T;
    LT* gs = (LT*)(G);
    LT* zs = (LT*)(Z);
    constexpr int NG = (NB + 3) / 4 * 4;
    T gv[2][NG], zv[2][BS];
    auto fetch = [&](int go, int zo, int buf) {
      LT* g = gs + go;
      LT* zz = zs + zo;
      if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int q = 0; q < NG / 4; ++q) {
          const f32x4 f = reinterpret_cast<const LdsF32x4*>(g)[q];
          gv[buf][4 * q] = f.x;
          gv[buf][4 * q + 1] = f.y;
          gv[buf][4 * q + 2] = f.z;
          gv[buf][4 * q + 3] = f.w;
        }
      } else {
#pragma unroll
        for (int q = 0; q < (NB + 1) / 2; ++q) {
          const f64x2 f = reinterpret_cast<const LdsF64x2*>(g)[q];
          gv[buf][2 * q] = f.x;
          gv[buf][2 * q + 1] = f.y;
        }
      }
      static_assert(BS % 4 == 0, "angular blocks are read in aligned 4-slot groups");
#pragma unroll
      for (int j = 0; j < BS; j += 4) {
        if constexpr (sizeof(T) == 4) {
          const f32x4 f = reinterpret_cast<const LdsF32x4*>(zz)[j / 4];
          zv[buf][j] = f.x;
          zv[buf][j + 1] = f.y;
          zv[buf][j + 2] = f.z;
          zv[buf][j + 3] = f.w;
        } else {
          const f64x2 f0 = reinterpret_cast<const LdsF64x2*>(zz)[j / 2];
          const f64x2 f1 = reinterpret_cast<const LdsF64x2*>(zz)[j / 2 + 1];
          zv[buf][j] = f0.x;
          zv[buf][j + 1] = f0.y;
          zv[buf][j + 2] = f1.x;
          zv[buf][j + 3] = f1.y;
        }
      }
    };
    auto madd = [&](int buf) {
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < BS; ++j) acc[i][j] = fma_(gv[buf][i], zv[buf][j], acc[i][j]);
    };
    // two particles per trip, each one's LDS reads issued before the other's FMAs.  The
    // look-ahead read past the tile is clamped to its last particle (read, never used),
    // so the reads need no branch and the two buffers keep their registers.
    const int gstep = streams * SPG, zstep = streams * SPZ;
    const int glast = goff + (tp - 1) * SPG, zlast = zoff0 + (tp - 1) * SPZ;
    int p = my_stream;
    int go = goff + p * SPG, zo = zoff0 + p * SPZ;
    fetch(go < glast ? go : glast, zo < zlast ? zo : zlast, 0);
    for (; p + streams < tp; p += 2 * streams) {
      fetch(go + gstep, zo + zstep, 1);
      madd(0);
      go += 2 * gstep;
      zo += 2 * zstep;
      fetch(go < glast ? go : glast, zo < zlast ? zo : zlast, 0);
      madd(1);
    }
    if (p < tp) madd(0);
  }

  // merge the streams in a fixed order through LDS (overwrites the tile) and write the
  // partial sums in coefficient layout: part[0..K) cos, part[K..2K) sin
  __device__ __forceinline__ void merge_write(unsigned char* lds, PT* part, int K) {
    PT* out = reinterpret_cast<PT*>(lds);
    for (int s = 0; s < streams; ++s) {
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
    const int L2 = (lmax + 1) * (lmax + 2) / 2;
    const int nent = nblocks * NB * BS;
    for (int e = tid; e < nent; e += kCoeffThreads) {
      const int j = e % BS;
      const int i = (e / BS) % NB;
      int l, nb0, sb0;
      decode_block<NB, BS>(e / (NB * BS), lmax, nchunks, l, nb0, sb0);
      const int nn = nb0 + i;
      const int slot = sb0 + j;
      if (nn > nmax || slot > 2 * l) continue;
      const int m = slot == 2 * l ? 0 : slot / 2 + 1;
      const bool is_sin = slot < 2 * l && (slot & 1) == 1;
      const int k = nn * L2 + l * (l + 1) / 2 + m;
      part[(is_sin ? K : 0) + k] = out[e];
    }
  }
};

// ------------------------------------------------------------ phase 2 on the matrix cores
// In the FP32 modes phase 2 can run on the matrix cores instead of the VALU.  The sums of
// one l form an (orders x slots) matrix of outer products summed over the particles; it
// is cut into 4 x 4 blocks (4 orders x 4 angular slots), and v_mfma_f32_4x4x1f32
// accumulates 16 such blocks at once, one particle per instruction: lanes 4b .. 4b+3
// hold the four orders (A operand, from the radial row) and the four slots (B operand,
// from the angular row) of block b, and accumulator register v of lane 4b + j holds
// (order v, slot j) of block b.  4 x 4 blocks waste few entries on the ragged edges of
// the (orders x (2l+1) slots) matrices (about a quarter at (10, 10)); larger tiles would
// waste most of each instruction on the small l.  The blocks of the cutoff, slot blocks
// fastest, are dealt 16 to an instruction and the instructions to the four wavefronts
// round-robin, so the blocks of one instruction mostly share their radial values (one
// LDS broadcast) and read consecutive angular slots.  The VALU is then left to phase 1
// of the other wavefronts of the CU.
template <int LB, int NRP>
constexpr int mfma_block_count() {
  int c = 0;
  for (int l = 0; l <= LB; ++l) c += (NRP / 4) * (slot_pad(l, 4) / 4);
  return c;
}

// block q of the cutoff (lmax, nmax): its l, first order and first slot; false past the
// last block
__device__ __forceinline__ bool mfma_block(int q, int lmax, int nmax, int& l, int& n0, int& s0) {
  const int nt = nmax / 4 + 1;  // order blocks holding an order <= nmax
  for (int k = 0; k <= lmax; ++k) {
    const int sb = slot_pad(k, 4) / 4;
    if (q < nt * sb) {
      l = k;
      n0 = 4 * (q / sb);
      s0 = 4 * (q % sb);
      return true;
    }
    q -= nt * sb;
  }
  l = n0 = s0 = 0;
  return false;
}

template <int LB, int NB, int MODE, int NW, int BASIS>
struct CoeffWGMM : CoeffWG<float, LB, NB, 4, MODE, NW, BASIS> {
  using Base = CoeffWG<float, LB, NB, 4, MODE, NW, BASIS>;
  using PT = typename Base::PT;
  static constexpr int NRP = Base::NRP, SPG = Base::SPG, SPZ = Base::SPZ;
  static constexpr int NI = (mfma_block_count<LB, NRP>() + 15) / 16;  // instructions per particle
  static constexpr int JPW = (NI + 3) / 4;                            // ... per wavefront
  // two accumulator sets (even and odd particles), so consecutive instructions on one
  // block do not wait for each other
  f32x4 macc[2][JPW];
  Wide<float, MODE> mwide[JPW][4];
  int aoff[JPW], boff[JPW];  // this lane's A / B element within a particle's rows

  __device__ __forceinline__ void init(unsigned char* lds, int tp_, int lmax_, int nmax_,
                                       int nblocks_, int streams_, int nchunks_) {
    Base::init(lds, tp_, lmax_, nmax_, nblocks_, streams_, nchunks_);
    const int i = this->lane & 3;
#pragma unroll
    for (int c = 0; c < JPW; ++c) {
      int l, n0, s0;
      // unused blocks read the first values of a row: in bounds, never written out
      if (!mfma_block(16 * (this->wave + 4 * c) + (this->lane >> 2), this->lmax, this->nmax, l, n0, s0))
        l = n0 = s0 = 0;
      aoff[c] = l * NRP + n0 + i;
      boff[c] = zoff_rt<4>(l) + s0 + i;
    }
    clear_mm();
    clear_wide();
  }
  __device__ __forceinline__ void clear_mm() {
#pragma unroll
    for (int c = 0; c < JPW; ++c) macc[0][c] = macc[1][c] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  __device__ __forceinline__ void clear_wide() {
#pragma unroll
    for (int c = 0; c < JPW; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) mwide[c][v] = Wide<float, MODE>{};
  }
  __device__ __forceinline__ void zero_slots() { Base::zero_slots(); }
  __device__ __forceinline__ void fold() {
#pragma unroll
    for (int c = 0; c < JPW; ++c) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        mwide[c][v].add(macc[0][c][v]);
        mwide[c][v].add(macc[1][c][v]);
      }
      macc[0][c] = macc[1][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  }
  // one particle per instruction, two per trip: the operands of the next particle are
  // read before the instructions of the current one (the look-ahead past the tile is
  // clamped to its last particle: read, never used), so the loop has no branch
  __device__ __forceinline__ void phase2() {
    using LT = __attribute__((address_space(3))) const float;
    LT* gs = (LT*)(this->G);
    LT* zs = (LT*)(this->Z);
    float a0[JPW], b0[JPW], a1[JPW], b1[JPW];
    auto load = [&](int p, float (&a)[JPW], float (&b)[JPW]) {
      const int gb = p * SPG, zb = p * SPZ;
#pragma unroll
      for (int c = 0; c < JPW; ++c) {
        a[c] = gs[gb + aoff[c]];
        b[c] = zs[zb + boff[c]];
      }
    };
    auto mma = [&](int set, const float (&a)[JPW], const float (&b)[JPW]) {
#pragma unroll
      for (int c = 0; c < JPW; ++c)
        macc[set][c] = __builtin_amdgcn_mfma_f32_4x4x1f32(a[c], b[c], macc[set][c], 0, 0, 0);
    };
    const int last = this->tp - 1;
    int p = 0;
    load(0, a0, b0);
    for (; p < last; p += 2) {
      load(p + 1, a1, b1);
      mma(0, a0, b0);
      load(p + 2 < last ? p + 2 : last, a0, b0);
      mma(1, a1, b1);
    }
    if (p == last) mma(0, a0, b0);
  }
  // every (n, l, slot) entry belongs to one lane of one wavefront: written straight to
  // the partial vector (part[0..K) cos, part[K..2K) sin)
  __device__ __forceinline__ void merge_write(unsigned char*, PT* part, int K) {
    const int L2 = (this->lmax + 1) * (this->lmax + 2) / 2;
    const int j = this->lane & 3;
#pragma unroll
    for (int c = 0; c < JPW; ++c) {
      int l, n0, s0;
      if (!mfma_block(16 * (this->wave + 4 * c) + (this->lane >> 2), this->lmax, this->nmax, l, n0, s0))
        continue;
      const int slot = s0 + j;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int nn = n0 + v;
        if (nn > this->nmax || slot > 2 * l) continue;
        const int m = slot == 2 * l ? 0 : slot / 2 + 1;
        const bool is_sin = slot < 2 * l && (slot & 1) == 1;
        part[(is_sin ? K : 0) + nn * L2 + l * (l + 1) / 2 + m] = wide_value(mwide[c][v]);
      }
    }
  }
};

template <bool MM, typename T, int LB, int NB, int BS, int MODE, int NW, int BASIS>
struct CoeffWGSel {
  using type = CoeffWG<T, LB, NB, BS, MODE, NW, BASIS>;
};
template <int LB, int NB, int BS, int MODE, int NW, int BASIS>
struct CoeffWGSel<true, float, LB, NB, BS, MODE, NW, BASIS> {
  using type = CoeffWGMM<LB, NB, MODE, NW, BASIS>;
};

// DUAL: the time derivatives of the sums along the particles' velocities; every
// particle then fills two rows of the tile, so a tile holds tp/2 particles.
template <typename T, int LB, int NB, int BS, int MODE, int NW, int BASIS, bool DUAL, bool MM>
__global__ __launch_bounds__(kCoeffThreads, sizeof(T) == 4 ? 2 : 1) void scf_coeff_kernel(
    const CoeffArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  using W = typename CoeffWGSel<MM, T, LB, NB, BS, MODE, NW, BASIS>::type;
  W w;
  w.init(lds_raw, a.tp, a.lmax, a.nmax, a.nblocks, a.streams, a.nchunks);
  w.zero_slots();
  __syncthreads();
  const int tpr = DUAL ? a.tp / 2 : a.tp;  // particles per tile

  // each workgroup takes a contiguous run of tiles, so the cache lines shared by two
  // neighbouring tiles are fetched once, into one L2
  const int t0 = int(int64_t(blockIdx.x) * a.ntiles / gridDim.x);
  const int t1 = int(int64_t(blockIdx.x + 1) * a.ntiles / gridDim.x);
  // particle data of the first tile (later tiles are prefetched during phase 2)
  double xd = 0.0, yd = 0.0, zd = 0.0, md = 0.0, vxd = 0.0, vyd = 0.0, vzd = 0.0;
  auto load_particle = [&](int tile) {
    const int64_t pi = int64_t(tile) * tpr + w.pidx;
    const bool valid = tile < t1 && w.pidx < tpr && pi < a.n;
    xd = valid ? a.x[pi] : 0.0;
    yd = valid ? a.y[pi] : 0.0;
    zd = valid ? a.z[pi] : 0.0;
    md = valid ? a.m[pi] : 0.0;
    if constexpr (DUAL) {
      vxd = valid ? a.vx[pi] : 0.0;
      vyd = valid ? a.vy[pi] : 0.0;
      vzd = valid ? a.vz[pi] : 0.0;
    }
  };
  load_particle(t0);

  int tcount = 0;
  for (int tile = t0; tile < t1; ++tile) {
    if constexpr (DUAL)
      w.phase1_dual(xd, yd, zd, vxd, vyd, vzd, md);
    else
      w.phase1(xd, yd, zd, md);
    __syncthreads();
    load_particle(tile + 1);  // next tile's particles load while phase 2 runs
    w.phase2();
    if (++tcount == a.flush_tiles) {
      tcount = 0;
      w.fold();
    }
    __syncthreads();
  }
  w.fold();
  using PT = typename W::PT;
  w.merge_write(lds_raw, reinterpret_cast<PT*>(a.partials) + size_t(blockIdx.x) * 2 * a.K, a.K);
}

// Batched systems: the work is cut into units of at most `unit` particles of one system
// (unit u of system s covers its particles from (u - ustart[s]) * unit on); each unit's
// sums go to their own partial slot, so the per-system reduction below has a fixed order
// whatever the schedule.
struct BatchedCoeffArgs {
  const double *x, *y, *z, *m;
  const double *vx, *vy, *vz;  // velocities (time-derivative sums only)
  const int64_t* offsets;
  const int* ustart;  // [nsys+1] first unit of each system; ustart[nsys] = number of units
  const int* usys;    // [units] system of each unit
  int64_t ntotal;
  void* partials;     // [units][2K]
  int nsys, K, nmax, lmax, tp, nblocks, streams, nchunks, flush_tiles, unit;
};

template <typename T, int LB, int NB, int BS, int MODE, int NW, bool DUAL, bool MM>
__global__ __launch_bounds__(kCoeffThreads, sizeof(T) == 4 ? 2 : 1) void scf_coeff_batched_kernel(
    const BatchedCoeffArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  using W = typename CoeffWGSel<MM, T, LB, NB, BS, MODE, NW, kBasisHO>::type;
  W w;
  w.init(lds_raw, a.tp, a.lmax, a.nmax, a.nblocks, a.streams, a.nchunks);
  const int tpr = DUAL ? a.tp / 2 : a.tp;  // particles per tile
  const int nunits = a.ustart[a.nsys];
  // particles [ub, ue) of unit u
  auto range = [&](int u, int64_t& ub, int64_t& ue) {
    const int s = a.usys[u];
    int64_t b = a.offsets[s], e = a.offsets[s + 1];
    b = b < 0 ? 0 : (b > a.ntotal ? a.ntotal : b);
    e = e < b ? b : (e > a.ntotal ? a.ntotal : e);
    ub = b + int64_t(u - a.ustart[s]) * a.unit;
    ue = ub + a.unit < e ? ub + a.unit : e;
  };
  // particle data of this lane for a tile; each tile's data is loaded while the previous
  // tile's outer products run (the first tile of the workgroup's next unit during the
  // last tile of the current one)
  double xd = 0.0, yd = 0.0, zd = 0.0, md = 0.0, vxd = 0.0, vyd = 0.0, vzd = 0.0;
  auto load_particle = [&](int64_t ub, int64_t ue, int tile) {
    const int64_t pi = ub + int64_t(tile) * tpr + w.pidx;
    const bool valid = w.pidx < tpr && pi < ue;
    xd = valid ? a.x[pi] : 0.0;
    yd = valid ? a.y[pi] : 0.0;
    zd = valid ? a.z[pi] : 0.0;
    md = valid ? a.m[pi] : 0.0;
    if constexpr (DUAL) {
      vxd = valid ? a.vx[pi] : 0.0;
      vyd = valid ? a.vy[pi] : 0.0;
      vzd = valid ? a.vz[pi] : 0.0;
    }
  };
  int64_t ub = 0, ue = 0;
  if (int(blockIdx.x) < nunits) {
    range(blockIdx.x, ub, ue);
    load_particle(ub, ue, 0);
  }
  for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
    const int ntiles = int((ue - ub + tpr - 1) / tpr);
    const int un = u + gridDim.x;  // this workgroup's next unit
    int64_t nb = 0, ne = 0;
    if (un < nunits) range(un, nb, ne);
    w.zero_slots();
    w.clear_wide();
    __syncthreads();
    int tcount = 0;
    for (int tile = 0; tile < ntiles; ++tile) {
      if constexpr (DUAL)
        w.phase1_dual(xd, yd, zd, vxd, vyd, vzd, md);
      else
        w.phase1(xd, yd, zd, md);
      __syncthreads();
      if (tile + 1 < ntiles)
        load_particle(ub, ue, tile + 1);
      else if (un < nunits)
        load_particle(nb, ne, 0);
      w.phase2();
      if (++tcount == a.flush_tiles) {
        tcount = 0;
        w.fold();
      }
      __syncthreads();
    }
    if (ntiles == 0 && un < nunits) load_particle(nb, ne, 0);
    w.fold();
    w.merge_write(lds_raw, reinterpret_cast<typename W::PT*>(a.partials) + size_t(u) * 2 * a.K, a.K);
    __syncthreads();
    ub = nb;
    ue = ne;
  }
}

// ------------------------------------------------------------------ launches
// Dispatch from a plan to the kernel instantiation of its cutoff bucket, register
// block, accumulation mode and particle groups.

template <bool BATCHED, bool DUAL, bool MM, int BASIS, typename T, int LB, int NB, int BS, int MODE,
          int NW, typename Args>
int launch_coeff_t(const CoeffPlan& p, const Args& a, int grid, hipStream_t st) {
  static_assert(!(BATCHED || DUAL) || BASIS == kBasisHO,
                "batched systems and time derivatives use the Hernquist-Ostriker basis");
  const void* kfn;
  if constexpr (BATCHED)
    kfn = reinterpret_cast<const void*>(scf_coeff_batched_kernel<T, LB, NB, BS, MODE, NW, DUAL, MM>);
  else
    kfn = reinterpret_cast<const void*>(scf_coeff_kernel<T, LB, NB, BS, MODE, NW, BASIS, DUAL, MM>);
  // the kernel has no static LDS: the whole 160 KiB of a CU may be requested (once per
  // device and kernel)
  static std::atomic<uint64_t> attr_done{0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  const uint64_t bit = dev < 64 ? (uint64_t(1) << dev) : 0;
  if (!bit || !(attr_done.load(std::memory_order_acquire) & bit)) {
    hipError_t e = hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(scf_coeff)");
    attr_done.fetch_or(bit, std::memory_order_acq_rel);
  }
  int rc = hook_before(st);
  if (rc) return rc;
  if constexpr (BATCHED)
    hipLaunchKernelGGL((scf_coeff_batched_kernel<T, LB, NB, BS, MODE, NW, DUAL, MM>), dim3(grid),
                       dim3(kCoeffThreads), p.lds_bytes, st, a);
  else
    hipLaunchKernelGGL((scf_coeff_kernel<T, LB, NB, BS, MODE, NW, BASIS, DUAL, MM>), dim3(grid),
                       dim3(kCoeffThreads), p.lds_bytes, st, a);
  rc = hip_fail(hipGetLastError(), "scf_coeff_kernel launch");
  return rc ? rc : hook_after(st);
}

template <bool BATCHED, bool DUAL, bool MM, typename T, int MODE, int LB, int NW, int NB, typename Args>
int launch_coeff_basis(const CoeffPlan& p, const Args& a, int grid, hipStream_t st) {
  if constexpr (!BATCHED && !DUAL) {
    if (p.basis == kBasisCB)
      return launch_coeff_t<BATCHED, DUAL, MM, kBasisCB, T, LB, NB, 4, MODE, NW>(p, a, grid, st);
  }
  return launch_coeff_t<BATCHED, DUAL, MM, kBasisHO, T, LB, NB, 4, MODE, NW>(p, a, grid, st);
}

template <bool BATCHED, bool DUAL, bool MM, typename T, int MODE, int LB, int NW, typename Args>
int launch_coeff_nb(const CoeffPlan& p, const Args& a, int grid, hipStream_t st) {
  switch (p.nb) {
    case 9: return launch_coeff_basis<BATCHED, DUAL, MM, T, MODE, LB, NW, 9>(p, a, grid, st);
    case 11: return launch_coeff_basis<BATCHED, DUAL, MM, T, MODE, LB, NW, 11>(p, a, grid, st);
    default: return launch_coeff_basis<BATCHED, DUAL, MM, T, MODE, LB, NW, 12>(p, a, grid, st);
  }
}

// particle groups per tile: only the small cutoff buckets have the LDS for 128 or 256
// particles per tile
template <bool BATCHED, bool DUAL, bool MM, typename T, int MODE, int LB, typename Args>
int launch_coeff_nw(const CoeffPlan& p, const Args& a, int grid, hipStream_t st) {
  if constexpr (LB <= 6) {
    if (p.nw == 1) return launch_coeff_nb<BATCHED, DUAL, MM, T, MODE, LB, 1>(p, a, grid, st);
    if (p.nw == 2) return launch_coeff_nb<BATCHED, DUAL, MM, T, MODE, LB, 2>(p, a, grid, st);
  }
  return launch_coeff_nb<BATCHED, DUAL, MM, T, MODE, LB, 4>(p, a, grid, st);
}

template <bool BATCHED, bool DUAL, bool MM, typename T, int MODE, typename Args>
int launch_coeff_lb(const CoeffPlan& p, const Args& a, int grid, hipStream_t st) {
  switch (p.lb) {
    case 2: return launch_coeff_nw<BATCHED, DUAL, MM, T, MODE, 2>(p, a, grid, st);
    case 6: return launch_coeff_nw<BATCHED, DUAL, MM, T, MODE, 6>(p, a, grid, st);
    case 10: return launch_coeff_nw<BATCHED, DUAL, MM, T, MODE, 10>(p, a, grid, st);
    default: return launch_coeff_nw<BATCHED, DUAL, MM, T, MODE, 14>(p, a, grid, st);
  }
}

// the matrix-core phase 2 (FP32 modes): instantiated in etics_coeff_mm.hip (sums) and
// etics_coeff_mm_dot.hip (time derivatives), so their compile time is spread over files
int launch_coeff_mm(const CoeffPlan& p, const CoeffArgs& a, int grid, hipStream_t st);
int launch_coeff_mm(const CoeffPlan& p, const BatchedCoeffArgs& a, int grid, hipStream_t st);
int launch_coeff_mm_dual(const CoeffPlan& p, const CoeffArgs& a, int grid, hipStream_t st);
int launch_coeff_mm_dual(const CoeffPlan& p, const BatchedCoeffArgs& a, int grid, hipStream_t st);

template <bool BATCHED, bool DUAL, bool MM, typename Args>
int launch_coeff_modes(const CoeffPlan& p, const Args& a, int grid, hipStream_t st) {
  if constexpr (MM) {
    if (p.prec == ETICS_FP64) {
      set_error("internal: matrix-core phase 2 is FP32 only");
      return ETICS_EUNSUPPORTED;
    }
    if (p.prec == ETICS_MIXED_FP64ACC) return launch_coeff_lb<BATCHED, DUAL, true, float, 0>(p, a, grid, st);
    return launch_coeff_lb<BATCHED, DUAL, true, float, 1>(p, a, grid, st);
  } else {
    if (p.prec == ETICS_FP64) return launch_coeff_lb<BATCHED, DUAL, false, double, 0>(p, a, grid, st);
    if (p.prec == ETICS_MIXED_FP64ACC) return launch_coeff_lb<BATCHED, DUAL, false, float, 0>(p, a, grid, st);
    return launch_coeff_lb<BATCHED, DUAL, false, float, 1>(p, a, grid, st);
  }
}

template <bool BATCHED, bool DUAL, typename Args>
int launch_coeff_any(const CoeffPlan& p, const Args& a, int grid, hipStream_t st) {
  if (p.mfma) return DUAL ? launch_coeff_mm_dual(p, a, grid, st) : launch_coeff_mm(p, a, grid, st);
  return launch_coeff_modes<BATCHED, DUAL, false>(p, a, grid, st);
}

// host side (etics_coeff.hip): argument blocks, the fixed-order reductions and the plan
// of the time-derivative sums
CoeffArgs coeff_args(const CoeffPlan& p, const double* x, const double* y, const double* z,
                     const double* m, int64_t n, int tile_particles, void* ws);
BatchedCoeffArgs batched_coeff_args(const CoeffPlan& p, const double* x, const double* y,
                                    const double* z, const double* m, const int64_t* offsets,
                                    const int* ustart, const int* usys, int nsys, int64_t ntotal,
                                    void* partials);
int launch_coeff_reduce(const CoeffPlan& p, const void* partials, int grid, double* A, double* B,
                        hipStream_t st);
int launch_coeff_reduce_batched(const CoeffPlan& p, const void* partials, const int* ustart, int nsys,
                                double* A, double* B, hipStream_t st);

}  // namespace etics
