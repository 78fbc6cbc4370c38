// etics_internal.hpp -- shared declarations of the library's host side.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "etics.h"
#include "etics_tables.hpp"

namespace etics {

void set_error(const std::string& msg);
int hip_fail(hipError_t e, const char* where);

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
inline int lm_count(int lmax) { return (lmax + 1) * (lmax + 2) / 2; }
inline int coeff_count(int nmax, int lmax) { return (nmax + 1) * lm_count(lmax); }

// ---------------------------------------------------------------- SCF plan
// Tile configuration of the coefficient kernel (chosen per (nmax, lmax, precision)).
constexpr int kCoeffThreads = 256;  // 4 wavefronts
constexpr int kMaxJobs = 32;        // basis jobs per wavefront (2 (lmax+1) <= 30)
constexpr int kMaxStreams = 32;

struct CoeffPlan {
  int nmax, lmax, prec;   // prec: ETICS_* precision mode
  int lb;                 // compile-time lmax bucket of the kernel (lmax <= lb)
  int nb, bs;             // register block: nb radial orders x bs angular slots
  int nchunks;            // radial chunks of nb orders
  int spg, spz;           // LDS strides (elements) per particle: radial rows, angular slots
  int tp;                 // particles per tile
  int nblocks, streams;   // register blocks per stream, streams per workgroup
  int flush_tiles;        // FP32 run length (tiles) before folding into the wide accumulator
  int grid;               // workgroups
  size_t lds_bytes;
};

bool make_coeff_plan(int64_t n, int nmax, int lmax, int prec, CoeffPlan* p);
size_t coeff_partials_bytes(const CoeffPlan& p);
size_t force_prep_bytes(int nmax, int lmax, int prec);

int launch_fill_zero(double* p, int64_t count, hipStream_t st);

int launch_scf_coeffs(const CoeffPlan& p, const double* x, const double* y, const double* z,
                      const double* m, int64_t n, double* A, double* B, void* ws,
                      hipStream_t st);
int launch_scf_force(const double* x, const double* y, const double* z, int64_t n, int nmax,
                     int lmax, const double* A, const double* B, int prec, int outputs,
                     double* pot, double* ax, double* ay, double* az, void* ws, hipStream_t st);

size_t mex_ws_bytes(int64_t n, int lmax);
int launch_mex_force(const double* x, const double* y, const double* z, const double* m, int64_t n,
                     int lmax, int prec, int outputs, double* pot, double* ax, double* ay,
                     double* az, void* ws, hipStream_t st);

}  // namespace etics
