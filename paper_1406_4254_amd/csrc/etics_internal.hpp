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

// Timing events of the calling thread (etics_set_timing_events): recorded on the
// stream right before and right after the main kernel of a compute call.
struct TimingHook {
  hipEvent_t before = nullptr, after = nullptr;
  bool suspended = false;  // set while a call replays captured work (leapfrog)
};
TimingHook& timing_hook();
int hook_before(hipStream_t st);
int hook_after(hipStream_t st);

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
inline int lm_count(int lmax) { return (lmax + 1) * (lmax + 2) / 2; }
inline int coeff_count(int nmax, int lmax) { return (nmax + 1) * lm_count(lmax); }

// ---------------------------------------------------------------- SCF plan
// Tile configuration of the coefficient kernel (chosen per (nmax, lmax, precision)).
constexpr int kCoeffThreads = 256;  // 4 wavefronts
constexpr int kMaxStreams = 32;      // stream copies merged one after another at the end
constexpr int kUnitParticles = 4096;  // batched work unit (default): particles of one system
constexpr int kMinUnitParticles = 256;      // limits of a tuned work unit
constexpr int kMaxUnitParticles = 1 << 20;
constexpr int kForceSplit = 4;  // batched force workgroups per unit (default)

struct CoeffPlan {
  int nmax, lmax, prec;   // prec: ETICS_* precision mode
  int basis;              // radial basis (kBasisHO or kBasisCB)
  int lb;                 // compile-time lmax bucket of the kernel (lmax <= lb)
  int nb, bs;             // register block: nb radial orders x bs angular slots
  int nchunks;            // radial chunks of nb orders
  int spg, spz;           // LDS strides (elements) per particle: radial rows, angular slots
  int nw;                 // wavefronts sharing the basis jobs of a group of 64 particles
  int tp;                 // particles per tile
  int nblocks, streams;   // register blocks per stream, streams per workgroup
  int flush_tiles;        // FP32 run length (tiles) before folding into the wide accumulator
  int grid_mult;          // workgroups per CU (grid = 256 grid_mult, at most the work items)
  int grid;               // workgroups of a single-system launch
  int unit, split;        // batched: particles per work unit, force workgroups per unit
  bool mfma;              // FP32 outer products on the matrix cores (else the VALU)
  bool tuned;             // the tile shape came from the tuner's table
  size_t lds_bytes;
};

// Tile shape measured by the tuner (0 = keep the fixed rule's value; phase2: 1 = VALU,
// 2 = matrix cores).
struct TunedParams {
  int nw, tp, streams, grid_mult, unit, split, phase2;
};
// The tuner's plan for this key and particle count, if it holds one (etics_tune.cpp).
bool tuned_lookup(int batched, int nmax, int lmax, int prec, int basis, int64_t n, TunedParams* out);

// The plan of a coefficient call over n particles (batched: ntotal); false if the
// cutoffs have none.  A valid tuned plan overrides the fixed rules.
bool make_coeff_plan(int64_t n, int nmax, int lmax, int prec, CoeffPlan* p, int basis = kBasisHO,
                     bool batched = false);
// workgroups of a launch over work_items tiles (single system) or units (batched)
int coeff_grid(const CoeffPlan& p, int64_t work_items);
size_t coeff_partials_bytes(const CoeffPlan& p);
size_t force_prep_bytes(int nmax, int lmax, int prec);

int launch_fill_zero(double* p, int64_t count, hipStream_t st);

// Plan of the time-derivative sums derived from a coefficient plan p over n particles
// (tiles of an even number of rows, two per particle); false if none fits.
bool dot_plan(const CoeffPlan& p, int64_t n, CoeffPlan* out);
// d/dt of the coefficients along the velocities (etics_coeff_dot.hip); ws as for
// launch_scf_coeffs (sized for the plan's dot_plan)
int launch_scf_coeffs_dot(const CoeffPlan& p, const double* x, const double* y, const double* z,
                          const double* vx, const double* vy, const double* vz, const double* m,
                          int64_t n, double* Ad, double* Bd, void* ws, hipStream_t st);
int launch_scf_coeffs_dot_batched(const CoeffPlan& p, const double* x, const double* y,
                                  const double* z, const double* vx, const double* vy,
                                  const double* vz, const double* m, const int64_t* offsets,
                                  const int* ustart, const int* usys, int nsys, int64_t ntotal,
                                  double* Ad, double* Bd, void* partials, hipStream_t st);
size_t jerk_prep_bytes(int nmax, int lmax, int prec);
// acceleration and jerk at (x, v) from A, B and their time derivatives (etics_jerk.hip)
int launch_scf_jerk(const double* x, const double* y, const double* z, const double* vx,
                    const double* vy, const double* vz, int64_t n, int nmax, int lmax,
                    const double* A, const double* B, const double* Ad, const double* Bd, int prec,
                    double* ax, double* ay, double* az, double* jx, double* jy, double* jz, void* ws,
                    hipStream_t st);
size_t hermite_ws_bytes(int64_t ntotal, int nsys, int nmax, int lmax, int prec);
int run_hermite(double* x, double* y, double* z, double* vx, double* vy, double* vz,
                const double* m, const int64_t* offsets, int nsys, int64_t ntotal, int nmax, int lmax,
                int prec, double dt, int nsteps, int flags, void* ws, size_t ws_bytes, hipStream_t st);

// device memory of the allocation-free coefficient call (partials of one call)
constexpr size_t kNoallocScratchBytes = size_t(24) << 20;
// device address of that memory on the current device (looked up once per device)
int noalloc_scratch(void** out);

int launch_scf_coeffs(const CoeffPlan& p, const double* x, const double* y, const double* z,
                      const double* m, int64_t n, double* A, double* B, void* ws,
                      hipStream_t st);
int launch_scf_force(const double* x, const double* y, const double* z, int64_t n, int nmax,
                     int lmax, const double* A, const double* B, int prec, int outputs,
                     double* pot, double* ax, double* ay, double* az, void* ws, hipStream_t st,
                     int basis = kBasisHO);

int max_units(int64_t ntotal, int nsys, int unit);
int launch_scf_coeffs_batched(const CoeffPlan& p, const double* x, const double* y, const double* z,
                              const double* m, const int64_t* offsets, const int* ustart,
                              const int* usys, int nsys, int64_t ntotal, double* A, double* B,
                              void* partials, hipStream_t st);
// Leapfrog update applied by the batched force kernel to each particle right after its
// acceleration a is known, instead of storing a: mode 1 = closing kick v += h a;
// mode 2 = closing kick, then the next step's opening kick v += h a and drift
// x += dt v.  Each operation is one FP64 fused multiply-add, as in the separate kernels.
struct LfUpdate {
  double *x, *y, *z, *vx, *vy, *vz;
  double h, dt;
  int mode;
};

int launch_scf_force_batched(const CoeffPlan& plan, const double* x, const double* y,
                             const double* z, const int64_t* offsets, const int* ustart,
                             const int* usys, int nsys, int64_t ntotal, const double* A,
                             const double* B, int outputs, double* pot, double* ax, double* ay,
                             double* az, void* prep, hipStream_t st, const LfUpdate* lf = nullptr);

struct BatchedLayout {
  size_t off_ustart, off_usys, off_partials, off_prep, off_A, off_B, off_acc, total;
  int max_units;
  CoeffPlan plan;  // the batched plan the layout was sized for
  bool ok;         // false: no plan for these cutoffs
};
BatchedLayout batched_layout(int64_t ntotal, int nsys, int nmax, int lmax, int prec);
int launch_units(const int64_t* offsets, int nsys, int64_t ntotal, int unit, int* ustart, int* usys,
                 hipStream_t st);
int run_leapfrog(double* x, double* y, double* z, double* vx, double* vy, double* vz,
                 const double* m, const int64_t* offsets, int nsys, int64_t ntotal, int nmax,
                 int lmax, int prec, double dt, int nsteps, int flags, void* ws, size_t ws_bytes,
                 hipStream_t st);

size_t mex_ws_bytes(int64_t n, int lmax);
int launch_mex_force(const double* x, const double* y, const double* z, const double* m, int64_t n,
                     int lmax, int prec, int outputs, double* pot, double* ax, double* ay,
                     double* az, void* ws, hipStream_t st);
int launch_direct_force(const double* x, const double* y, const double* z, const double* m,
                        int64_t n, int outputs, double* pot, double* ax, double* ay, double* az,
                        hipStream_t st);

}  // namespace etics
