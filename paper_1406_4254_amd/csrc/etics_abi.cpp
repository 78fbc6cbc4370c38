// etics_abi.cpp -- the C-ABI entry points of libetics.so: argument validation,
// workspace sizing and dispatch to the HIP kernels.  No entry point allocates device
// memory, synchronises or copies to/from the host; the leapfrog alone creates a
// library stream and instantiates a graph on its first use.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <cstring>
#include <string>

#include "etics_internal.hpp"

namespace etics {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int hip_fail(hipError_t e, const char* where) {
  if (e == hipSuccess) return ETICS_OK;
  set_error(std::string(where) + ": " + hipGetErrorString(e));
  return ETICS_EHIP;
}

static thread_local TimingHook g_hook;

TimingHook& timing_hook() { return g_hook; }

int hook_before(hipStream_t st) {
  if (!g_hook.before || g_hook.suspended) return ETICS_OK;
  return hip_fail(hipEventRecord(g_hook.before, st), "hipEventRecord(timing before)");
}

int hook_after(hipStream_t st) {
  if (!g_hook.after || g_hook.suspended) return ETICS_OK;
  return hip_fail(hipEventRecord(g_hook.after, st), "hipEventRecord(timing after)");
}

static int einval(const char* what) {
  set_error(std::string("invalid argument: ") + what);
  return ETICS_EINVAL;
}

static bool valid_prec(int p) {
  return p == ETICS_FP64 || p == ETICS_MIXED_FP64ACC || p == ETICS_MIXED_COMP32;
}

static bool valid_cut(int nmax, int lmax) {
  return nmax >= 0 && nmax <= ETICS_NMAX_CAP && lmax >= 0 && lmax <= ETICS_LMAX_CAP;
}

static const size_t kAlign = 256;

size_t scf_ws_bytes(int64_t n, int nmax, int lmax, int prec) {
  // the largest partials over both bases (their plans may be tuned differently) and the
  // time-derivative sums, or the prepared coefficients of the force and jerk passes
  CoeffPlan p, q, d;
  if (!make_coeff_plan(n, nmax, lmax, prec, &p, kBasisHO) ||
      !make_coeff_plan(n, nmax, lmax, prec, &q, kBasisCB) || !dot_plan(p, n, &d))
    return 0;
  size_t need = coeff_partials_bytes(p);
  if (coeff_partials_bytes(q) > need) need = coeff_partials_bytes(q);
  if (coeff_partials_bytes(d) > need) need = coeff_partials_bytes(d);
  if (force_prep_bytes(nmax, lmax, prec) > need) need = force_prep_bytes(nmax, lmax, prec);
  if (jerk_prep_bytes(nmax, lmax, prec) > need) need = jerk_prep_bytes(nmax, lmax, prec);
  return align_up(need, kAlign);
}

}  // namespace etics

using namespace etics;

extern "C" {

int etics_coeff_count(int nmax, int lmax) {
  if (!valid_cut(nmax, lmax)) return -1;
  return coeff_count(nmax, lmax);
}

int etics_set_timing_events(void* before, void* after) {
  if ((before == nullptr) != (after == nullptr))
    return einval("timing events must both be set or both be NULL");
  g_hook.before = static_cast<hipEvent_t>(before);
  g_hook.after = static_cast<hipEvent_t>(after);
  return ETICS_OK;
}

int etics_plan_info(int batched, int64_t n, int nmax, int lmax, int precision, int basis, int* out,
                    int nout) {
  if (n < 0 || !valid_cut(nmax, lmax) || !valid_prec(precision)) return einval("n, cutoffs or precision");
  if (basis != ETICS_BASIS_HO && basis != ETICS_BASIS_CB) return einval("basis");
  if ((batched != 0 && batched != 1) || (batched && basis != ETICS_BASIS_HO)) return einval("batched");
  if (!out || nout < 9) return einval("out needs 9 entries");
  CoeffPlan p;
  if (!make_coeff_plan(n, nmax, lmax, precision, &p, basis, batched != 0)) {
    set_error("no tile plan for these cutoffs");
    return ETICS_EUNSUPPORTED;
  }
  const int v[9] = {p.nw, p.tp, p.streams, p.grid_mult, p.unit, p.split, p.mfma ? 2 : 1, p.tuned ? 1 : 0,
                    p.grid};
  for (int i = 0; i < 9; ++i) out[i] = v[i];
  return ETICS_OK;
}

const char* etics_last_error(void) { return g_last_error.c_str(); }

const char* etics_version(void) { return "etics-mi355x 0.1 (gfx950)"; }

size_t etics_scf_workspace_size(int64_t n, int nmax, int lmax, int precision) {
  if (n < 0 || !valid_cut(nmax, lmax) || !valid_prec(precision)) return 0;
  return scf_ws_bytes(n, nmax, lmax, precision);
}

static int scf_coeffs_impl(const double* x, const double* y, const double* z, const double* m,
                           int64_t n, int nmax, int lmax, int precision, int basis, double* A,
                           double* B, void* workspace, size_t ws_bytes, void* stream) {
  if (n < 0) return einval("n < 0");
  if (!valid_cut(nmax, lmax)) return einval("nmax/lmax outside [0, cap]");
  if (!valid_prec(precision)) return einval("precision");
  if (basis != ETICS_BASIS_HO && basis != ETICS_BASIS_CB) return einval("basis");
  if (!A || !B) return einval("A/B is NULL");
  if (n > 0 && (!x || !y || !z || !m)) return einval("x/y/z/m is NULL");
  const size_t need = scf_ws_bytes(n, nmax, lmax, precision);
  if (need == 0) {
    set_error("no tile plan for these cutoffs");
    return ETICS_EUNSUPPORTED;
  }
  if (!workspace || ws_bytes < need) {
    set_error("workspace too small: need " + std::to_string(need) + " bytes");
    return ETICS_EWORKSPACE;
  }
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return einval("workspace not 256-byte aligned");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int K = coeff_count(nmax, lmax);
  if (n == 0) {
    int rc = launch_fill_zero(A, K, st);
    return rc ? rc : launch_fill_zero(B, K, st);
  }
  CoeffPlan p;
  make_coeff_plan(n, nmax, lmax, precision, &p, basis);
  return launch_scf_coeffs(p, x, y, z, m, n, A, B, workspace, st);
}

int etics_scf_coeffs(const double* x, const double* y, const double* z, const double* m,
                     int64_t n, int nmax, int lmax, int precision, double* A, double* B,
                     void* workspace, size_t ws_bytes, void* stream) {
  return scf_coeffs_impl(x, y, z, m, n, nmax, lmax, precision, ETICS_BASIS_HO, A, B, workspace,
                         ws_bytes, stream);
}

int etics_scf_coeffs_basis(const double* x, const double* y, const double* z, const double* m,
                           int64_t n, int nmax, int lmax, int precision, int basis, double* A,
                           double* B, void* workspace, size_t ws_bytes, void* stream) {
  return scf_coeffs_impl(x, y, z, m, n, nmax, lmax, precision, basis, A, B, workspace, ws_bytes,
                         stream);
}

int etics_scf_coeffs_noalloc(const double* x, const double* y, const double* z, const double* m,
                             int64_t n, int nmax, int lmax, int precision, double* A, double* B,
                             void* stream) {
  if (n < 0) return einval("n < 0");
  if (!valid_cut(nmax, lmax)) return einval("nmax/lmax outside [0, cap]");
  if (!valid_prec(precision)) return einval("precision");
  if (!A || !B) return einval("A/B is NULL");
  if (n > 0 && (!x || !y || !z || !m)) return einval("x/y/z/m is NULL");
  CoeffPlan p;
  if (!make_coeff_plan(n, nmax, lmax, precision, &p)) {
    set_error("no tile plan for these cutoffs");
    return ETICS_EUNSUPPORTED;
  }
  const size_t need = coeff_partials_bytes(p);
  if (need > kNoallocScratchBytes) {
    set_error("etics_scf_coeffs_noalloc: the partial sums need " + std::to_string(need) +
              " bytes, above the fixed " + std::to_string(kNoallocScratchBytes) + "-byte scratch");
    return ETICS_EWORKSPACE;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (n == 0) {
    const int K = coeff_count(nmax, lmax);
    int rc = launch_fill_zero(A, K, st);
    return rc ? rc : launch_fill_zero(B, K, st);
  }
  void* ws = nullptr;
  int rc = noalloc_scratch(&ws);
  if (rc) return rc;
  return launch_scf_coeffs(p, x, y, z, m, n, A, B, ws, st);
}

static int scf_force_impl(const double* x, const double* y, const double* z, int64_t n, int nmax,
                          int lmax, const double* A, const double* B, int precision, int basis,
                          int outputs, double* pot, double* ax, double* ay, double* az,
                          void* workspace, size_t ws_bytes, void* stream) {
  if (n < 0) return einval("n < 0");
  if (!valid_cut(nmax, lmax)) return einval("nmax/lmax outside [0, cap]");
  if (!valid_prec(precision)) return einval("precision");
  if (outputs < 1 || outputs > 3) return einval("outputs");
  if (basis != ETICS_BASIS_HO && basis != ETICS_BASIS_CB) return einval("basis");
  if (!A || !B) return einval("A/B is NULL");
  if (n > 0 && (!x || !y || !z)) return einval("x/y/z is NULL");
  if (n > 0 && (outputs & ETICS_POT) && !pot) return einval("pot is NULL");
  if (n > 0 && (outputs & ETICS_ACC) && (!ax || !ay || !az)) return einval("ax/ay/az is NULL");
  const size_t need = scf_ws_bytes(n, nmax, lmax, precision);
  if (need == 0) {
    set_error("no tile plan for these cutoffs");
    return ETICS_EUNSUPPORTED;
  }
  if (!workspace || ws_bytes < need) {
    set_error("workspace too small: need " + std::to_string(need) + " bytes");
    return ETICS_EWORKSPACE;
  }
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return einval("workspace not 256-byte aligned");
  if (n == 0) return ETICS_OK;
  return launch_scf_force(x, y, z, n, nmax, lmax, A, B, precision, outputs, pot, ax, ay, az,
                          workspace, reinterpret_cast<hipStream_t>(stream), basis);
}

int etics_scf_force(const double* x, const double* y, const double* z, int64_t n, int nmax,
                    int lmax, const double* A, const double* B, int precision, int outputs,
                    double* pot, double* ax, double* ay, double* az, void* workspace,
                    size_t ws_bytes, void* stream) {
  return scf_force_impl(x, y, z, n, nmax, lmax, A, B, precision, ETICS_BASIS_HO, outputs, pot, ax,
                        ay, az, workspace, ws_bytes, stream);
}

int etics_scf_force_basis(const double* x, const double* y, const double* z, int64_t n, int nmax,
                          int lmax, const double* A, const double* B, int precision, int basis,
                          int outputs, double* pot, double* ax, double* ay, double* az,
                          void* workspace, size_t ws_bytes, void* stream) {
  return scf_force_impl(x, y, z, n, nmax, lmax, A, B, precision, basis, outputs, pot, ax, ay, az,
                        workspace, ws_bytes, stream);
}

// ---------------------------------------------------------------- jerk
static int check_ws(void* workspace, size_t ws_bytes, size_t need) {
  if (need == 0) {
    set_error("no tile plan for these cutoffs");
    return ETICS_EUNSUPPORTED;
  }
  if (!workspace || ws_bytes < need) {
    set_error("workspace too small: need " + std::to_string(need) + " bytes");
    return ETICS_EWORKSPACE;
  }
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return einval("workspace not 256-byte aligned");
  return ETICS_OK;
}

int etics_scf_coeffs_dot(const double* x, const double* y, const double* z, const double* vx,
                         const double* vy, const double* vz, const double* m, int64_t n, int nmax,
                         int lmax, int precision, double* Adot, double* Bdot, void* workspace,
                         size_t ws_bytes, void* stream) {
  if (n < 0) return einval("n < 0");
  if (!valid_cut(nmax, lmax)) return einval("nmax/lmax outside [0, cap]");
  if (!valid_prec(precision)) return einval("precision");
  if (!Adot || !Bdot) return einval("Adot/Bdot is NULL");
  if (n > 0 && (!x || !y || !z || !vx || !vy || !vz || !m)) return einval("x/y/z/vx/vy/vz/m is NULL");
  int rc = check_ws(workspace, ws_bytes, scf_ws_bytes(n, nmax, lmax, precision));
  if (rc) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (n == 0) {
    const int K = coeff_count(nmax, lmax);
    rc = launch_fill_zero(Adot, K, st);
    return rc ? rc : launch_fill_zero(Bdot, K, st);
  }
  CoeffPlan p;
  make_coeff_plan(n, nmax, lmax, precision, &p);
  return launch_scf_coeffs_dot(p, x, y, z, vx, vy, vz, m, n, Adot, Bdot, workspace, st);
}

int etics_scf_jerk(const double* x, const double* y, const double* z, const double* vx,
                   const double* vy, const double* vz, int64_t n, int nmax, int lmax, const double* A,
                   const double* B, const double* Adot, const double* Bdot, int precision, double* ax,
                   double* ay, double* az, double* jx, double* jy, double* jz, void* workspace,
                   size_t ws_bytes, void* stream) {
  if (n < 0) return einval("n < 0");
  if (!valid_cut(nmax, lmax)) return einval("nmax/lmax outside [0, cap]");
  if (!valid_prec(precision)) return einval("precision");
  if (!A || !B || !Adot || !Bdot) return einval("A/B/Adot/Bdot is NULL");
  if (n > 0 && (!x || !y || !z || !vx || !vy || !vz)) return einval("x/y/z/vx/vy/vz is NULL");
  if (n > 0 && (!ax || !ay || !az || !jx || !jy || !jz)) return einval("ax/ay/az/jx/jy/jz is NULL");
  int rc = check_ws(workspace, ws_bytes, scf_ws_bytes(n, nmax, lmax, precision));
  if (rc) return rc;
  if (n == 0) return ETICS_OK;
  return launch_scf_jerk(x, y, z, vx, vy, vz, n, nmax, lmax, A, B, Adot, Bdot, precision, ax, ay, az, jx,
                         jy, jz, workspace, reinterpret_cast<hipStream_t>(stream));
}

size_t etics_mex_workspace_size(int64_t n, int lmax, int precision) {
  if (n < 0 || n > INT32_MAX || lmax < 0 || lmax > ETICS_LMAX_CAP || !valid_prec(precision)) return 0;
  return mex_ws_bytes(n, lmax);
}

int etics_mex_force(const double* x, const double* y, const double* z, const double* m, int64_t n,
                    int lmax, int precision, int outputs, double* pot, double* ax, double* ay,
                    double* az, void* workspace, size_t ws_bytes, void* stream) {
  if (n < 0) return einval("n < 0");
  if (n > INT32_MAX) {
    set_error("etics_mex_force: n must be below 2^31 (32-bit sort indices)");
    return ETICS_EUNSUPPORTED;
  }
  if (lmax < 0 || lmax > ETICS_LMAX_CAP) return einval("lmax outside [0, cap]");
  if (!valid_prec(precision)) return einval("precision");
  if (outputs < 1 || outputs > 3) return einval("outputs");
  if (n > 0 && (!x || !y || !z || !m)) return einval("x/y/z/m is NULL");
  if (n > 0 && (outputs & ETICS_POT) && !pot) return einval("pot is NULL");
  if (n > 0 && (outputs & ETICS_ACC) && (!ax || !ay || !az)) return einval("ax/ay/az is NULL");
  const size_t need = mex_ws_bytes(n, lmax);
  if (!workspace || ws_bytes < need) {
    set_error("workspace too small: need " + std::to_string(need) + " bytes");
    return ETICS_EWORKSPACE;
  }
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return einval("workspace not 256-byte aligned");
  if (n == 0) return ETICS_OK;
  return launch_mex_force(x, y, z, m, n, lmax, precision, outputs, pot, ax, ay, az, workspace,
                          reinterpret_cast<hipStream_t>(stream));
}

// ---------------------------------------------------------------- direct summation
int etics_direct_force(const double* x, const double* y, const double* z, const double* m,
                       int64_t n, int outputs, double* pot, double* ax, double* ay, double* az,
                       void* stream) {
  if (n < 0) return einval("n < 0");
  if (n > INT32_MAX) return einval("n must be below 2^31");
  if (outputs < 1 || outputs > 3) return einval("outputs");
  if (n > 0 && (!x || !y || !z || !m)) return einval("x/y/z/m is NULL");
  if (n > 0 && (outputs & ETICS_POT) && !pot) return einval("pot is NULL");
  if (n > 0 && (outputs & ETICS_ACC) && (!ax || !ay || !az)) return einval("ax/ay/az is NULL");
  if (n == 0) return ETICS_OK;
  return launch_direct_force(x, y, z, m, n, outputs, pot, ax, ay, az,
                             reinterpret_cast<hipStream_t>(stream));
}

// ---------------------------------------------------------------- batched + leapfrog
static int check_batched(int64_t ntotal, int nsys, int nmax, int lmax, int prec, const void* offsets) {
  if (ntotal < 0) return einval("ntotal < 0");
  if (nsys < 1) return einval("nsys < 1");
  if (!valid_cut(nmax, lmax)) return einval("nmax/lmax outside [0, cap]");
  if (!valid_prec(prec)) return einval("precision");
  if (!offsets) return einval("offsets is NULL");
  if (ntotal / kMinUnitParticles + nsys > INT32_MAX / 2) {
    set_error("too many particles or systems for 32-bit unit indices");
    return ETICS_EUNSUPPORTED;
  }
  return ETICS_OK;
}

size_t etics_batched_workspace_size(int64_t ntotal, int nsys, int nmax, int lmax, int precision) {
  if (ntotal < 0 || nsys < 1 || !valid_cut(nmax, lmax) || !valid_prec(precision)) return 0;
  if (ntotal / kMinUnitParticles + nsys > INT32_MAX / 2) return 0;
  const BatchedLayout L = batched_layout(ntotal, nsys, nmax, lmax, precision);
  return L.ok ? L.total : 0;
}

int etics_scf_coeffs_batched(const double* x, const double* y, const double* z, const double* m,
                             const int64_t* offsets, int nsys, int64_t ntotal, int nmax, int lmax,
                             int precision, double* A, double* B, void* workspace, size_t ws_bytes,
                             void* stream) {
  int rc = check_batched(ntotal, nsys, nmax, lmax, precision, offsets);
  if (rc) return rc;
  if (!A || !B) return einval("A/B is NULL");
  if (ntotal > 0 && (!x || !y || !z || !m)) return einval("x/y/z/m is NULL");
  const BatchedLayout L = batched_layout(ntotal, nsys, nmax, lmax, precision);
  if (!L.ok) {
    set_error("no tile plan for these cutoffs");
    return ETICS_EUNSUPPORTED;
  }
  if (!workspace || ws_bytes < L.total) {
    set_error("workspace too small: need " + std::to_string(L.total) + " bytes");
    return ETICS_EWORKSPACE;
  }
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return einval("workspace not 256-byte aligned");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* base = reinterpret_cast<char*>(workspace);
  int* ustart = reinterpret_cast<int*>(base + L.off_ustart);
  int* usys = reinterpret_cast<int*>(base + L.off_usys);
  rc = launch_units(offsets, nsys, ntotal, L.plan.unit, ustart, usys, st);
  if (rc) return rc;
  return launch_scf_coeffs_batched(L.plan, x, y, z, m, offsets, ustart, usys, nsys, ntotal, A, B,
                                   base + L.off_partials, st);
}

int etics_scf_force_batched(const double* x, const double* y, const double* z,
                            const int64_t* offsets, int nsys, int64_t ntotal, int nmax, int lmax,
                            const double* A, const double* B, int precision, int outputs,
                            double* pot, double* ax, double* ay, double* az, void* workspace,
                            size_t ws_bytes, void* stream) {
  int rc = check_batched(ntotal, nsys, nmax, lmax, precision, offsets);
  if (rc) return rc;
  if (outputs < 1 || outputs > 3) return einval("outputs");
  if (!A || !B) return einval("A/B is NULL");
  if (ntotal > 0 && (!x || !y || !z)) return einval("x/y/z is NULL");
  if (ntotal > 0 && (outputs & ETICS_POT) && !pot) return einval("pot is NULL");
  if (ntotal > 0 && (outputs & ETICS_ACC) && (!ax || !ay || !az)) return einval("ax/ay/az is NULL");
  const BatchedLayout L = batched_layout(ntotal, nsys, nmax, lmax, precision);
  if (!L.ok) {
    set_error("no tile plan for these cutoffs");
    return ETICS_EUNSUPPORTED;
  }
  if (!workspace || ws_bytes < L.total) {
    set_error("workspace too small: need " + std::to_string(L.total) + " bytes");
    return ETICS_EWORKSPACE;
  }
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return einval("workspace not 256-byte aligned");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* base = reinterpret_cast<char*>(workspace);
  int* ustart = reinterpret_cast<int*>(base + L.off_ustart);
  int* usys = reinterpret_cast<int*>(base + L.off_usys);
  rc = launch_units(offsets, nsys, ntotal, L.plan.unit, ustart, usys, st);
  if (rc) return rc;
  return launch_scf_force_batched(L.plan, x, y, z, offsets, ustart, usys, nsys, ntotal, A, B, outputs,
                                  pot, ax, ay, az, base + L.off_prep, st);
}

size_t etics_hermite_workspace_size(int64_t ntotal, int nsys, int nmax, int lmax, int precision) {
  if (ntotal < 0 || nsys < 1 || !valid_cut(nmax, lmax) || !valid_prec(precision)) return 0;
  if (ntotal / kMinUnitParticles + nsys > INT32_MAX / 2) return 0;
  return hermite_ws_bytes(ntotal, nsys, nmax, lmax, precision);
}

int etics_hermite_scf_batched(double* x, double* y, double* z, double* vx, double* vy, double* vz,
                              const double* m, const int64_t* offsets, int nsys, int64_t ntotal,
                              int nmax, int lmax, int precision, double dt, int nsteps, int flags,
                              void* workspace, size_t ws_bytes, void* stream) {
  int rc = check_batched(ntotal, nsys, nmax, lmax, precision, offsets);
  if (rc) return rc;
  if (nsteps < 0) return einval("nsteps < 0");
  if (!(dt == dt)) return einval("dt is NaN");
  if (ntotal > 0 && (!x || !y || !z || !vx || !vy || !vz || !m)) return einval("state pointer is NULL");
  rc = check_ws(workspace, ws_bytes, hermite_ws_bytes(ntotal, nsys, nmax, lmax, precision));
  if (rc) return rc;
  if (nsteps == 0 || ntotal == 0) return ETICS_OK;
  return run_hermite(x, y, z, vx, vy, vz, m, offsets, nsys, ntotal, nmax, lmax, precision, dt, nsteps, flags,
                     workspace, ws_bytes, reinterpret_cast<hipStream_t>(stream));
}

int etics_leapfrog_scf_batched(double* x, double* y, double* z, double* vx, double* vy, double* vz,
                               const double* m, const int64_t* offsets, int nsys, int64_t ntotal,
                               int nmax, int lmax, int precision, double dt, int nsteps, int flags,
                               void* workspace, size_t ws_bytes, void* stream) {
  int rc = check_batched(ntotal, nsys, nmax, lmax, precision, offsets);
  if (rc) return rc;
  if (nsteps < 0) return einval("nsteps < 0");
  if (!(dt == dt)) return einval("dt is NaN");
  if (ntotal > 0 && (!x || !y || !z || !vx || !vy || !vz || !m)) return einval("state pointer is NULL");
  const BatchedLayout L = batched_layout(ntotal, nsys, nmax, lmax, precision);
  if (!L.ok) {
    set_error("no tile plan for these cutoffs");
    return ETICS_EUNSUPPORTED;
  }
  if (!workspace || ws_bytes < L.total) {
    set_error("workspace too small: need " + std::to_string(L.total) + " bytes");
    return ETICS_EWORKSPACE;
  }
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return einval("workspace not 256-byte aligned");
  if (nsteps == 0 || ntotal == 0) return ETICS_OK;
  return run_leapfrog(x, y, z, vx, vy, vz, m, offsets, nsys, ntotal, nmax, lmax, precision, dt,
                      nsteps, flags, workspace, ws_bytes, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
