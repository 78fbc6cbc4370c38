// etics_jerk.hip -- the SCF jerk and the batched fourth-order Hermite integrator.
//
// The paper notes that Hernquist's SCF code computes the jerk, the time derivative of
// the force (Section 3.4), for its fourth-order Hermite scheme, and names that scheme
// as the next integrator for SCF (Section 5.4; not for MEX, whose force derivative is
// discontinuous at shell crossings).  Here the jerk of particle i is the total time
// derivative of its acceleration when every particle moves with its velocity:
//   j_i = d/dt a(x_i + v_i t; A(t), B(t)) at t = 0,
// with dA/dt, dB/dt from etics_coeff_dot.hip.  The synthesis of etics_force_synth.hpp
// runs on Dual numbers (value, time derivative): the field point carries its velocity
// and each prepared coefficient its time derivative, so the one pass returns a and j.
//
// Hermite predictor-corrector (Makino & Aarseth 1992), one shared step dt per call:
//   predict  x_p = x + v dt + a dt^2/2 + j dt^3/6,   v_p = v + a dt + j dt^2/2,
//   evaluate a_1, j_1 at (x_p, v_p)  (coefficients and their derivatives there),
//   correct  v_1 = v + (a + a_1) dt/2 + (j - j_1) dt^2/12,
//            x_1 = x + (v + v_1) dt/2 + (a - a_1) dt^2/12.
// The jerk kernel applies the corrector to its particle as soon as a_1, j_1 are known,
// and (except in the last step) the next step's predictor, so a step is: coefficients
// and their derivatives at the predicted state, two reductions, the coefficient
// rescale and the jerk pass.  Steps 1 .. nsteps-1 are captured once into a hipGraph
// and replayed, the last step runs directly (as the leapfrog in etics_batched.hip).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>

#include "etics_device.hpp"
#include "etics_force_synth.hpp"
#include "etics_internal.hpp"

namespace etics {

// ---------------------------------------------------------------- coefficient prep
// Prepared coefficients with their time derivatives, Dual<S> [4K] per system, the same
// scaling as the force pass (Hernquist-Ostriker basis):
//   [0,K)   (su A, su dA/dt)   [K,2K)  (su B, su dB/dt)
//   [2K,3K) (sw A, sw dA/dt)   [3K,4K) (sw B, sw dB/dt)
template <typename S>
__global__ __launch_bounds__(256) void scf_jerk_prep_kernel(const double* __restrict__ A,
                                                           const double* __restrict__ B,
                                                           const double* __restrict__ Ad,
                                                           const double* __restrict__ Bd, int nmax,
                                                           int lmax, int nsys, Dual<S>* __restrict__ cf) {
  const int K = (nmax + 1) * (lmax + 1) * (lmax + 2) / 2;
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= int64_t(nsys) * K) return;
  const int sys = int(g / K);
  const int k = int(g - int64_t(sys) * K);
  const int L2 = (lmax + 1) * (lmax + 2) / 2;
  const int n = k / L2;
  const int lm = k - n * L2;
  int l = 0;
  while ((l + 1) * (l + 2) / 2 <= lm) ++l;
  const double al = basis_alpha(kBasisHO, l);
  const double s4 = -2.0 * sqrt(kPi);
  const double su = s4 * gegen_k(n, al);
  const double sw = n >= 1 ? s4 * 2.0 * al * 2.0 * gegen_k(n - 1, al + 1.0) : 0.0;
  Dual<S>* c = cf + size_t(sys) * 4 * K;
  c[k] = Dual<S>(S(su * A[g]), S(su * Ad[g]));
  c[K + k] = Dual<S>(S(su * B[g]), S(su * Bd[g]));
  c[2 * K + k] = Dual<S>(S(sw * A[g]), S(sw * Ad[g]));
  c[3 * K + k] = Dual<S>(S(sw * B[g]), S(sw * Bd[g]));
}

size_t jerk_prep_bytes(int nmax, int lmax, int prec) {
  return size_t(8) * coeff_count(nmax, lmax) * (prec == ETICS_FP64 ? 8 : 4);
}

// ---------------------------------------------------------------- jerk pass
// What the jerk pass does with a particle's a and j:
//   kOut:     write them to the output arrays;
//   kStart:   store them as the state's a, j and predict the first step;
//   kStep:    correct the state with them, store them, predict the next step;
//   kLast:    correct the state with them and store them.
enum HermiteMode { kOut = 0, kStart = 1, kStep = 2, kLast = 3 };

struct JerkArgs {
  const double *x, *y, *z, *vx, *vy, *vz;  // field points and their velocities
  int64_t n;
  const void* cf;                          // prepared Dual coefficients
  double *ax, *ay, *az, *jx, *jy, *jz;     // kOut: outputs; otherwise the state's a and j
  // Hermite state (modes other than kOut): positions and velocities corrected in place,
  // and the predicted ones (the field points of the next pass)
  double *sx, *sy, *sz, *svx, *svy, *svz;
  double *px, *py, *pz, *pvx, *pvy, *pvz;
  int K, nmax, lmax, mode;
  double dt;
};

// cf: the prepared coefficients through the constant address space ([4][K]) or in LDS
// (LdsPtr, QUAD: [K][4])
template <typename S, int LB, typename CP = ConstPtr<Dual<S>>, bool QUAD = false>
__device__ __forceinline__ void jerk_point(const JerkArgs& a, CP cf, int64_t i) {
  const Sph<Dual<S>> s = sph_dual<S, kBasisHO>(a.x[i], a.y[i], a.z[i], a.vx[i], a.vy[i], a.vz[i]);
  const ForceOut<Dual<S>> o =
      synth_point<Dual<S>, LB, true, kBasisHO, CP, QUAD>(s, cf, a.K, a.nmax, a.lmax);
  const double g[3] = {double(o.gx.v), double(o.gy.v), double(o.gz.v)};
  const double jk[3] = {double(o.gx.d), double(o.gy.d), double(o.gz.d)};
  double* A[3] = {a.ax, a.ay, a.az};
  double* J[3] = {a.jx, a.jy, a.jz};
  if (a.mode == kOut) {
    for (int c = 0; c < 3; ++c) {
      A[c][i] = g[c];
      J[c][i] = jk[c];
    }
    return;
  }
  double* X[3] = {a.sx, a.sy, a.sz};
  double* V[3] = {a.svx, a.svy, a.svz};
  double* P[3] = {a.px, a.py, a.pz};
  double* PV[3] = {a.pvx, a.pvy, a.pvz};
  const double dt = a.dt, h = 0.5 * dt, q = dt * dt / 12.0;
  for (int c = 0; c < 3; ++c) {
    double x = X[c][i], v = V[c][i];
    if (a.mode != kStart) {  // corrector with the step's starting a, j
      const double a0 = A[c][i], j0 = J[c][i];
      const double v1 = __builtin_fma(q, j0 - jk[c], __builtin_fma(h, a0 + g[c], v));
      x = __builtin_fma(q, a0 - g[c], __builtin_fma(h, v + v1, x));
      v = v1;
      X[c][i] = x;
      V[c][i] = v;
    }
    A[c][i] = g[c];
    J[c][i] = jk[c];
    if (a.mode != kLast) {  // predictor of the next step
      P[c][i] = __builtin_fma(dt * dt * dt / 6.0, jk[c], __builtin_fma(0.5 * dt * dt, g[c], __builtin_fma(dt, v, x)));
      PV[c][i] = __builtin_fma(0.5 * dt * dt, jk[c], __builtin_fma(dt, g[c], v));
    }
  }
}

template <typename S, int LB>
__global__ __launch_bounds__(256) void scf_jerk_kernel(const JerkArgs a) {
  const Dual<S>* __restrict__ cf = reinterpret_cast<const Dual<S>*>(a.cf);
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n;
       i += int64_t(gridDim.x) * blockDim.x)
    jerk_point<S, LB>(a, ConstPtr<Dual<S>>(cf), i);
}

// batched systems: `split` workgroups per unit of `unit` particles of one system, as the
// batched force kernel; the workgroup first copies its system's prepared coefficients to
// LDS as [K][4] and reads them as broadcast VGPR operands (a Dual coefficient would take
// two SGPRs)
template <typename S, int LB>
__global__ __launch_bounds__(256) void scf_jerk_batched_kernel(const JerkArgs a,
                                                               const int64_t* __restrict__ offsets,
                                                               const int* __restrict__ ustart,
                                                               const int* __restrict__ usys, int nsys,
                                                               int unit, int split) {
  extern __shared__ __align__(16) unsigned char jerk_lds[];
  const int u = blockIdx.x / split;
  const int part = blockIdx.x % split;
  if (u >= ustart[nsys]) return;
  const int sys = usys[u];
  int64_t b = offsets[sys], e = offsets[sys + 1];
  b = b < 0 ? 0 : (b > a.n ? a.n : b);
  e = e < b ? b : (e > a.n ? a.n : e);
  const int64_t kPart = (unit + split - 1) / split;
  const int64_t u0 = b + int64_t(u - ustart[sys]) * unit;
  const int64_t ue0 = u0 + unit < e ? u0 + unit : e;
  const int64_t ub = u0 + part * kPart < ue0 ? u0 + part * kPart : ue0;
  const int64_t ue = ub + kPart < ue0 ? ub + kPart : ue0;
  const Dual<S>* __restrict__ cf = reinterpret_cast<const Dual<S>*>(a.cf) + size_t(sys) * 4 * a.K;
  Dual<S>* lds_cf = reinterpret_cast<Dual<S>*>(jerk_lds);
  for (int i = threadIdx.x; i < 4 * a.K; i += blockDim.x) {
    const int which = i / a.K, idx = i - which * a.K;
    lds_cf[4 * idx + which] = cf[i];
  }
  __syncthreads();
  const LdsPtr<Dual<S>> src = (LdsPtr<Dual<S>>)(lds_cf);
  for (int64_t i = ub + threadIdx.x; i < ue; i += blockDim.x)
    jerk_point<S, LB, LdsPtr<Dual<S>>, true>(a, src, i);
}

namespace {

struct JerkBatch {
  const int64_t* offsets;
  const int* ustart;
  const int* usys;
  int nsys, unit, split;
};

template <typename S, int LBV>
void launch_jerk_kernel(const JerkArgs& a, int grid, const JerkBatch* bi, hipStream_t st) {
  if (bi) {
    // 4 K Dual values of LDS (at the largest cutoffs 79 KiB in FP32, 158 KiB in FP64;
    // failures surface at the launch)
    const size_t lds = size_t(4) * a.K * sizeof(Dual<S>);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(scf_jerk_batched_kernel<S, LBV>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    hipLaunchKernelGGL((scf_jerk_batched_kernel<S, LBV>), dim3(grid), dim3(256), lds, st, a, bi->offsets,
                       bi->ustart, bi->usys, bi->nsys, bi->unit, bi->split);
  } else
    hipLaunchKernelGGL((scf_jerk_kernel<S, LBV>), dim3(grid), dim3(256), 0, st, a);
}

template <typename S>
int launch_jerk_lb(const JerkArgs& a, int grid, const JerkBatch* bi, hipStream_t st) {
  const int lb = a.lmax <= 2 ? 2 : (a.lmax + 1) / 2 * 2;
  switch (lb) {
    case 2: launch_jerk_kernel<S, 2>(a, grid, bi, st); break;
    case 4: launch_jerk_kernel<S, 4>(a, grid, bi, st); break;
    case 6: launch_jerk_kernel<S, 6>(a, grid, bi, st); break;
    case 8: launch_jerk_kernel<S, 8>(a, grid, bi, st); break;
    case 10: launch_jerk_kernel<S, 10>(a, grid, bi, st); break;
    case 12: launch_jerk_kernel<S, 12>(a, grid, bi, st); break;
    case 14: launch_jerk_kernel<S, 14>(a, grid, bi, st); break;
    default:
      set_error("internal: no jerk kernel bucket");
      return ETICS_EUNSUPPORTED;
  }
  return hip_fail(hipGetLastError(), "scf_jerk_kernel launch");
}

int launch_jerk_prep(const double* A, const double* B, const double* Ad, const double* Bd, int nmax,
                     int lmax, int nsys, int prec, void* cf, hipStream_t st) {
  const int K = coeff_count(nmax, lmax);
  const int pb = int((int64_t(nsys) * K + 255) / 256);
  if (prec == ETICS_FP64)
    hipLaunchKernelGGL(scf_jerk_prep_kernel<double>, dim3(pb), dim3(256), 0, st, A, B, Ad, Bd, nmax, lmax,
                       nsys, reinterpret_cast<Dual<double>*>(cf));
  else
    hipLaunchKernelGGL(scf_jerk_prep_kernel<float>, dim3(pb), dim3(256), 0, st, A, B, Ad, Bd, nmax, lmax,
                       nsys, reinterpret_cast<Dual<float>*>(cf));
  return hip_fail(hipGetLastError(), "scf_jerk_prep_kernel launch");
}

int launch_jerk_any(const JerkArgs& a, int prec, int grid, const JerkBatch* bi, hipStream_t st) {
  return prec == ETICS_FP64 ? launch_jerk_lb<double>(a, grid, bi, st) : launch_jerk_lb<float>(a, grid, bi, st);
}

}  // namespace

int launch_scf_jerk(const double* x, const double* y, const double* z, const double* vx,
                    const double* vy, const double* vz, int64_t n, int nmax, int lmax,
                    const double* A, const double* B, const double* Ad, const double* Bd, int prec,
                    double* ax, double* ay, double* az, double* jx, double* jy, double* jz, void* ws,
                    hipStream_t st) {
  int rc = launch_jerk_prep(A, B, Ad, Bd, nmax, lmax, 1, prec, ws, st);
  if (rc || n == 0) return rc;
  JerkArgs a{};
  a.x = x;
  a.y = y;
  a.z = z;
  a.vx = vx;
  a.vy = vy;
  a.vz = vz;
  a.n = n;
  a.cf = ws;
  a.ax = ax;
  a.ay = ay;
  a.az = az;
  a.jx = jx;
  a.jy = jy;
  a.jz = jz;
  a.K = coeff_count(nmax, lmax);
  a.nmax = nmax;
  a.lmax = lmax;
  a.mode = kOut;
  int64_t grid = (n + 255) / 256;
  if (grid > 65536) grid = 65536;
  return launch_jerk_any(a, prec, int(grid), nullptr, st);
}

// ---------------------------------------------------------------- Hermite driver
namespace {

struct HermiteLayout {
  size_t off_ustart, off_usys, off_partials, off_prep, off_A, off_B, off_Ad, off_Bd, off_state, total;
  CoeffPlan plan;
  bool ok;
};

// workspace: unit tables, partial vectors (shared by both coefficient passes), the
// prepared Dual coefficients, A, B, dA/dt, dB/dt per system, and per particle a, j
// and the predicted position and velocity (12 doubles)
HermiteLayout hermite_layout(int64_t ntotal, int nsys, int nmax, int lmax, int prec) {
  HermiteLayout L{};
  L.ok = make_coeff_plan(ntotal, nmax, lmax, prec, &L.plan, kBasisHO, true);
  if (!L.ok) return L;
  const int K = coeff_count(nmax, lmax);
  const int mu = max_units(ntotal, nsys, L.plan.unit);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + (bytes > 0 ? bytes : 1), 256);
    return at;
  };
  const size_t nn = size_t(ntotal > 0 ? ntotal : 1);
  L.off_ustart = take(size_t(nsys + 1) * 4);
  L.off_usys = take(size_t(mu) * 4);
  L.off_partials = take(size_t(mu) * 2 * K * 8);
  L.off_prep = take(size_t(nsys) * jerk_prep_bytes(nmax, lmax, prec));
  L.off_A = take(size_t(nsys) * K * 8);
  L.off_B = take(size_t(nsys) * K * 8);
  L.off_Ad = take(size_t(nsys) * K * 8);
  L.off_Bd = take(size_t(nsys) * K * 8);
  L.off_state = take(12 * nn * 8);
  L.total = o;
  return L;
}

struct HermiteCall {
  double *x, *y, *z, *vx, *vy, *vz;
  const double* m;
  const int64_t* offsets;
  int nsys;
  int64_t ntotal;
  int nmax, lmax, prec;
  double dt;
  void* ws;
  size_t ws_bytes;
  int device;
  int plan[7];
};

bool same_call(const HermiteCall& a, const HermiteCall& b) {
  return a.x == b.x && a.y == b.y && a.z == b.z && a.vx == b.vx && a.vy == b.vy && a.vz == b.vz &&
         a.m == b.m && a.offsets == b.offsets && a.nsys == b.nsys && a.ntotal == b.ntotal &&
         a.nmax == b.nmax && a.lmax == b.lmax && a.prec == b.prec && a.dt == b.dt && a.ws == b.ws &&
         a.ws_bytes == b.ws_bytes && a.device == b.device && std::memcmp(a.plan, b.plan, sizeof a.plan) == 0;
}

// One jerk evaluation of every system: coefficients and their derivatives at the field
// points (fx.., fv..), reductions, rescale, then the jerk pass in `mode`.
int evaluate(const HermiteCall& c, const HermiteLayout& L, int mode, bool at_state, hipStream_t st) {
  char* base = reinterpret_cast<char*>(c.ws);
  const int* ustart = reinterpret_cast<const int*>(base + L.off_ustart);
  const int* usys = reinterpret_cast<const int*>(base + L.off_usys);
  double* A = reinterpret_cast<double*>(base + L.off_A);
  double* B = reinterpret_cast<double*>(base + L.off_B);
  double* Ad = reinterpret_cast<double*>(base + L.off_Ad);
  double* Bd = reinterpret_cast<double*>(base + L.off_Bd);
  double* s = reinterpret_cast<double*>(base + L.off_state);
  const int64_t n = c.ntotal;
  double *ax = s, *ay = s + n, *az = s + 2 * n, *jx = s + 3 * n, *jy = s + 4 * n, *jz = s + 5 * n;
  double *px = s + 6 * n, *py = s + 7 * n, *pz = s + 8 * n, *pvx = s + 9 * n, *pvy = s + 10 * n,
         *pvz = s + 11 * n;
  const double *fx = at_state ? c.x : px, *fy = at_state ? c.y : py, *fz = at_state ? c.z : pz;
  const double *fvx = at_state ? c.vx : pvx, *fvy = at_state ? c.vy : pvy, *fvz = at_state ? c.vz : pvz;
  const CoeffPlan& p = L.plan;
  int rc = launch_scf_coeffs_batched(p, fx, fy, fz, c.m, c.offsets, ustart, usys, c.nsys, n, A, B,
                                     base + L.off_partials, st);
  if (rc) return rc;
  rc = launch_scf_coeffs_dot_batched(p, fx, fy, fz, fvx, fvy, fvz, c.m, c.offsets, ustart, usys, c.nsys, n,
                                     Ad, Bd, base + L.off_partials, st);
  if (rc) return rc;
  rc = launch_jerk_prep(A, B, Ad, Bd, c.nmax, c.lmax, c.nsys, c.prec, base + L.off_prep, st);
  if (rc) return rc;
  JerkArgs a{};
  a.x = fx;
  a.y = fy;
  a.z = fz;
  a.vx = fvx;
  a.vy = fvy;
  a.vz = fvz;
  a.n = n;
  a.cf = base + L.off_prep;
  a.ax = ax;
  a.ay = ay;
  a.az = az;
  a.jx = jx;
  a.jy = jy;
  a.jz = jz;
  a.sx = c.x;
  a.sy = c.y;
  a.sz = c.z;
  a.svx = c.vx;
  a.svy = c.vy;
  a.svz = c.vz;
  a.px = px;
  a.py = py;
  a.pz = pz;
  a.pvx = pvx;
  a.pvy = pvy;
  a.pvz = pvz;
  a.K = coeff_count(c.nmax, c.lmax);
  a.nmax = c.nmax;
  a.lmax = c.lmax;
  a.mode = mode;
  a.dt = c.dt;
  const JerkBatch bi{c.offsets, ustart, usys, c.nsys, p.unit, p.split};
  return launch_jerk_any(a, c.prec, max_units(n, c.nsys, p.unit) * p.split, &bi, st);
}

struct GraphCache {
  bool valid = false;
  HermiteCall call{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t capture = nullptr;
};

std::mutex g_graph_mutex;
GraphCache g_graph;

void drop_graph(GraphCache& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  g.exec = nullptr;
  g.graph = nullptr;
  g.valid = false;
}

}  // namespace

size_t hermite_ws_bytes(int64_t ntotal, int nsys, int nmax, int lmax, int prec) {
  const HermiteLayout L = hermite_layout(ntotal, nsys, nmax, lmax, prec);
  return L.ok ? L.total : 0;
}

int run_hermite(double* x, double* y, double* z, double* vx, double* vy, double* vz,
                const double* m, const int64_t* offsets, int nsys, int64_t ntotal, int nmax, int lmax,
                int prec, double dt, int nsteps, int flags, void* ws, size_t ws_bytes, hipStream_t st) {
  HermiteCall c{x, y, z, vx, vy, vz, m, offsets, nsys, ntotal, nmax, lmax, prec, dt, ws, ws_bytes, 0, {}};
  struct HookPause {
    bool prev;
    HookPause() : prev(timing_hook().suspended) { timing_hook().suspended = true; }
    ~HookPause() { timing_hook().suspended = prev; }
  } pause;
  int rc = hip_fail(hipGetDevice(&c.device), "hipGetDevice");
  if (rc) return rc;
  const HermiteLayout L = hermite_layout(ntotal, nsys, nmax, lmax, prec);
  if (!L.ok) {
    set_error("no tile plan for these cutoffs");
    return ETICS_EUNSUPPORTED;
  }
  if (ws_bytes < L.total) {
    set_error("workspace too small: need " + std::to_string(L.total) + " bytes");
    return ETICS_EWORKSPACE;
  }
  const CoeffPlan& plan = L.plan;
  const int shape[7] = {plan.nw, plan.tp, plan.streams, plan.grid_mult, plan.unit, plan.split, plan.mfma ? 2 : 1};
  std::memcpy(c.plan, shape, sizeof shape);
  char* base = reinterpret_cast<char*>(ws);
  rc = launch_units(offsets, nsys, ntotal, plan.unit, reinterpret_cast<int*>(base + L.off_ustart),
                    reinterpret_cast<int*>(base + L.off_usys), st);
  if (rc || nsteps < 1) return rc;
  // a, j at the starting state, and the first prediction
  rc = evaluate(c, L, kStart, true, st);
  if (rc) return rc;
  if ((flags & ETICS_LEAPFROG_EAGER) || nsteps == 1) {
    for (int k = 1; k < nsteps; ++k) {
      rc = evaluate(c, L, kStep, false, st);
      if (rc) return rc;
    }
    return evaluate(c, L, kLast, false, st);
  }
  std::lock_guard<std::mutex> lock(g_graph_mutex);
  if (!g_graph.valid || !same_call(g_graph.call, c)) {
    drop_graph(g_graph);
    if (!g_graph.capture) {
      rc = hip_fail(hipStreamCreateWithFlags(&g_graph.capture, hipStreamNonBlocking),
                    "hipStreamCreateWithFlags");
      if (rc) return rc;
    }
    rc = hip_fail(hipStreamBeginCapture(g_graph.capture, hipStreamCaptureModeThreadLocal),
                  "hipStreamBeginCapture");
    if (rc) return rc;
    const int rs = evaluate(c, L, kStep, false, g_graph.capture);
    hipGraph_t graph = nullptr;
    rc = hip_fail(hipStreamEndCapture(g_graph.capture, &graph), "hipStreamEndCapture");
    if (rs) {
      if (graph) (void)hipGraphDestroy(graph);
      return rs;
    }
    if (rc) return rc;
    g_graph.graph = graph;
    rc = hip_fail(hipGraphInstantiate(&g_graph.exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    if (rc) {
      drop_graph(g_graph);
      return rc;
    }
    g_graph.call = c;
    g_graph.valid = true;
  }
  for (int k = 1; k < nsteps; ++k) {
    rc = hip_fail(hipGraphLaunch(g_graph.exec, st), "hipGraphLaunch");
    if (rc) return rc;
  }
  return evaluate(c, L, kLast, false, st);
}

}  // namespace etics
