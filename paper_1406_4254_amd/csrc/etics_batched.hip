// etics_batched.hip -- many independent systems in one launch, and the leapfrog.
//
// Systems are stored back to back (offsets[nsys+1], on the device).  The work is cut
// into units of at most `unit` particles of one system (the plan's; 4096 unless the
// tuner chose another): batched_units_kernel
// builds, on the device, the first unit of every system (ustart) and the system of
// every unit (usys).  The batched coefficient kernel gives each unit its own partial
// slot and the batched reduction sums a system's slots in unit order, so every
// system's coefficients are reproducible; the batched force kernel runs a few
// workgroups per unit, so each workgroup reads one system's coefficients.
//
// Leapfrog (the paper integrates with a leapfrog, Section 3.4), kick-drift-kick:
//   v += dt/2 a(x);  x += dt v;  a = a(x);  v += dt/2 a.
// The first opening kick and drift run as their own kernel; after that, the batched
// force kernel applies each particle's closing kick and, except in the last step, the
// next step's opening kick and drift as soon as its acceleration is known, so a step is
// coefficients, reduction, coefficient rescale and force.  Steps 1 .. nsteps-1 are
// captured once into a hipGraph and replayed (the capture is cached per argument set);
// the last step runs directly.  Every kick and drift is one FP64 fused multiply-add per
// component in both kernels, so eager and graph runs give identical bits.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>

#include "etics_internal.hpp"

namespace etics {

// ------------------------------------------------------------------ unit tables
__device__ __forceinline__ int64_t clamp64(int64_t v, int64_t lo, int64_t hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

__device__ __forceinline__ int system_units(const int64_t* off, int s, int64_t ntotal, int unit) {
  const int64_t b = clamp64(off[s], 0, ntotal);
  const int64_t e = clamp64(off[s + 1], b, ntotal);
  return int((e - b + unit - 1) / unit);
}

__global__ __launch_bounds__(1024) void batched_units_kernel(const int64_t* __restrict__ offsets,
                                                             int nsys, int64_t ntotal, int unit,
                                                             int* __restrict__ ustart,
                                                             int* __restrict__ usys) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int per = (nsys + 1023) / 1024;
  const int a = t * per < nsys ? t * per : nsys;
  const int b = a + per < nsys ? a + per : nsys;
  int cnt = 0;
  for (int s = a; s < b; ++s) cnt += system_units(offsets, s, ntotal, unit);
  part[t] = cnt;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {  // inclusive scan
    const int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = t > 0 ? part[t - 1] : 0;
  for (int s = a; s < b; ++s) {
    ustart[s] = run;
    const int nu = system_units(offsets, s, ntotal, unit);
    for (int j = 0; j < nu; ++j) usys[run + j] = s;
    run += nu;
  }
  if (t == 1023) ustart[nsys] = part[1023];
}

// ------------------------------------------------------------------ leapfrog
__global__ __launch_bounds__(256) void lf_kick_drift_kernel(double* __restrict__ x,
                                                            double* __restrict__ y,
                                                            double* __restrict__ z,
                                                            double* __restrict__ vx,
                                                            double* __restrict__ vy,
                                                            double* __restrict__ vz,
                                                            const double* __restrict__ ax,
                                                            const double* __restrict__ ay,
                                                            const double* __restrict__ az,
                                                            int64_t n, double hdt, double dt) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const double ux = __builtin_fma(hdt, ax[i], vx[i]);
    const double uy = __builtin_fma(hdt, ay[i], vy[i]);
    const double uz = __builtin_fma(hdt, az[i], vz[i]);
    vx[i] = ux;
    vy[i] = uy;
    vz[i] = uz;
    x[i] = __builtin_fma(dt, ux, x[i]);
    y[i] = __builtin_fma(dt, uy, y[i]);
    z[i] = __builtin_fma(dt, uz, z[i]);
  }
}

// ------------------------------------------------------------------ host side
BatchedLayout batched_layout(int64_t ntotal, int nsys, int nmax, int lmax, int prec) {
  BatchedLayout L{};
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
  L.off_prep = take(size_t(nsys) * 4 * K * (prec == ETICS_FP64 ? 8 : 4));
  L.off_A = take(size_t(nsys) * K * 8);
  L.off_B = take(size_t(nsys) * K * 8);
  L.off_acc = take(3 * nn * 8);
  L.total = o;
  L.max_units = mu;
  return L;
}

int launch_units(const int64_t* offsets, int nsys, int64_t ntotal, int unit, int* ustart, int* usys,
                 hipStream_t st) {
  hipLaunchKernelGGL(batched_units_kernel, dim3(1), dim3(1024), 0, st, offsets, nsys, ntotal, unit,
                     ustart, usys);
  return hip_fail(hipGetLastError(), "batched_units_kernel launch");
}

namespace {

struct LeapfrogCall {
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
  int plan[7];  // tile shape of the plan the step was captured with
};

bool same_call(const LeapfrogCall& a, const LeapfrogCall& b) {
  return a.x == b.x && a.y == b.y && a.z == b.z && a.vx == b.vx && a.vy == b.vy && a.vz == b.vz &&
         a.m == b.m && a.offsets == b.offsets && a.nsys == b.nsys && a.ntotal == b.ntotal &&
         a.nmax == b.nmax && a.lmax == b.lmax && a.prec == b.prec && a.dt == b.dt &&
         a.ws == b.ws && a.ws_bytes == b.ws_bytes && a.device == b.device &&
         std::memcmp(a.plan, b.plan, sizeof a.plan) == 0;
}

struct Parts {
  int* ustart;
  int* usys;
  void* partials;
  void* prep;
  double *A, *B, *ax, *ay, *az;
};

Parts parts_of(const LeapfrogCall& c, const BatchedLayout& L) {
  char* base = reinterpret_cast<char*>(c.ws);
  Parts p;
  p.ustart = reinterpret_cast<int*>(base + L.off_ustart);
  p.usys = reinterpret_cast<int*>(base + L.off_usys);
  p.partials = base + L.off_partials;
  p.prep = base + L.off_prep;
  p.A = reinterpret_cast<double*>(base + L.off_A);
  p.B = reinterpret_cast<double*>(base + L.off_B);
  p.ax = reinterpret_cast<double*>(base + L.off_acc);
  p.ay = p.ax + c.ntotal;
  p.az = p.ay + c.ntotal;
  return p;
}

// a(x) for every system: coefficients, reduction, rescale, force
int accelerations(const LeapfrogCall& c, const CoeffPlan& plan, const Parts& p, hipStream_t st) {
  int rc = launch_scf_coeffs_batched(plan, c.x, c.y, c.z, c.m, c.offsets, p.ustart, p.usys, c.nsys,
                                     c.ntotal, p.A, p.B, p.partials, st);
  if (rc) return rc;
  return launch_scf_force_batched(plan, c.x, c.y, c.z, c.offsets, p.ustart, p.usys, c.nsys, c.ntotal,
                                  p.A, p.B, ETICS_ACC, nullptr, p.ax, p.ay, p.az, p.prep, st);
}

// the opening kick and drift of the first step, from the accelerations in p.ax..p.az
int first_kick_drift(const LeapfrogCall& c, const Parts& p, hipStream_t st) {
  int64_t grid = (c.ntotal + 255) / 256;
  if (grid > 8192) grid = 8192;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(lf_kick_drift_kernel, dim3(int(grid)), dim3(256), 0, st, c.x, c.y, c.z, c.vx,
                     c.vy, c.vz, p.ax, p.ay, p.az, c.ntotal, 0.5 * c.dt, c.dt);
  return hip_fail(hipGetLastError(), "lf_kick_drift_kernel launch");
}

// The rest of a step once x has drifted: a(x) from this step's coefficients, the closing
// kick and, unless it is the last step (last = true), the next step's opening kick and
// drift, all in the force kernel (KDK: v += dt/2 a; x += dt v; a = a(x); v += dt/2 a).
int step_tail(const LeapfrogCall& c, const CoeffPlan& plan, const Parts& p, bool last,
              hipStream_t st) {
  int rc = launch_scf_coeffs_batched(plan, c.x, c.y, c.z, c.m, c.offsets, p.ustart, p.usys, c.nsys,
                                     c.ntotal, p.A, p.B, p.partials, st);
  if (rc) return rc;
  LfUpdate lf{c.x, c.y, c.z, c.vx, c.vy, c.vz, 0.5 * c.dt, c.dt, last ? 1 : 2};
  return launch_scf_force_batched(plan, c.x, c.y, c.z, c.offsets, p.ustart, p.usys, c.nsys,
                                  c.ntotal, p.A, p.B, ETICS_ACC, nullptr, p.ax, p.ay, p.az, p.prep,
                                  st, &lf);
}

struct GraphCache {
  bool valid = false;
  LeapfrogCall call{};
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

int run_leapfrog(double* x, double* y, double* z, double* vx, double* vy, double* vz,
                 const double* m, const int64_t* offsets, int nsys, int64_t ntotal, int nmax,
                 int lmax, int prec, double dt, int nsteps, int flags, void* ws, size_t ws_bytes,
                 hipStream_t st) {
  LeapfrogCall c{x, y, z, vx, vy, vz, m, offsets, nsys, ntotal, nmax, lmax, prec, dt, ws, ws_bytes, 0, {}};
  // timing events are not recorded inside the steps (they would be captured too)
  struct HookPause {
    bool prev;
    HookPause() : prev(timing_hook().suspended) { timing_hook().suspended = true; }
    ~HookPause() { timing_hook().suspended = prev; }
  } pause;
  int rc = hip_fail(hipGetDevice(&c.device), "hipGetDevice");
  if (rc) return rc;
  const BatchedLayout L = batched_layout(ntotal, nsys, nmax, lmax, prec);
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
  const Parts p = parts_of(c, L);
  rc = launch_units(offsets, nsys, ntotal, plan.unit, p.ustart, p.usys, st);
  if (rc) return rc;
  if (nsteps < 1) return ETICS_OK;
  rc = accelerations(c, plan, p, st);  // a(x) at the start of the first step
  if (rc) return rc;
  rc = first_kick_drift(c, p, st);
  if (rc) return rc;
  // steps 1 .. nsteps-1 end with the next step's kick and drift; the last one does not
  if ((flags & ETICS_LEAPFROG_EAGER) || nsteps == 1) {
    for (int k = 1; k < nsteps; ++k) {
      rc = step_tail(c, plan, p, false, st);
      if (rc) return rc;
    }
    return step_tail(c, plan, p, true, st);
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
    const int rs = step_tail(c, plan, p, false, g_graph.capture);
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
  return step_tail(c, plan, p, true, st);
}

}  // namespace etics
