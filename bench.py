#!/usr/bin/env python3
"""Benchmark: SCF force calculation throughput on one MI355X.

One step = one full SCF force calculation of the workload through the C-ABI:
etics_scf_coeffs (coefficients summed over all particles) followed by
etics_scf_force (potential and acceleration of every particle), inputs and outputs
resident in HBM.  The timed steps issue the two calls eagerly with nothing else in
the timed region; the same steps are then run again with events around the calls and
their main kernels (stage and kernel durations), and replayed from a captured hipGraph
(stages_ms.graph_ms_per_step).  The headline workload is N = 10^6 particles of a triaxial
Hernquist model (x,y,z scaled 1 : 0.8 : 0.6, seed 2) at (nmax, lmax) = (10, 10) in
the mixed mode (FP32 basis and synthesis, FP64 coefficient reduction); the plain
FP64 path is timed beside it.  Accuracy of both is measured against the FP64 CPU
oracle, which is also timed on the host as the CPU baseline.

The main kernel of each call is bracketed by HIP events through
etics_set_timing_events, on the stream the kernels run on; the roofline figure of the
dominant kernel uses those durations.  Also timed (reported under "extras", not the
headline): the MEX force of N = 10^6 (Plummer + Hernquist mixture, lmax = 10) and a
hipGraph leapfrog step of 256 independent systems (about 5.5e6 particles, (8, 6)).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_FP64_VECTOR_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

CSRC = os.path.join(ROOT, "paper_1406_4254_amd", "csrc")
KERNEL_SOURCES = {
    "coeff": ["etics_coeff.hip", "etics_coeff_wg.hpp", "etics_device.hpp", "etics_tables.hpp"],
    "force": ["etics_force.hip", "etics_force_synth.hpp", "etics_device.hpp", "etics_tables.hpp"],
}


def coeff_count(nmax, lmax):
    return (nmax + 1) * (lmax + 1) * (lmax + 2) // 2


def flops_per_particle(nmax, lmax):
    """Algorithmic FP operations per particle of one force calculation (FMA = 2).

    C = (nmax+1)(lmax+1)^2 real coefficients.
      coefficients: C products accumulated (2C), Gegenbauer values (3 per (n,l)),
                    Legendre values and angular weights (4 per (l,m) slot)
      force:        2C accumulations of the radial sums (4C), two Gegenbauer
                    families (5 per (n,l)), angular synthesis (8 per (l,m) slot)
    """
    C = (nmax + 1) * (lmax + 1) ** 2
    L = (lmax + 1) ** 2
    R = (nmax + 1) * (lmax + 1)
    coef = 2 * C + 4 * L + 3 * R
    force = 4 * C + 8 * L + 5 * R
    return coef, force


def source_digest(which):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[which]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(which, workload):
    """HBM bytes per launch from the committed counter summary of this kernel and
    workload, or None if there is none or the kernel's sources changed since."""
    path = os.path.join(ROOT, "profiles", f"traffic_{which}_kernel_{workload}.md")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        m = re.search(r"^traffic_json:\s*(\{.*\})\s*$", fh.read(), re.M)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("source_sha256") != source_digest(which):
        return None
    return rec["hbm_bytes_per_launch"]


def measured_counters(which, workload, kernel):
    """Per-particle VALU figures (rocprofv3 SQ counters) from the committed counter
    summary of this kernel and workload, or None if there is none, it covers another
    kernel, or the kernel's sources changed since."""
    prec = "mixed" if kernel.startswith(f"scf_{which}_kernel<float") else "fp64"
    path = os.path.join(ROOT, "profiles", f"counters_{which}_kernel_{prec}_{workload}.md")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        m = re.search(r"^counters_json:\s*(\{.*\})\s*$", fh.read(), re.M)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("source_sha256") != source_digest(which) or rec.get("kernel") != kernel:
        return None
    return rec


def cpu_model():
    """CPU model name of the host (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def copy_calibration(torch, nbytes=256 << 20, reps=3):
    """Plain device-to-device copies of a known size; a counter run over this program
    reads them to scale the HBM byte counters."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


class KernelTimer:
    """Pairs of events recorded around the main kernel of one call each."""

    def __init__(self, torch, etics, count, stream):
        self.etics = etics
        self.pairs = []
        for _ in range(count):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)  # creates the device events
            b.record(stream)
            self.pairs.append((a, b))
        self.k = 0

    def arm(self):
        a, b = self.pairs[self.k]
        self.k += 1
        self.etics.etics_set_timing_events(a, b)

    def mean_ms(self):
        self.etics.etics_set_timing_events(None, None)
        return sum(a.elapsed_time(b) for a, b in self.pairs[:self.k]) / max(self.k, 1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--nmax", type=int, default=10)
    ap.add_argument("--lmax", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--extras", default="mex,batched,hermite,potonly,cb,direct",
                    help="comma list of the extra workloads to time (mex, batched, hermite, potonly, cb, direct)")
    ap.add_argument("--lf-steps", type=int, default=100, help="leapfrog steps of the batched extra")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run plain 256 MiB device copies (for scaling byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "etics runs on one GPU; runs on several GPUs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1406_4254_amd import accuracy, etics, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.copy_calibration:
        copy_calibration(torch)

    nmax, lmax, n = args.nmax, args.lmax, args.n
    headline = (n, nmax, lmax) == (1_000_000, 10, 10)
    workload = "scf_triaxial_hernquist_n1e6_n10_l10" if headline else f"scf_triaxial_hernquist_n{n}_n{nmax}_l{lmax}"
    p = workloads.triaxial_hernquist(n, seed=2)
    x, y, z, m = (torch.from_numpy(a).cuda() for a in (p.x, p.y, p.z, p.m))
    K = coeff_count(nmax, lmax)

    def run_mode(prec, steps, warmup):
        A = torch.empty(K, dtype=torch.float64, device="cuda")
        B = torch.empty_like(A)
        pot, ax, ay, az = (torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(4))
        ws = etics.workspace(etics.etics_scf_workspace_size(n, nmax, lmax, prec), "cuda")
        kc = KernelTimer(torch, etics, steps, stream)
        kf = KernelTimer(torch, etics, steps, stream)

        def step(ev=None):
            if ev is not None:
                ev[0].record(stream)
                kc.arm()
            etics.etics_scf_coeffs(x, y, z, m, nmax, lmax, prec, A, B, ws, stream)
            if ev is not None:
                ev[1].record(stream)
                kf.arm()
            etics.etics_scf_force(x, y, z, nmax, lmax, A, B, prec, etics.ETICS_POT_ACC, pot, ax, ay, az,
                                  ws, stream)
            if ev is not None:
                ev[2].record(stream)
                etics.etics_set_timing_events(None, None)

        for _ in range(warmup):
            step()
        # the headline: eager calls, nothing else in the timed region
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        eager_wall = time.perf_counter() - t0
        # the same calls with events around them and around their main kernels
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        torch.cuda.synchronize()
        for k in range(steps):
            step(evs[k])
        torch.cuda.synchronize()
        res = {
            "wall_s": eager_wall,
            "coeff_call_ms": float(np.mean([e[0].elapsed_time(e[1]) for e in evs])),
            "force_call_ms": float(np.mean([e[1].elapsed_time(e[2]) for e in evs])),
            "step_ms_sd": float(np.std([e[0].elapsed_time(e[2]) for e in evs])),
            "coeff_kernel_ms": kc.mean_ms(),
            "force_kernel_ms": kf.mean_ms(),
        }
        # the same step captured once into a graph (the calls allocate and synchronise
        # nothing, so they can be captured) and replayed
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            etics.etics_scf_coeffs(x, y, z, m, nmax, lmax, prec, A, B, ws)
            etics.etics_scf_force(x, y, z, nmax, lmax, A, B, prec, etics.ETICS_POT_ACC, pot, ax, ay, az, ws)
        for _ in range(warmup):
            g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.replay()
        torch.cuda.synchronize()
        res["graph_ms_per_step"] = (time.perf_counter() - t0) / steps * 1e3
        out = [t.cpu().numpy() for t in (A, B, pot, ax, ay, az)]
        return res, out

    mixed, res = run_mode(etics.ETICS_MIXED_FP64ACC, args.steps, args.warmup)
    ms_per_step = mixed["wall_s"] / args.steps * 1e3
    value = n / (mixed["wall_s"] / args.steps)

    fp64 = None
    if not args.no_fp64:
        r64, res64 = run_mode(etics.ETICS_FP64, args.steps, args.warmup)
        fp64 = {"value": n / (r64["wall_s"] / args.steps), "ms_per_step": r64["wall_s"] / args.steps * 1e3,
                **{k: v for k, v in r64.items() if k != "wall_s"}}

    fc, ff = flops_per_particle(nmax, lmax)
    # kernel names as the profiler prints them (template arguments: compute type, lmax
    # bucket, radial orders per register block, angular slots per block, accumulation
    # mode, wavefronts per particle group, radial basis)
    plan = etics.etics_plan_info(n, nmax, lmax, etics.ETICS_MIXED_FP64ACC)
    lb_force = 2 if lmax <= 2 else (lmax + 1) // 2 * 2
    lb_coeff = 2 if lmax <= 2 else (6 if lmax <= 6 else (10 if lmax <= 10 else 14))
    nb = 9 if nmax + 1 <= 9 else (11 if nmax + 1 <= 11 else 12)
    coeff_name = (f"scf_coeff_kernel<float, {lb_coeff}, {nb}, 4, 0, {plan['nw']}, 0, false, "
                  f"{'true' if plan['phase2'] == 2 else 'false'}>")
    kernels = {
        "force": (mixed["force_kernel_ms"], ff, f"scf_force_kernel<float, {lb_force}, true, 0>"),
        "coeff": (mixed["coeff_kernel_ms"], fc, coeff_name),
    }
    dom = max(kernels, key=lambda k: kernels[k][0])
    dom_ms, dom_fpp, dom_name = kernels[dom]
    achieved = dom_fpp * n / (dom_ms * 1e-3) / 1e12
    traffic = measured_traffic(dom, workload)
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": traffic,
                "kernel": dom_name, "kernel_ms": dom_ms, "flops_per_particle": dom_fpp,
                "particles_per_launch": n,
                "frac_of_nonpacked_fp32": achieved / (PEAK_FP32_VECTOR_TFLOPS / 2)}
    if traffic is not None:
        roofline["traffic_frac_of_hbm_peak"] = traffic / (dom_ms * 1e-3) / 1e9 / PEAK_HBM_GBS
    # executed VALU work from the committed SQ counter summary, over this run's kernel time
    ctr = measured_counters(dom, workload, dom_name)
    if ctr is not None:
        ex = ctr["executed_fp32_flop_per_unit"] * n / (dom_ms * 1e-3) / 1e12
        roofline["counters"] = {
            "valu_instr_per_particle": ctr["valu_instr_per_unit"],
            "valu_issue_busy": ctr["valu_issue_busy"],
            "executed_fp32_flop_per_particle": ctr["executed_fp32_flop_per_unit"],
            "executed_tflops": ex, "executed_frac": ex / PEAK_FP32_VECTOR_TFLOPS,
            "source": "profiles/counters_*_kernel_mixed_" + workload + ".md (SQ_INSTS_VALU, "
                      "SQ_ACTIVE_INST_VALU, SQ_INSTS_VALU_FLOPS_FP32, GRBM_GUI_ACTIVE)"}
    other = "coeff" if dom == "force" else "force"
    o_ms, o_fpp, o_name = kernels[other]
    step_tflops = (fc + ff) * n / (ms_per_step * 1e-3) / 1e12

    out = {
        "metric": "SCF particles/s (force calc) at N=1e6,nmax=10,lmax=10; mixed vs FP64 GPU",
        "value": value,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "n": n, "nmax": nmax, "lmax": lmax, "seed": 2,
                   "axes": [1.0, 0.8, 0.6], "precision": "mixed: fp32 basis/synthesis, fp64 reduction",
                   "execution": "etics_scf_coeffs + etics_scf_force issued eagerly per step "
                                "(graph replay: stages_ms.graph_ms_per_step)",
                   "coeff_plan": plan},
        "stages_ms": {k: v for k, v in mixed.items() if k != "wall_s"},
        "step_tflops": step_tflops,
        "roofline": roofline,
        "other_kernel": {"kernel": o_name, "kernel_ms": o_ms, "achieved": o_fpp * n / (o_ms * 1e-3) / 1e12,
                         "unit": "TFLOP/s", "flops_per_particle": o_fpp},
    }
    if fp64:
        out["fp64"] = fp64
        out["speedup_vs_fp64"] = value / fp64["value"]

    if not args.no_extras:
        out["extras"] = extras(torch, np, etics, workloads, stream, set(args.extras.split(",")), args.lf_steps)

    if not args.no_cpu_baseline:
        import oracle
        # the oracle as it stands, all host threads, on the full workload: one force calculation
        t0 = time.perf_counter()
        rA, rB = oracle.scf_coeffs(p.x, p.y, p.z, p.m, nmax, lmax)
        rp, rx, ry, rz = oracle.scf_force(p.x, p.y, p.z, nmax, lmax, rA, rB)
        cpu_s = time.perf_counter() - t0
        # one thread on a bounded sample of the same workload
        ns = 200_000
        nthr = oracle.num_threads()
        oracle.set_threads(1)
        t1 = time.perf_counter()
        sA, sB = oracle.scf_coeffs(p.x[:ns], p.y[:ns], p.z[:ns], p.m[:ns], nmax, lmax)
        oracle.scf_force(p.x[:ns], p.y[:ns], p.z[:ns], nmax, lmax, sA, sB)
        one_s = time.perf_counter() - t1
        oracle.set_threads(nthr)
        out["cpu_baseline"] = {"value": n / cpu_s, "unit": "particles/s", "cores": nthr,
                               "kind": "oracle",
                               "sample": f"the full workload (N={n}, ({nmax},{lmax})), one force calculation "
                                         f"(coefficients then potential and acceleration), {cpu_s:.2f} s",
                               "cpu_model": cpu_model(),
                               "one_thread": {"value": ns / one_s, "unit": "particles/s", "cores": 1,
                                              "sample": f"the first {ns} particles of the workload, one force "
                                                        f"calculation, {one_s:.2f} s"}}
        A, B, pot, ax, ay, az = res
        ce = accuracy.coeff_errors(A, B, rA, rB)
        fe = accuracy.summarize(accuracy.force_rel_err(ax, ay, az, rx, ry, rz))
        pe = accuracy.summarize(accuracy.pot_rel_err(pot, rp))
        out["accuracy_vs_oracle"] = {"mixed": {"coeff_norm_rel": ce["norm_rel"], "force": fe, "pot": pe}}
        if fp64:
            A, B, pot, ax, ay, az = res64
            out["accuracy_vs_oracle"]["fp64"] = {
                "coeff_norm_rel": accuracy.coeff_errors(A, B, rA, rB)["norm_rel"],
                "force": accuracy.summarize(accuracy.force_rel_err(ax, ay, az, rx, ry, rz)),
                "pot": accuracy.summarize(accuracy.pot_rel_err(pot, rp))}
    print(json.dumps(out), flush=True)


def extras(torch, np, etics, workloads, stream, which, lf_steps, reps=10):
    """MEX force (N = 10^6, lmax = 10), the batched hipGraph leapfrog step, the
    potential-only SCF step and the FP64 direct summation of the accuracy study
    (N = 10^5); `which` selects among them."""
    ex = {}
    if "mex" in which:
        mex_extra(torch, np, etics, workloads, stream, reps, ex)
    if "batched" in which:
        batched_extra(torch, np, etics, workloads, stream, lf_steps, ex)
    if "hermite" in which:
        hermite_extra(torch, np, etics, workloads, stream, ex)
    if "potonly" in which:
        potonly_extra(torch, np, etics, workloads, stream, reps, ex)
    if "cb" in which:
        cb_extra(torch, np, etics, workloads, stream, reps, ex)
    if "direct" in which:
        direct_extra(torch, np, etics, workloads, stream, ex)
    return ex


def mex_extra(torch, np, etics, workloads, stream, reps, ex):
    p = workloads.make_config(4)
    n = p.x.shape[0]
    x, y, z, m = (torch.from_numpy(a).cuda() for a in (p.x, p.y, p.z, p.m))
    for name, prec in (("mixed", etics.ETICS_MIXED_FP64ACC), ("fp64", etics.ETICS_FP64)):
        pot, ax, ay, az = (torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(4))
        ws = etics.workspace(etics.etics_mex_workspace_size(n, 10, prec), "cuda")
        call = lambda: etics.etics_mex_force(x, y, z, m, 10, prec, etics.ETICS_POT_ACC, pot, ax, ay, az, ws,
                                             stream)
        call()
        kt = KernelTimer(torch, etics, reps, stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            kt.arm()
            call()
        e1.record(stream)
        etics.etics_set_timing_events(None, None)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        # algorithmic bytes: x, y, z, m in and pot, a out (64 B) plus 8 radix passes over
        # an 8-byte key and a 4-byte index, read and written (8 x 24 B)
        mex_bytes = n * (64 + 8 * 24)
        ex[f"mex_{name}"] = {"workload": "mex_plummer_hernquist_n1e6_l10", "ms_per_call": ms,
                             "particles_per_s": n / (ms * 1e-3), "synthesis_kernel_ms": kt.mean_ms(),
                             "algorithmic_bytes": mex_bytes,
                             "achieved_GBs": mex_bytes / (ms * 1e-3) / 1e9,
                             "frac_of_hbm_peak": mex_bytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS}


def batched_extra(torch, np, etics, workloads, stream, nsteps, ex):
    q = workloads.make_config(5)
    nt = q.x.shape[0]
    st = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (q.x, q.y, q.z, q.vx, q.vy, q.vz, q.m)]
    ics = [t.clone() for t in st[:6]]
    off = torch.from_numpy(q.offsets).cuda()
    prec = etics.ETICS_MIXED_FP64ACC
    ws = etics.workspace(etics.etics_batched_workspace_size(nt, 256, 8, 6, prec), "cuda")

    def energies():
        """Per-system energy, kinetic plus half the mass-weighted SCF potential (FP64 on the GPU)."""
        A, B = etics.etics_scf_coeffs_batched(*st[:3], st[6], off, 8, 6, etics.ETICS_FP64)
        pot = etics.etics_scf_force_batched(*st[:3], off, 8, 6, A, B, etics.ETICS_FP64, etics.ETICS_POT)[0]
        v2 = st[3] * st[3] + st[4] * st[4] + st[5] * st[5]
        e = (0.5 * st[6] * (v2 + pot)).cpu().numpy()
        return np.add.reduceat(e, q.offsets[:-1])

    e_start = energies()
    etics.etics_leapfrog_scf_batched(*st, off, 8, 6, 0.01, 2, prec, 0, ws, stream)  # capture + warm
    for t, t0 in zip(st[:6], ics):  # back to the initial conditions (same buffers: the graph stays valid)
        t.copy_(t0)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    etics.etics_leapfrog_scf_batched(*st, off, 8, 6, 0.01, nsteps, prec, 0, ws, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    drift = np.abs(energies() / e_start - 1.0)
    # one call = one extra force calculation at the start + nsteps graph replays
    fc, ff = flops_per_particle(8, 6)
    step_ms = ms / (nsteps + 1)
    ex["leapfrog_batched_mixed"] = {"workload": "batched_256_spheres_n8_l6", "particles": nt, "nsteps": nsteps,
                                    "ms_per_call": ms, "ms_per_step": step_ms,
                                    "particle_steps_per_s": nt * (nsteps + 1) / (ms * 1e-3),
                                    "step_tflops": (fc + ff) * nt / (step_ms * 1e-3) / 1e12,
                                    "plan": etics.etics_plan_info(nt, 8, 6, prec, batched=True),
                                    "energy_drift_rel": {"median": float(np.median(drift)),
                                                         "max": float(np.max(drift)),
                                                         "what": f"|E(t)/E(0) - 1| per system after the "
                                                                 f"{nsteps} mixed-precision steps of 0.01, E = "
                                                                 f"kinetic + half the mass-weighted SCF potential"}}
    del st, ics, off, ws


def hermite_extra(torch, np, etics, workloads, stream, ex, nsteps=20):
    """The batched fourth-order Hermite integrator on the 256-system workload (mixed):
    a step is the coefficients and their time derivatives at the predicted state, the
    jerk pass and the corrector, replayed from a captured graph."""
    q = workloads.make_config(5)
    nt = q.x.shape[0]
    st = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (q.x, q.y, q.z, q.vx, q.vy, q.vz, q.m)]
    ics = [t.clone() for t in st[:6]]
    off = torch.from_numpy(q.offsets).cuda()
    prec = etics.ETICS_MIXED_FP64ACC
    ws = etics.workspace(etics.etics_hermite_workspace_size(nt, 256, 8, 6, prec), "cuda")

    def energies():
        A, B = etics.etics_scf_coeffs_batched(*st[:3], st[6], off, 8, 6, etics.ETICS_FP64)
        pot = etics.etics_scf_force_batched(*st[:3], off, 8, 6, A, B, etics.ETICS_FP64, etics.ETICS_POT)[0]
        v2 = st[3] * st[3] + st[4] * st[4] + st[5] * st[5]
        return np.add.reduceat((0.5 * st[6] * (v2 + pot)).cpu().numpy(), q.offsets[:-1])

    e_start = energies()
    etics.etics_hermite_scf_batched(*st, off, 8, 6, 0.01, 2, prec, 0, ws, stream)  # capture + warm
    for t, t0 in zip(st[:6], ics):
        t.copy_(t0)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    etics.etics_hermite_scf_batched(*st, off, 8, 6, 0.01, nsteps, prec, 0, ws, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    drift = np.abs(energies() / e_start - 1.0)
    step_ms = ms / (nsteps + 1)  # one extra evaluation at the start
    ex["hermite_batched_mixed"] = {"workload": "batched_256_spheres_n8_l6", "particles": nt, "nsteps": nsteps,
                                   "ms_per_call": ms, "ms_per_step": step_ms,
                                   "particle_steps_per_s": nt * (nsteps + 1) / (ms * 1e-3),
                                   "energy_drift_rel": {"median": float(np.median(drift)),
                                                        "max": float(np.max(drift)),
                                                        "what": f"|E(t)/E(0) - 1| per system after {nsteps} "
                                                                f"mixed-precision Hermite steps of 0.01"}}
    del st, ics, off, ws


def cb_extra(torch, np, etics, workloads, stream, reps, ex):
    """One SCF force calculation in the Clutton-Brock basis (Section 2.5) at the headline
    size and cutoffs, on a triaxial Plummer model (mixed)."""
    p = workloads.triaxial_plummer(1_000_000, 2)
    n = p.n
    x, y, z, m = (torch.from_numpy(a).cuda() for a in (p.x, p.y, p.z, p.m))
    prec, cb = etics.ETICS_MIXED_FP64ACC, etics.ETICS_BASIS_CB
    K = etics.etics_coeff_count(10, 10)
    A = torch.empty(K, dtype=torch.float64, device="cuda")
    B = torch.empty_like(A)
    outs = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(4)]
    ws = etics.workspace(etics.etics_scf_workspace_size(n, 10, 10, prec), "cuda")

    def step():
        etics.etics_scf_coeffs_basis(x, y, z, m, 10, 10, prec, cb, A, B, ws, stream)
        etics.etics_scf_force_basis(x, y, z, 10, 10, A, B, prec, cb, etics.ETICS_POT_ACC, *outs, ws, stream)

    step()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ex["scf_clutton_brock_mixed"] = {"workload": "scf_triaxial_plummer_n1e6_n10_l10_cb", "ms_per_step": ms,
                                     "particles_per_s": n / (ms * 1e-3)}
    del x, y, z, m, A, B, outs, ws


def potonly_extra(torch, np, etics, workloads, stream, reps, ex):
    # potential only (no acceleration): the SCF step of the headline workload with the
    # force call asked for ETICS_POT, which runs the kernel without the derivative sums
    p2 = workloads.make_config(2)
    n2 = p2.n
    x, y, z, m = (torch.from_numpy(a).cuda() for a in (p2.x, p2.y, p2.z, p2.m))
    prec = etics.ETICS_MIXED_FP64ACC
    K = etics.etics_coeff_count(10, 10)
    A = torch.empty(K, dtype=torch.float64, device="cuda")
    B = torch.empty_like(A)
    pot = torch.empty(n2, dtype=torch.float64, device="cuda")
    ws = etics.workspace(etics.etics_scf_workspace_size(n2, 10, 10, prec), "cuda")

    def pstep():
        etics.etics_scf_coeffs(x, y, z, m, 10, 10, prec, A, B, ws, stream)
        etics.etics_scf_force(x, y, z, 10, 10, A, B, prec, etics.ETICS_POT, pot, None, None, None, ws, stream)

    pstep()
    kt = KernelTimer(torch, etics, reps, stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        etics.etics_scf_coeffs(x, y, z, m, 10, 10, prec, A, B, ws, stream)
        kt.arm()
        etics.etics_scf_force(x, y, z, 10, 10, A, B, prec, etics.ETICS_POT, pot, None, None, None, ws, stream)
        etics.etics_set_timing_events(None, None)  # the next coefficient call is not timed
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ex["scf_potential_only_mixed"] = {"workload": "scf_triaxial_hernquist_n1e6_n10_l10", "ms_per_step": ms,
                                      "particles_per_s": n2 / (ms * 1e-3), "force_kernel_ms": kt.mean_ms()}
    del x, y, z, m, A, B, pot, ws


def direct_extra(torch, np, etics, workloads, stream, ex):
    # FP64 direct summation (the N-body reference of the accuracy study), N = 10^5
    # Ferrers model2: 19 flops per pair (3 differences, 5 for r^2, 1 reciprocal square
    # root, 3 for m/r and m/r^3, 1 for the potential, 6 for the acceleration)
    pd = workloads.ferrers1(100_000, 41, workloads.FERRERS_MODELS["model2"])
    nd = pd.n
    x, y, z, m = (torch.from_numpy(a).cuda() for a in (pd.x, pd.y, pd.z, pd.m))
    outs = [torch.empty(nd, dtype=torch.float64, device="cuda") for _ in range(4)]
    call = lambda: etics.etics_direct_force(x, y, z, m, etics.ETICS_POT_ACC, *outs, stream=stream)
    call()
    dreps = 3
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(dreps):
        call()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / dreps
    pairs = float(nd) * nd
    tf = 19.0 * pairs / (ms * 1e-3) / 1e12
    ex["direct_fp64"] = {"workload": "direct_ferrers_model2_n1e5", "ms_per_call": ms,
                         "pairs_per_s": pairs / (ms * 1e-3), "flops_per_pair": 19,
                         "achieved_tflops": tf, "frac_of_fp64_peak": tf / PEAK_FP64_VECTOR_TFLOPS}


if __name__ == "__main__":
    main()
