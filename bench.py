#!/usr/bin/env python3
"""Benchmark: SCF force calculation throughput on one MI355X.

One step = one full SCF force calculation of the workload through the C-ABI:
etics_scf_coeffs (coefficients summed over all particles) followed by
etics_scf_force (potential and acceleration of every particle), inputs and outputs
resident in HBM.  The headline workload is N = 10^6 particles of a triaxial
Hernquist model (x,y,z scaled 1 : 0.8 : 0.6, seed 2) at (nmax, lmax) = (10, 10) in
the mixed mode (FP32 basis and synthesis, FP64 coefficient reduction); the plain
FP64 path is timed beside it.  Accuracy of both is measured against the FP64 CPU
oracle, which is also timed on the host as the CPU baseline.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_FP64_VECTOR_TFLOPS = 78.6


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
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1406_4254_amd import accuracy, etics, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    nmax, lmax, n = args.nmax, args.lmax, args.n
    p = workloads.triaxial_hernquist(n, seed=2)
    dev = [torch.from_numpy(a).cuda() for a in (p.x, p.y, p.z, p.m)]
    x, y, z, m = dev
    K = coeff_count(nmax, lmax)
    stream = torch.cuda.current_stream()

    def run_mode(prec, steps, warmup):
        A = torch.empty(K, dtype=torch.float64, device="cuda")
        B = torch.empty_like(A)
        pot, ax, ay, az = (torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(4))
        ws = etics.workspace(etics.etics_scf_workspace_size(n, nmax, lmax, prec), "cuda")

        def step(ev=None):
            if ev is not None:
                ev[0].record(stream)
            etics.etics_scf_coeffs(x, y, z, m, nmax, lmax, prec, A, B, ws, stream)
            if ev is not None:
                ev[1].record(stream)
            etics.etics_scf_force(x, y, z, nmax, lmax, A, B, prec, etics.ETICS_POT_ACC, pot, ax, ay, az,
                                  ws, stream)
            if ev is not None:
                ev[2].record(stream)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            step(evs[k])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        coef_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
        force_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
        out = [t.cpu().numpy() for t in (A, B, pot, ax, ay, az)]
        return wall, coef_ms, force_ms, out

    wall, coef_ms, force_ms, res = run_mode(etics.ETICS_MIXED_FP64ACC, args.steps, args.warmup)
    ms_per_step = wall / args.steps * 1e3
    value = n / (wall / args.steps)

    fp64 = None
    if not args.no_fp64:
        w64, c64, f64, res64 = run_mode(etics.ETICS_FP64, args.steps, args.warmup)
        fp64 = {"value": n / (w64 / args.steps), "ms_per_step": w64 / args.steps * 1e3,
                "coeff_call_ms": c64, "force_call_ms": f64}

    fc, ff = flops_per_particle(nmax, lmax)
    # dominant kernel: the force call (force kernel + a coefficient rescale of K entries)
    dom = "force" if force_ms >= coef_ms else "coeff"
    dom_ms = force_ms if dom == "force" else coef_ms
    dom_flops = (ff if dom == "force" else fc) * n
    achieved = dom_flops / (dom_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": None,
                "kernel": "scf_force_kernel<float,10,true>" if dom == "force" else "scf_coeff_kernel<float,11,4,0>",
                "flops_per_particle": ff if dom == "force" else fc,
                "frac_of_nonpacked_fp32": achieved / (PEAK_FP32_VECTOR_TFLOPS / 2)}
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
        "config": {"workload": "scf_triaxial_hernquist_n1e6_n10_l10" if (n, nmax, lmax) == (1_000_000, 10, 10)
                   else f"scf_triaxial_hernquist_n{n}_n{nmax}_l{lmax}",
                   "n": n, "nmax": nmax, "lmax": lmax, "seed": 2, "axes": [1.0, 0.8, 0.6],
                   "precision": "mixed: fp32 basis/synthesis, fp64 reduction"},
        "stages_ms": {"coeff_call": coef_ms, "force_call": force_ms},
        "step_tflops": step_tflops,
        "roofline": roofline,
    }
    if fp64:
        out["fp64"] = fp64
        out["speedup_vs_fp64"] = value / fp64["value"]

    import oracle
    if not args.no_cpu_baseline:
        # the oracle as it stands, all host threads, on the full workload: one force calculation
        t0 = time.perf_counter()
        rA, rB = oracle.scf_coeffs(p.x, p.y, p.z, p.m, nmax, lmax)
        rp, rx, ry, rz = oracle.scf_force(p.x, p.y, p.z, nmax, lmax, rA, rB)
        cpu_s = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": n / cpu_s, "unit": "particles/s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": f"the full workload (N={n}, ({nmax},{lmax})), one force calculation, "
                                         f"{cpu_s:.2f} s"}
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


if __name__ == "__main__":
    main()
