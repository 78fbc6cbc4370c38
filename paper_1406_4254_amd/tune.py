"""Autotuner of the coefficient kernels' tile plans.

The coefficient kernels (single system and batched) take their tile shape from a plan
(see include/etics.h, "Tile plans and the autotuner"): wavefronts per particle group
``nw``, particles per tile ``tp``, stream copies ``streams``, workgroups per CU
``grid_mult``, where the FP32 outer products run ``phase2`` (1 = vector ALUs, 2 =
matrix cores) and, for batched systems, particles per work unit ``unit`` and force
workgroups per unit ``split``.  The library derives a plan from fixed rules; this
module measures candidate plans on the device and keeps the fastest per workload:

  * candidates: every valid combination of the shape parameters around the fixed
    rules' plan (the fixed plan itself always included);
  * each candidate is installed with ``etics_tuning_set``, checked to be in force with
    ``etics_plan_info`` (an invalid shape falls back to the fixed rules and is skipped),
    timed with HIP events over repeated calls (median), and its coefficients are
    compared with those of the fixed plan (same sums in another order);
  * the winner replaces the fixed plan only if it is at least ``margin`` faster; either
    way the chosen shape is written to the JSON table the library reads.

Run on the GPU:  python -m paper_1406_4254_amd.tune --out <json> --report <md>
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import platform
import sys
import time

import numpy as np
import torch

from paper_1406_4254_amd import etics as E
from paper_1406_4254_amd import workloads as W

PREC_NAMES = {E.ETICS_FP64: "fp64", E.ETICS_MIXED_FP64ACC: "mixed", E.ETICS_MIXED_COMP32: "comp32"}


def _median_ms(fn, reps, warm=1):
    for _ in range(warm):
        fn()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    st = torch.cuda.current_stream()
    torch.cuda.synchronize()
    for a, b in ev:
        a.record(st)
        fn()
        b.record(st)
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def _rel(A, B, A0, B0):
    d = torch.cat([A - A0, B - B0])
    r = torch.cat([A0, B0])
    return float(torch.linalg.norm(d) / torch.linalg.norm(r))


def single_candidates(base, lmax, prec):
    """Shapes around the fixed plan of a single-system coefficient call (1 or 2
    wavefronts per particle group exist for lmax <= 6 only; the matrix-core phase 2 for
    the FP32 modes only, without streams)."""
    smax = max(base["streams"], 1)
    nws = [1, 2, 4] if lmax <= 6 else [4]
    out = []
    for nw, s, gm in itertools.product(nws, range(1, smax + 1), (1, 2)):
        tmax = 64 * (4 // nw)
        tps = sorted({t for t in (tmax // s * s, (3 * tmax // 4) // s * s, (tmax // 2) // s * s) if t >= s})
        for tp in tps:
            out.append({"nw": nw, "tp": tp, "streams": s, "grid_mult": gm, "unit": 0, "split": 0, "phase2": 1})
    if prec != E.ETICS_FP64:
        for nw, gm in itertools.product(nws, (1, 2)):
            tmax = 64 * (4 // nw)
            for tp in sorted({tmax, 3 * tmax // 4 // 4 * 4, tmax // 2, 60, 56, 48, 32}):
                if 4 <= tp <= tmax:
                    out.append({"nw": nw, "tp": tp, "streams": base["streams"], "grid_mult": gm, "unit": 0,
                                "split": 0, "phase2": 2})
    return out


def batched_candidates(base):
    """Work unit, force split and tile shape around the fixed plan of batched calls."""
    out = []
    for unit, split, gm in itertools.product((1024, 2048, 4096, 8192), (1, 2, 4, 8), (1, 2)):
        if unit // split < 64:
            continue
        out.append({"nw": base["nw"], "tp": base["tp"], "streams": base["streams"], "grid_mult": gm,
                    "unit": unit, "split": split, "phase2": base["phase2"]})
    for nw, ph in itertools.product((1, 2, 4), (1, 2)):
        tmax = 64 * (4 // nw)
        s = base["streams"]
        if s > tmax:
            continue
        out.append({"nw": nw, "tp": tmax // s * s if ph == 1 else tmax, "streams": s,
                    "grid_mult": base["grid_mult"], "unit": base["unit"], "split": base["split"], "phase2": ph})
    return out


def _shape(plan):
    return {k: plan[k] for k in E.PLAN_FIELDS}


def _in_force(info, c):
    """The plan in force is the candidate (its zero fields keep the fixed rules)."""
    return info["tuned"] and all(c[k] == 0 or info[k] == c[k] for k in E.PLAN_FIELDS)


def tune_single(name, p, nmax, lmax, prec, basis=E.ETICS_BASIS_HO, reps=7, margin=0.02, log=print):
    n = p.n
    x, y, z, m = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (p.x, p.y, p.z, p.m))
    K = E.etics_coeff_count(nmax, lmax)
    A = torch.empty(K, dtype=torch.float64, device="cuda")
    B = torch.empty_like(A)

    def run_plan(shape):
        if shape is not None:
            E.etics_tuning_set(nmax, lmax, prec, n, shape, basis=basis)
        info = E.etics_plan_info(n, nmax, lmax, prec, basis=basis)
        ws = E.workspace(E.etics_scf_workspace_size(n, nmax, lmax, prec), "cuda")
        call = lambda: E.etics_scf_coeffs_basis(x, y, z, m, nmax, lmax, prec, basis, A, B, ws)
        ms = _median_ms(call, reps)
        return info, ms, A.clone(), B.clone()

    E.etics_tuning_clear()
    base, base_ms, A0, B0 = run_plan(None)
    tol = 1e-12 if prec == E.ETICS_FP64 else 2e-5
    rows = [dict(_shape(base), ms=base_ms, rel=0.0, fixed=True)]
    for c in single_candidates(base, lmax, prec):
        info, ms, A1, B1 = run_plan(c)
        E.etics_tuning_clear()
        if not _in_force(info, c):
            continue  # not a valid shape for this kernel
        rel = _rel(A1, B1, A0, B0)
        rows.append(dict(_shape(info), ms=ms, rel=rel, fixed=False))
        if not rel < tol:
            raise RuntimeError(f"{name}: plan {c} differs from the fixed plan by {rel:.2e}")

    def retime(shape, fixed):
        ms = run_plan(None if fixed else shape)[1]
        E.etics_tuning_clear()
        return ms

    return _choose(name, dict(batched=0, nmax=nmax, lmax=lmax, prec=prec, basis=basis, n=n), rows, margin, log,
                   retime)


def tune_batched(name, q, nmax, lmax, prec, reps=5, margin=0.02, log=print):
    nt = q.n
    nsys = len(q.offsets) - 1
    x, y, z, m = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (q.x, q.y, q.z, q.m))
    off = torch.from_numpy(q.offsets).cuda()
    K = E.etics_coeff_count(nmax, lmax)
    A = torch.empty(nsys * K, dtype=torch.float64, device="cuda")
    B = torch.empty_like(A)
    outs = [torch.empty(nt, dtype=torch.float64, device="cuda") for _ in range(3)]

    def run_plan(shape):
        if shape is not None:
            E.etics_tuning_set(nmax, lmax, prec, nt, shape, batched=True)
        info = E.etics_plan_info(nt, nmax, lmax, prec, batched=True)
        ws = E.workspace(E.etics_batched_workspace_size(nt, nsys, nmax, lmax, prec), "cuda")

        def call():
            E.etics_scf_coeffs_batched(x, y, z, m, off, nmax, lmax, prec, A, B, ws)
            E.etics_scf_force_batched(x, y, z, off, nmax, lmax, A, B, prec, E.ETICS_ACC, None, *outs, ws)

        ms = _median_ms(call, reps)
        return info, ms, A.clone(), B.clone()

    E.etics_tuning_clear()
    base, base_ms, A0, B0 = run_plan(None)
    tol = 1e-12 if prec == E.ETICS_FP64 else 2e-5
    rows = [dict(_shape(base), ms=base_ms, rel=0.0, fixed=True)]
    for c in batched_candidates(base):
        info, ms, A1, B1 = run_plan(c)
        E.etics_tuning_clear()
        if not _in_force(info, c):
            continue
        rel = _rel(A1, B1, A0, B0)
        rows.append(dict(_shape(info), ms=ms, rel=rel, fixed=False))
        if not rel < tol:
            raise RuntimeError(f"{name}: plan {c} differs from the fixed plan by {rel:.2e}")

    def retime(shape, fixed):
        ms = run_plan(None if fixed else shape)[1]
        E.etics_tuning_clear()
        return ms

    return _choose(name, dict(batched=1, nmax=nmax, lmax=lmax, prec=prec, basis=0, n=nt), rows, margin, log,
                   retime)


def _choose(name, key, rows, margin, log, retime=None):
    """Pick the plan: the fastest candidates of the sweep are timed again against the
    fixed plan in interleaved rounds (the sweep's single timings carry warm-up and
    clock noise), and a candidate replaces the fixed plan only if its median over the
    rounds is at least `margin` faster."""
    fixed = rows[0]
    if retime is not None:
        top = [r for r in sorted(rows[1:], key=lambda r: r["ms"]) if _shape(r) != _shape(fixed)][:3]
        pool = [fixed] + top
        times = {id(r): [] for r in pool}
        for _ in range(5):
            for r in pool:
                times[id(r)].append(retime(_shape(r), r is fixed))
        for r in pool:
            r["ms"] = float(np.median(times[id(r)]))
            r["retimed"] = True
        cand = min(top, key=lambda r: r["ms"]) if top else fixed
    else:
        cand = min(rows, key=lambda r: r["ms"])
    best = cand if cand["ms"] <= (1.0 - margin) * fixed["ms"] else fixed
    plan = dict(key, **_shape(best), ms=best["ms"], fixed_ms=fixed["ms"], workload=name,
                source="fixed rules" if best is fixed else "tuned")
    log(f"{name}: fixed {fixed['ms']:.4f} ms -> chosen {best['ms']:.4f} ms {_shape(best)} "
        f"({len(rows)} plans measured)")
    return plan, rows


WORKLOADS = {
    # name: (kind, particle factory, nmax, lmax, precisions)
    "scf_hernquist_n1e4_n10_l6": ("single", lambda: W.make_config(1), 10, 6,
                                  (E.ETICS_FP64, E.ETICS_MIXED_FP64ACC)),
    "scf_triaxial_hernquist_n1e6_n10_l10": ("single", lambda: W.make_config(2), 10, 10,
                                            (E.ETICS_MIXED_FP64ACC, E.ETICS_FP64)),
    "scf_hernquist_plummer_n1e7_n20_l14": ("single", lambda: W.make_config(3), 20, 14,
                                           (E.ETICS_MIXED_FP64ACC, E.ETICS_MIXED_COMP32, E.ETICS_FP64)),
    "batched_256_spheres_n8_l6": ("batched", lambda: W.make_config(5), 8, 6,
                                  (E.ETICS_MIXED_FP64ACC, E.ETICS_FP64)),
}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", required=True, help="JSON table to write (the library reads etics_tuning.json)")
    ap.add_argument("--report", help="markdown summary of every plan measured")
    ap.add_argument("--workloads", default=",".join(WORKLOADS))
    ap.add_argument("--margin", type=float, default=0.02)
    args = ap.parse_args(argv)
    assert torch.cuda.is_available(), "the tuner measures on the GPU"
    t0 = time.time()
    plans, tables = [], []
    for name in args.workloads.split(","):
        kind, make, nmax, lmax, precs = WORKLOADS[name]
        p = make()
        for prec in precs:
            tag = f"{name} {PREC_NAMES[prec]}"
            if kind == "single":
                plan, rows = tune_single(tag, p, nmax, lmax, prec, margin=args.margin)
            else:
                plan, rows = tune_batched(tag, p, nmax, lmax, prec, margin=args.margin)
            plans.append(plan)
            tables.append((tag, plan, rows))
            sys.stdout.flush()
        del p
        torch.cuda.empty_cache()
    E.etics_tuning_clear()
    doc = {"device": torch.cuda.get_device_name(0), "library": E.etics_version(),
           "host": platform.node(), "margin": args.margin, "plans": plans}
    with open(args.out, "w") as fh:
        json.dump(doc, fh, indent=1)
    if args.report:
        with open(args.report, "w") as fh:
            fh.write(report(doc, tables, " ".join(sys.argv[1:] if argv is None else argv), time.time() - t0))
    print(f"wrote {len(plans)} plans to {args.out}")


def report(doc, tables, cmd, secs, shown=8):
    lines = [f"# Coefficient-kernel tile plans measured by the autotuner ({doc['device']})", "",
             "Command (R = repository root; the tuner times each candidate plan with HIP events, "
             "median of repeated coefficient calls, batched: coefficients + force):", "", "```",
             f"cd $R && python -m paper_1406_4254_amd.tune {cmd}", "```", "",
             f"{sum(len(t[2]) for t in tables)} plans measured in {secs:.0f} s; the three fastest "
             f"candidates and the fixed rules' plan are then timed again in 5 interleaved rounds, and a "
             f"candidate replaces the fixed plan only if its median is at least "
             f"{100 * doc['margin']:.0f}% faster.  The library reads the written table from "
             f"etics_tuning.json next to libetics.so (or $ETICS_TUNING_FILE).", ""]
    lines += ["| workload | fixed plan ms | chosen ms | speed-up | chosen plan |", "|---|---|---|---|---|"]
    for tag, plan, rows in tables:
        lines.append(f"| {tag} | {plan['fixed_ms']:.4f} | {plan['ms']:.4f} | "
                     f"{plan['fixed_ms'] / plan['ms']:.3f} | {plan['source']}: "
                     f"{ {k: plan[k] for k in E.PLAN_FIELDS} } |")
    for tag, plan, rows in tables:
        order = sorted(rows, key=lambda r: r["ms"])
        # the fastest few, the fixed plan and the fastest of each phase-2 kind
        keep = order[:shown]
        for r in order:
            if r not in keep and (r["fixed"] or all(k["phase2"] != r["phase2"] for k in keep)):
                keep.append(r)
        lines += ["", f"## {tag}", "", f"{len(keep)} of {len(rows)} candidates, fastest first.", "",
                  "| phase2 | nw | tp | streams | grid_mult | unit | split | ms | rel. diff vs fixed |",
                  "|---|---|---|---|---|---|---|---|---|"]
        for r in sorted(keep, key=lambda r: r["ms"]):
            mark = " (fixed rules)" if r["fixed"] else ""
            mark += " (re-timed: median of 5 interleaved rounds)" if r.get("retimed") else ""
            ph = "matrix" if r["phase2"] == 2 else "VALU"
            lines.append(f"| {ph} | {r['nw']} | {r['tp']} | {r['streams']} | {r['grid_mult']} | {r['unit']} | "
                         f"{r['split']} | {r['ms']:.4f}{mark} | {r['rel']:.1e} |")
    return "\n".join(lines) + "\n"


if __name__ == "__main__":
    main()
