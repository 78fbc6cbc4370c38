"""Error measures used to report the accuracy of every result against a reference.

Per particle i the relative force error is |F_i - F_ref,i| / |F_ref,i| (the paper's
epsilon-tilde of Section 4.2, measured here against the FP64 oracle rather than an
FP64 run of the same code); the potential uses |dPhi_i| / |Phi_ref,i|.  Coefficient
sets are compared norm-wise, since individual coefficients can sit at the noise
floor where a relative error is meaningless.
"""
from __future__ import annotations

import numpy as np


def force_rel_err(ax, ay, az, rx, ry, rz) -> np.ndarray:
    num = np.sqrt((ax - rx) ** 2 + (ay - ry) ** 2 + (az - rz) ** 2)
    den = np.sqrt(rx * rx + ry * ry + rz * rz)
    return num / np.where(den > 0, den, 1.0)


def pot_rel_err(p, rp) -> np.ndarray:
    return np.abs(p - rp) / np.where(np.abs(rp) > 0, np.abs(rp), 1.0)


def coeff_errors(A, B, rA, rB) -> dict:
    d = np.concatenate([A - rA, B - rB])
    r = np.concatenate([rA, rB])
    nr = np.linalg.norm(r)
    mr = np.max(np.abs(r)) if r.size else 0.0
    return {
        "norm_rel": float(np.linalg.norm(d) / nr) if nr > 0 else float(np.linalg.norm(d)),
        "max_rel_to_max": float(np.max(np.abs(d)) / mr) if mr > 0 else float(np.max(np.abs(d), initial=0.0)),
    }


def summarize(e: np.ndarray) -> dict:
    if e.size == 0:
        return {"median": 0.0, "p99": 0.0, "max": 0.0}
    return {"median": float(np.median(e)), "p99": float(np.percentile(e, 99)), "max": float(np.max(e))}
