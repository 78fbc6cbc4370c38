"""GPU parity of every coefficient-kernel tile plan the tuner may pick: the outer
products on the VALU or on the matrix cores, other tile shapes, stream counts and
particle groups, for single systems, time derivatives, batched systems and the
Clutton-Brock basis, against the FP64 oracle and against the fixed rules' plan."""
import os

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from paper_1406_4254_amd import accuracy as acc  # noqa: E402
from paper_1406_4254_amd import workloads as W  # noqa: E402

FP64, MIXED, COMP32 = 0, 1, 2
HO, CB = 0, 1
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TUNING = os.path.join(ROOT, "paper_1406_4254_amd", "etics_tuning.json")


@pytest.fixture(scope="module")
def E():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1406_4254_amd import etics
    etics.lib()
    return etics


@pytest.fixture(autouse=True)
def clean_table(E):
    E.etics_tuning_clear()
    yield
    if os.path.exists(TUNING):
        E.etics_tuning_load(TUNING)
    else:
        E.etics_tuning_clear()


def dev(*arrs):
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda() for a in arrs]


def force_plan(E, n, nmax, lmax, prec, shape, batched=False, basis=HO):
    """Install a plan and check it is the one in force (a shape the kernel cannot run
    would silently fall back to the fixed rules)."""
    E.etics_tuning_set(nmax, lmax, prec, n, shape, batched=batched, basis=basis)
    info = E.etics_plan_info(n, nmax, lmax, prec, batched=batched, basis=basis)
    assert info["tuned"], (shape, info)
    for k, v in shape.items():
        if v:
            assert info[k] == v, (k, shape, info)
    return info


def coeffs(E, p, nmax, lmax, prec, basis=HO):
    x, y, z, m = dev(p.x, p.y, p.z, p.m)
    A, B = E.etics_scf_coeffs_basis(x, y, z, m, nmax, lmax, prec, basis)
    return A.cpu().numpy(), B.cpu().numpy()


# (nmax, lmax, plan): matrix phase 2 at every cutoff bucket (lmax 2, 6, 10, 14; one and two
# radial chunks) and 1, 2 or 4 wavefronts per particle group; VALU shapes off the fixed rules
SINGLE = [
    (10, 10, {"phase2": 2, "nw": 4, "tp": 64}),
    (10, 10, {"phase2": 2, "nw": 4, "tp": 37}),
    (20, 14, {"phase2": 2, "nw": 4, "tp": 32}),
    (3, 1, {"phase2": 2, "nw": 1, "tp": 256}),
    (8, 6, {"phase2": 2, "nw": 2, "tp": 128}),
    (10, 6, {"phase2": 2, "nw": 1, "tp": 192}),
    (12, 6, {"phase2": 2, "nw": 4, "tp": 60}),
    (0, 0, {"phase2": 2, "nw": 4, "tp": 64}),
    (10, 10, {"phase2": 1, "nw": 4, "tp": 42, "streams": 7}),
    (10, 6, {"phase2": 1, "nw": 2, "tp": 125, "streams": 5}),
    (20, 14, {"phase2": 1, "nw": 4, "tp": 30, "streams": 2, "grid_mult": 1}),
]


@pytest.mark.parametrize("prec", [MIXED, COMP32])
@pytest.mark.parametrize("nmax,lmax,shape", SINGLE)
def test_single_system_plans(E, orc, prec, nmax, lmax, shape):
    p = W.make_config(2, 9_001)  # several tiles and a ragged tail
    A0, B0 = coeffs(E, p, nmax, lmax, prec)  # fixed rules
    force_plan(E, p.n, nmax, lmax, prec, shape)
    A, B = coeffs(E, p, nmax, lmax, prec)
    rA, rB = orc.scf_coeffs(p.x, p.y, p.z, p.m, nmax, lmax)
    e = acc.coeff_errors(A, B, rA, rB)
    e0 = acc.coeff_errors(A, B, A0, B0)
    print(f"({nmax},{lmax}) prec{prec} {shape}: vs oracle {e['norm_rel']:.2e}, vs fixed plan {e0['norm_rel']:.2e}",
          flush=True)
    assert e["norm_rel"] < 1e-5
    # the same FP32 sums in another order: far closer to each other than to the oracle
    assert e0["norm_rel"] < 2e-6


@pytest.mark.parametrize("shape", [{"nw": 4, "tp": 48, "streams": 4}, {"nw": 2, "tp": 96, "streams": 6},
                                   {"nw": 1, "tp": 120, "streams": 10, "grid_mult": 2}])
def test_fp64_plans_match_oracle(E, orc, shape):
    p = W.make_config(2, 7_003)
    force_plan(E, p.n, 10, 6, FP64, shape)
    A, B = coeffs(E, p, 10, 6, FP64)
    rA, rB = orc.scf_coeffs(p.x, p.y, p.z, p.m, 10, 6)
    assert acc.coeff_errors(A, B, rA, rB)["norm_rel"] < 3e-14


@pytest.mark.parametrize("prec", [MIXED, COMP32])
@pytest.mark.parametrize("nmax,lmax", [(10, 10), (6, 4)])
def test_matrix_phase2_clutton_brock(E, orc, prec, nmax, lmax):
    p = W.make_config(2, 6_007)
    force_plan(E, p.n, nmax, lmax, prec, {"phase2": 2}, basis=CB)
    A, B = coeffs(E, p, nmax, lmax, prec, basis=CB)
    rA, rB = orc.scf_coeffs(p.x, p.y, p.z, p.m, nmax, lmax, basis=CB)
    e = acc.coeff_errors(A, B, rA, rB)
    print(f"CB ({nmax},{lmax}) prec{prec} matrix: {e}", flush=True)
    assert e["norm_rel"] < 1e-5


@pytest.mark.parametrize("prec", [MIXED, COMP32])
@pytest.mark.parametrize("nmax,lmax,shape", [(10, 6, {"phase2": 2}), (10, 10, {"phase2": 2, "tp": 38}),
                                             (8, 6, {"phase2": 1, "nw": 4, "tp": 64, "streams": 4})])
def test_time_derivative_plans(E, prec, nmax, lmax, shape):
    from oracle import jerk as J
    n = 5_001
    p = W.make_config(2, n)
    rng = np.random.default_rng(5)
    X = np.stack([p.x, p.y, p.z], 1)
    v = rng.normal(size=(n, 3)) * 0.4
    m = p.m
    _, _, dA, dB = J.coeffs_dot(torch.from_numpy(X), torch.from_numpy(v), torch.from_numpy(m), nmax, lmax)
    force_plan(E, n, nmax, lmax, prec, shape)
    cols = dev(X[:, 0], X[:, 1], X[:, 2], v[:, 0], v[:, 1], v[:, 2], m)
    gA, gB = E.etics_scf_coeffs_dot(*cols, nmax, lmax, prec)
    e = acc.coeff_errors(gA.cpu().numpy(), gB.cpu().numpy(), dA.numpy().ravel(), dB.numpy().ravel())
    print(f"coeffs_dot ({nmax},{lmax}) prec{prec} {shape}: {e}", flush=True)
    assert e["norm_rel"] < 1e-5


@pytest.mark.parametrize("prec", [MIXED, COMP32])
@pytest.mark.parametrize("shape", [{"phase2": 2}, {"phase2": 2, "nw": 4, "tp": 64, "unit": 1024, "split": 2},
                                   {"phase2": 1, "nw": 1, "tp": 256, "streams": 16, "unit": 8192, "split": 8}])
def test_batched_plans(E, orc, prec, shape):
    p = W.batched_systems(nsys=6, seed=17, nlog=(2.0, 3.7))
    nmax, lmax = 8, 6
    K = E.etics_coeff_count(nmax, lmax)
    force_plan(E, p.offsets[-1], nmax, lmax, prec, shape, batched=True)
    x, y, z, m = dev(p.x, p.y, p.z, p.m)
    off = torch.from_numpy(np.ascontiguousarray(p.offsets)).cuda()
    A, B = E.etics_scf_coeffs_batched(x, y, z, m, off, nmax, lmax, prec)
    pot, ax, ay, az = E.etics_scf_force_batched(x, y, z, off, nmax, lmax, A, B, prec)
    A, B, ax, ay, az = (t.cpu().numpy() for t in (A, B, ax, ay, az))
    for s in range(len(p.offsets) - 1):
        b, en = p.offsets[s], p.offsets[s + 1]
        rA, rB = orc.scf_coeffs(p.x[b:en], p.y[b:en], p.z[b:en], p.m[b:en], nmax, lmax)
        e = acc.coeff_errors(A[s * K:(s + 1) * K], B[s * K:(s + 1) * K], rA, rB)
        assert e["norm_rel"] < 1e-5, (s, e)
        _, rx, ry, rz = orc.scf_force(p.x[b:en], p.y[b:en], p.z[b:en], nmax, lmax, rA, rB)
        ef = acc.summarize(acc.force_rel_err(ax[b:en], ay[b:en], az[b:en], rx, ry, rz))
        assert ef["median"] <= 1e-5 and ef["p99"] <= 1e-4, (s, ef)
