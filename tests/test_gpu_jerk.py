"""GPU parity of the coefficient time derivatives, the jerk and the batched Hermite
integrator (through the C-ABI) against the FP64 oracle of oracle/jerk.py."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from paper_1406_4254_amd import accuracy as acc  # noqa: E402
from paper_1406_4254_amd import workloads as W  # noqa: E402

FP64, MIXED, COMP32 = 0, 1, 2


@pytest.fixture(scope="module")
def E():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1406_4254_amd import etics
    etics.lib()
    return etics


@pytest.fixture(scope="module")
def J(orc):
    from oracle import jerk
    return jerk


def moving_set(n, seed):
    """Triaxial Hernquist positions (rotated, so no symmetry hides a term), unequal
    masses and Gaussian velocities; none on the z axis."""
    p = W.make_config(2, n)
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    X = np.stack([p.x, p.y, p.z], 1) @ q.T
    m = rng.uniform(0.5, 1.5, n)
    m /= m.sum()
    v = rng.normal(size=(n, 3)) * 0.4
    return X, v, m


def cols(A):
    return [torch.from_numpy(np.ascontiguousarray(A[:, k])).cuda() for k in range(3)]


def dev(*arrs):
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda() for a in arrs]


def vec_err(got, ref):
    return np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)


def report(tag, e):
    s = acc.summarize(e)
    print(f"{tag}: median {s['median']:.3e} p99 {s['p99']:.3e} max {s['max']:.3e}", flush=True)
    return s


@pytest.mark.parametrize("nmax,lmax", [(6, 4), (10, 6), (8, 6), (2, 1), (10, 10), (20, 14)])
def test_coeffs_dot_fp64_match_oracle(E, J, nmax, lmax):
    X, v, m = moving_set(2003, 1)  # several tiles and a ragged tail
    A, B, dA, dB = J.coeffs_dot(torch.from_numpy(X), torch.from_numpy(v), torch.from_numpy(m), nmax, lmax)
    gA, gB = E.etics_scf_coeffs_dot(*cols(X), *cols(v), *dev(m), nmax, lmax, FP64)
    e = acc.coeff_errors(gA.cpu().numpy(), gB.cpu().numpy(), dA.numpy().ravel(), dB.numpy().ravel())
    print(f"coeffs_dot fp64 ({nmax},{lmax}) {e}", flush=True)
    # measured at most 2.9e-15 norm-wise, 3.8e-15 max/max (at (20,14))
    assert e["norm_rel"] < 4e-14 and e["max_rel_to_max"] < 4e-14


@pytest.mark.parametrize("prec", [MIXED, COMP32])
def test_coeffs_dot_mixed(E, J, prec):
    X, v, m = moving_set(20_000, 2)
    A, B, dA, dB = J.coeffs_dot(torch.from_numpy(X), torch.from_numpy(v), torch.from_numpy(m), 10, 6)
    gA, gB = E.etics_scf_coeffs_dot(*cols(X), *cols(v), *dev(m), 10, 6, prec)
    e = acc.coeff_errors(gA.cpu().numpy(), gB.cpu().numpy(), dA.numpy().ravel(), dB.numpy().ravel())
    print(f"coeffs_dot prec{prec} {e}", flush=True)
    assert e["norm_rel"] < 1e-5


@pytest.mark.parametrize("n", [1, 63, 64, 65, 129, 4099])
def test_coeffs_dot_ragged_and_repeatable(E, J, n):
    X, v, m = moving_set(n, 3)
    A, B, dA, dB = J.coeffs_dot(torch.from_numpy(X), torch.from_numpy(v), torch.from_numpy(m), 6, 5)
    a1 = E.etics_scf_coeffs_dot(*cols(X), *cols(v), *dev(m), 6, 5, FP64)
    a2 = E.etics_scf_coeffs_dot(*cols(X), *cols(v), *dev(m), 6, 5, FP64)
    assert torch.equal(a1[0], a2[0]) and torch.equal(a1[1], a2[1])
    e = acc.coeff_errors(a1[0].cpu().numpy(), a1[1].cpu().numpy(), dA.numpy().ravel(), dB.numpy().ravel())
    assert e["norm_rel"] < 4e-14


@pytest.mark.parametrize("nmax,lmax", [(6, 4), (10, 6), (8, 6), (10, 10)])
def test_jerk_fp64_matches_oracle(E, J, nmax, lmax):
    X, v, m = moving_set(1500, 4)
    P, V, M = torch.from_numpy(X), torch.from_numpy(v), torch.from_numpy(m)
    a_ref, j_ref = J.accel_jerk(P, V, M, nmax, lmax)
    A, B, dA, dB = J.coeffs_dot(P, V, M, nmax, lmax)
    d = dev(A.numpy().ravel(), B.numpy().ravel(), dA.numpy().ravel(), dB.numpy().ravel())
    out = E.etics_scf_jerk(*cols(X), *cols(v), nmax, lmax, *d, FP64)
    a = np.stack([t.cpu().numpy() for t in out[:3]], 1)
    j = np.stack([t.cpu().numpy() for t in out[3:]], 1)
    ea = report(f"jerk fp64 ({nmax},{lmax}) accel", vec_err(a, a_ref.numpy()))
    ej = report(f"jerk fp64 ({nmax},{lmax}) jerk", vec_err(j, j_ref.numpy()))
    # measured at most 2.8e-15 (acceleration) and 1.3e-13 (jerk, whose near-zero
    # values make the relative error of a few points larger)
    assert ea["max"] < 3e-14 and ej["max"] < 1.5e-12


@pytest.mark.parametrize("prec", [MIXED, COMP32])
def test_jerk_mixed_accuracy(E, J, prec):
    """Coefficients, their derivatives and the jerk pass all in the mixed mode against
    the FP64 oracle."""
    X, v, m = moving_set(20_000, 5)
    P, V, M = torch.from_numpy(X), torch.from_numpy(v), torch.from_numpy(m)
    a_ref, j_ref = J.accel_jerk(P, V, M, 8, 6)
    x, y, z = cols(X)
    vx, vy, vz = cols(v)
    md = dev(m)[0]
    A, B = E.etics_scf_coeffs(x, y, z, md, 8, 6, prec)
    dA, dB = E.etics_scf_coeffs_dot(x, y, z, vx, vy, vz, md, 8, 6, prec)
    out = E.etics_scf_jerk(x, y, z, vx, vy, vz, 8, 6, A, B, dA, dB, prec)
    a = np.stack([t.cpu().numpy() for t in out[:3]], 1)
    j = np.stack([t.cpu().numpy() for t in out[3:]], 1)
    ea = report(f"jerk prec{prec} accel", vec_err(a, a_ref.numpy()))
    ej = report(f"jerk prec{prec} jerk", vec_err(j, j_ref.numpy()))
    assert ea["median"] <= 1e-5 and ea["p99"] <= 1e-4
    assert ej["median"] <= 1e-5 and ej["p99"] <= 1e-4
    # max: about 10x the largest measured on MI355X (acceleration 6.7e-7, jerk 1.45e-5)
    assert ea["max"] < 1e-5 and ej["max"] < 1.5e-4


def test_jerk_off_axis_and_origin_finite(E):
    X, v, m = moving_set(300, 6)
    X[0] = 0.0
    X[1, :2] = 0.0
    A, B = E.etics_scf_coeffs(*cols(X), *dev(m), 6, 4, FP64)
    dA, dB = E.etics_scf_coeffs_dot(*cols(X), *cols(v), *dev(m), 6, 4, FP64)
    out = E.etics_scf_jerk(*cols(X), *cols(v), 6, 4, A, B, dA, dB, FP64)
    for t in out:
        assert bool(torch.isfinite(t).all())


def small_batch(nsys=3, seed=31):
    return W.batched_systems(nsys=nsys, seed=seed, nlog=(2.3, 2.6))


def run_hermite(E, p, nmax, lmax, dt, steps, prec, flags=0):
    x, y, z, vx, vy, vz, m, off = (torch.from_numpy(np.ascontiguousarray(a)).cuda()
                                   for a in (p.x, p.y, p.z, p.vx, p.vy, p.vz, p.m, p.offsets))
    E.etics_hermite_scf_batched(x, y, z, vx, vy, vz, m, off, nmax, lmax, dt, steps, prec, flags)
    return [t.cpu().numpy() for t in (x, y, z, vx, vy, vz)]


def test_hermite_fp64_matches_oracle(E, J):
    p = small_batch()
    nmax, lmax, dt, steps = 6, 4, 0.01, 8
    got = run_hermite(E, p, nmax, lmax, dt, steps, FP64)
    ref = J.hermite_systems(p.x, p.y, p.z, p.vx, p.vy, p.vz, p.m, p.offsets, nmax, lmax, dt, steps)
    for g, r in zip(got, ref):
        d = np.abs(g - r) / (1.0 + np.abs(r))
        print(f"hermite fp64: max {np.max(d):.3e}", flush=True)
        assert np.max(d) < 2e-15  # measured at most 1.4e-16


def test_hermite_mixed_close_to_oracle(E, J):
    p = small_batch(seed=32)
    nmax, lmax, dt, steps = 6, 4, 0.01, 8
    got = run_hermite(E, p, nmax, lmax, dt, steps, MIXED)
    ref = J.hermite_systems(p.x, p.y, p.z, p.vx, p.vy, p.vz, p.m, p.offsets, nmax, lmax, dt, steps)
    for g, r in zip(got, ref):
        d = np.abs(g - r) / (1.0 + np.abs(r))
        print(f"hermite mixed: median {np.median(d):.3e} max {np.max(d):.3e}", flush=True)
        assert np.median(d) < 2e-9 and np.max(d) < 4e-7  # measured: median 2.1e-10, max 3.9e-8


def test_hermite_graph_equals_eager(E):
    p = W.batched_systems(nsys=8, seed=36, nlog=(2.0, 3.5))
    g = run_hermite(E, p, 8, 6, 0.01, 6, MIXED, flags=0)
    e = run_hermite(E, p, 8, 6, 0.01, 6, MIXED, flags=E.ETICS_LEAPFROG_EAGER)
    for a, b in zip(g, e):
        assert np.array_equal(a, b)
    g2 = run_hermite(E, p, 8, 6, 0.01, 6, MIXED, flags=0)  # cached graph replayed
    for a, b in zip(g, g2):
        assert np.array_equal(a, b)


def test_hermite_step_counts(E, J):
    """nsteps = 0 changes nothing; 1 step (no graph) matches the oracle."""
    p = small_batch(nsys=2, seed=38)
    same = run_hermite(E, p, 5, 3, 0.02, 0, FP64)
    for a, b in zip(same, (p.x, p.y, p.z, p.vx, p.vy, p.vz)):
        assert np.array_equal(a, b)
    got = run_hermite(E, p, 5, 3, 0.02, 1, FP64)
    ref = J.hermite_systems(p.x, p.y, p.z, p.vx, p.vy, p.vz, p.m, p.offsets, 5, 3, 0.02, 1)
    for g, r in zip(got, ref):
        assert np.max(np.abs(g - r) / (1.0 + np.abs(r))) < 1e-13


def test_hermite_energy_error_is_fourth_order_on_gpu(E, J):
    """The GPU integrator itself: over a fixed time the relative energy error falls ~16x
    per halving of dt (fourth order; a second-order scheme gives ~4x)."""
    rng = np.random.default_rng(7)
    x, y, z = W.sphere(rng, 200, "plummer", 1.5)
    v = rng.normal(size=(200, 3)) * 0.3
    m = np.full(200, 1.0 / 200)
    p = W.Particles(x, y, z, m, v[:, 0].copy(), v[:, 1].copy(), v[:, 2].copy(),
                    np.array([0, 200], dtype=np.int64))
    X0 = torch.from_numpy(np.stack([x, y, z], 1))
    e0 = J.energy(X0, torch.from_numpy(v), torch.from_numpy(m), 4, 2)
    errs = []
    for dt in (0.05, 0.025, 0.0125):
        got = run_hermite(E, p, 4, 2, dt, int(round(0.4 / dt)), FP64)
        Xg = torch.from_numpy(np.stack(got[:3], 1))
        Vg = torch.from_numpy(np.stack(got[3:], 1))
        errs.append(abs(J.energy(Xg, Vg, torch.from_numpy(m), 4, 2) / e0 - 1.0))
    ratios = [errs[k] / errs[k + 1] for k in range(2)]
    print("gpu hermite energy errors", errs, "ratios", ratios, flush=True)
    for q in ratios:
        assert 12.0 < q < 28.0
