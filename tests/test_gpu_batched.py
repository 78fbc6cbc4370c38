"""GPU parity of the batched SCF calls and the hipGraph leapfrog (through the C-ABI)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_1406_4254_amd import accuracy as acc  # noqa: E402
from paper_1406_4254_amd import workloads as W  # noqa: E402

FP64, MIXED, COMP32 = 0, 1, 2


@pytest.fixture(scope="module")
def E():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1406_4254_amd import etics
    etics.lib()
    return etics


def small_batch(nsys=10, seed=31, nlog=(2.0, 3.5)):
    return W.batched_systems(nsys=nsys, seed=seed, nlog=nlog)


def dev(*arrs):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


def per_system(p, nmax, lmax, orc):
    out = []
    for s in range(len(p.offsets) - 1):
        b, e = p.offsets[s], p.offsets[s + 1]
        A, B = orc.scf_coeffs(p.x[b:e], p.y[b:e], p.z[b:e], p.m[b:e], nmax, lmax)
        out.append((A, B))
    return out


@pytest.mark.parametrize("prec", [FP64, MIXED, COMP32])
def test_batched_coeffs_and_force_match_oracle(E, orc, prec):
    p = small_batch()
    nmax, lmax = 8, 6
    K = E.etics_coeff_count(nmax, lmax)
    x, y, z, m, off = dev(p.x, p.y, p.z, p.m, p.offsets)
    A, B = E.etics_scf_coeffs_batched(x, y, z, m, off, nmax, lmax, prec)
    pot, ax, ay, az = E.etics_scf_force_batched(x, y, z, off, nmax, lmax, A, B, prec)
    A, B, pot, ax, ay, az = (t.cpu().numpy() for t in (A, B, pot, ax, ay, az))
    ref = per_system(p, nmax, lmax, orc)
    ctol = 3e-14 if prec == FP64 else 1e-5
    for s, (rA, rB) in enumerate(ref):
        e = acc.coeff_errors(A[s * K:(s + 1) * K], B[s * K:(s + 1) * K], rA, rB)
        assert e["norm_rel"] < ctol, (s, e)
        b, en = p.offsets[s], p.offsets[s + 1]
        rp, rx, ry, rz = orc.scf_force(p.x[b:en], p.y[b:en], p.z[b:en], nmax, lmax, rA, rB)
        ef = acc.summarize(acc.force_rel_err(ax[b:en], ay[b:en], az[b:en], rx, ry, rz))
        ep = acc.summarize(acc.pot_rel_err(pot[b:en], rp))
        if prec == FP64:
            assert ef["max"] < 1e-13 and ep["max"] < 1e-13, (s, ef, ep)
        else:
            assert ef["median"] <= 1e-5 and ef["p99"] <= 1e-4 and ep["p99"] <= 1e-4, (s, ef, ep)


@pytest.mark.parametrize("prec", [FP64, MIXED, COMP32])
def test_batched_systems_of_many_units(E, orc, prec):
    """A system of ~10 work units (4096 particles each) next to one- and two-unit ones:
    the per-system reduction adds many unit partials (double-float pairs in COMP32)."""
    p = W.batched_systems(nsys=4, seed=42, nlog=(3.0, 4.75))
    sizes = np.diff(p.offsets)
    assert sizes.max() > 8 * 4096, sizes
    nmax, lmax = 6, 4
    K = E.etics_coeff_count(nmax, lmax)
    x, y, z, m, off = dev(p.x, p.y, p.z, p.m, p.offsets)
    A, B = E.etics_scf_coeffs_batched(x, y, z, m, off, nmax, lmax, prec)
    A, B = A.cpu().numpy(), B.cpu().numpy()
    tol = 3e-14 if prec == FP64 else 1e-5
    for s in range(len(sizes)):
        b, e = p.offsets[s], p.offsets[s + 1]
        rA, rB = orc.scf_coeffs(p.x[b:e], p.y[b:e], p.z[b:e], p.m[b:e], nmax, lmax)
        er = acc.coeff_errors(A[s * K:(s + 1) * K], B[s * K:(s + 1) * K], rA, rB)
        assert er["norm_rel"] < tol, (s, int(sizes[s]), er)


def test_batched_equals_single_system_calls(E):
    p = small_batch(nsys=6, seed=32)
    nmax, lmax = 6, 4
    K = E.etics_coeff_count(nmax, lmax)
    x, y, z, m, off = dev(p.x, p.y, p.z, p.m, p.offsets)
    A, B = E.etics_scf_coeffs_batched(x, y, z, m, off, nmax, lmax, FP64)
    A, B = A.cpu().numpy(), B.cpu().numpy()
    for s in range(6):
        b, e = int(p.offsets[s]), int(p.offsets[s + 1])
        A1, B1 = E.etics_scf_coeffs(x[b:e].contiguous(), y[b:e].contiguous(), z[b:e].contiguous(),
                                    m[b:e].contiguous(), nmax, lmax, FP64)
        er = acc.coeff_errors(A[s * K:(s + 1) * K], B[s * K:(s + 1) * K], A1.cpu().numpy(), B1.cpu().numpy())
        assert er["norm_rel"] < 1e-13


def test_batched_empty_systems(E, orc):
    p = small_batch(nsys=5, seed=33)
    # insert two empty systems
    off = np.concatenate([[0], [p.offsets[1]] * 2, p.offsets[1:3], [p.offsets[3]] * 2, p.offsets[3:]])
    off = off.astype(np.int64)
    nsys = len(off) - 1
    nmax, lmax = 4, 3
    K = E.etics_coeff_count(nmax, lmax)
    x, y, z, m, doff = dev(p.x, p.y, p.z, p.m, off)
    A, B = E.etics_scf_coeffs_batched(x, y, z, m, doff, nmax, lmax, FP64)
    A, B = A.cpu().numpy(), B.cpu().numpy()
    for s in range(nsys):
        b, e = off[s], off[s + 1]
        if e == b:
            assert np.all(A[s * K:(s + 1) * K] == 0) and np.all(B[s * K:(s + 1) * K] == 0)
        else:
            rA, rB = orc.scf_coeffs(p.x[b:e], p.y[b:e], p.z[b:e], p.m[b:e], nmax, lmax)
            assert acc.coeff_errors(A[s * K:(s + 1) * K], B[s * K:(s + 1) * K], rA, rB)["norm_rel"] < 3e-14


def run_lf(E, p, nmax, lmax, dt, steps, prec, flags=0):
    x, y, z, vx, vy, vz, m, off = dev(p.x, p.y, p.z, p.vx, p.vy, p.vz, p.m, p.offsets)
    E.etics_leapfrog_scf_batched(x, y, z, vx, vy, vz, m, off, nmax, lmax, dt, steps, prec, flags)
    return [t.cpu().numpy() for t in (x, y, z, vx, vy, vz)]


def test_leapfrog_fp64_matches_oracle(E, orc):
    p = small_batch(nsys=4, seed=34, nlog=(2.5, 3.0))
    nmax, lmax, dt, steps = 6, 4, 0.01, 20
    got = run_lf(E, p, nmax, lmax, dt, steps, FP64)
    ref = orc.leapfrog_scf(p.x, p.y, p.z, p.vx, p.vy, p.vz, p.m, p.offsets, nmax, lmax, dt, steps)
    for g, r in zip(got, ref):
        np.testing.assert_allclose(g, r, rtol=1e-13, atol=1e-14)


def test_leapfrog_mixed_close_to_oracle(E, orc):
    p = small_batch(nsys=4, seed=35, nlog=(2.5, 3.0))
    nmax, lmax, dt, steps = 6, 4, 0.01, 20
    got = run_lf(E, p, nmax, lmax, dt, steps, MIXED)
    ref = orc.leapfrog_scf(p.x, p.y, p.z, p.vx, p.vy, p.vz, p.m, p.offsets, nmax, lmax, dt, steps)
    for g, r in zip(got[:3], ref[:3]):
        d = np.abs(g - r) / (1.0 + np.abs(r))
        assert np.median(d) < 1e-6 and np.max(d) < 1e-4


def test_leapfrog_graph_equals_eager(E):
    p = small_batch(nsys=8, seed=36)
    g = run_lf(E, p, 8, 6, 0.01, 10, MIXED, flags=0)
    e = run_lf(E, p, 8, 6, 0.01, 10, MIXED, flags=E.ETICS_LEAPFROG_EAGER)
    for a, b in zip(g, e):
        assert np.array_equal(a, b)
    # a second graph call with the same arguments replays the cached graph
    g2 = run_lf(E, p, 8, 6, 0.01, 10, MIXED, flags=0)
    for a, b in zip(g, g2):
        assert np.array_equal(a, b)


def test_leapfrog_time_reversible(E):
    import torch
    p = small_batch(nsys=3, seed=37, nlog=(2.5, 3.0))
    x, y, z, vx, vy, vz, m, off = dev(p.x, p.y, p.z, p.vx, p.vy, p.vz, p.m, p.offsets)
    E.etics_leapfrog_scf_batched(x, y, z, vx, vy, vz, m, off, 6, 4, 0.01, 20, FP64)
    for v in (vx, vy, vz):
        v.neg_()
    E.etics_leapfrog_scf_batched(x, y, z, vx, vy, vz, m, off, 6, 4, 0.01, 20, FP64)
    torch.cuda.synchronize()
    for a, b in zip((x, y, z), (p.x, p.y, p.z)):
        np.testing.assert_allclose(a.cpu().numpy(), b, rtol=1e-9, atol=1e-9)


def test_cfg5_full_size_sampled(E, orc):
    """256 systems (~5e6 particles), (8,6): coefficients and forces of 12 sampled
    systems against the oracle."""
    p = W.make_config(5)
    nmax, lmax = 8, 6
    K = E.etics_coeff_count(nmax, lmax)
    x, y, z, m, off = dev(p.x, p.y, p.z, p.m, p.offsets)
    A, B = E.etics_scf_coeffs_batched(x, y, z, m, off, nmax, lmax, MIXED)
    pot, ax, ay, az = E.etics_scf_force_batched(x, y, z, off, nmax, lmax, A, B, MIXED)
    A, B = A.cpu().numpy(), B.cpu().numpy()
    rng = np.random.default_rng(0)
    for s in rng.choice(256, size=12, replace=False):
        b, e = int(p.offsets[s]), int(p.offsets[s + 1])
        rA, rB = orc.scf_coeffs(p.x[b:e], p.y[b:e], p.z[b:e], p.m[b:e], nmax, lmax)
        assert acc.coeff_errors(A[s * K:(s + 1) * K], B[s * K:(s + 1) * K], rA, rB)["norm_rel"] < 1e-5
        rp, rx, ry, rz = orc.scf_force(p.x[b:e], p.y[b:e], p.z[b:e], nmax, lmax, rA, rB)
        ef = acc.summarize(acc.force_rel_err(ax[b:e].cpu().numpy(), ay[b:e].cpu().numpy(),
                                             az[b:e].cpu().numpy(), rx, ry, rz))
        print(f"cfg5 system {s} ({e - b} particles) mixed force {ef}", flush=True)
        # max: about 10x the largest measured on MI355X over these systems (9.5e-6,
        # at particles next to a sphere's centre, where the force tends to zero)
        assert ef["median"] <= 1e-5 and ef["p99"] <= 1e-4 and ef["max"] < 1e-4, (s, ef)


def test_leapfrog_step_counts_and_cache_replacement(E, orc):
    """nsteps = 0 changes nothing; nsteps = 1 (no graph) and several graph calls with
    different step counts and dt (the cached graph is replaced) all match the oracle."""
    p = small_batch(nsys=3, seed=38, nlog=(2.5, 3.0))
    nmax, lmax = 6, 4
    same = run_lf(E, p, nmax, lmax, 0.01, 0, FP64)
    for a, b in zip(same, (p.x, p.y, p.z, p.vx, p.vy, p.vz)):
        assert np.array_equal(a, b)
    for dt, steps in ((0.01, 1), (0.02, 3), (0.01, 5)):
        got = run_lf(E, p, nmax, lmax, dt, steps, FP64)
        ref = orc.leapfrog_scf(p.x, p.y, p.z, p.vx, p.vy, p.vz, p.m, p.offsets, nmax, lmax, dt, steps)
        for g, r in zip(got, ref):
            np.testing.assert_allclose(g, r, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("prec", [FP64, MIXED])
def test_cfg5_leapfrog_100_steps_sampled(E, orc, prec):
    """The benchmarked run: all 256 systems (~5.5e6 particles), (8,6), 100 graph-replayed
    KDK steps of dt = 0.01.  Twelve seeded systems are integrated by the oracle alone and
    compared with the GPU's final positions and velocities; the relative energy change of
    each sampled system (kinetic plus half the mass-weighted SCF potential, from the
    oracle) is printed beside the GPU's."""
    p = W.make_config(5)
    nmax, lmax, dt, steps = 8, 6, 0.01, 100
    got = run_lf(E, p, nmax, lmax, dt, steps, prec)
    rng = np.random.default_rng(5005)
    worst = 0.0
    for s in sorted(rng.choice(256, size=12, replace=False)):
        b, e = int(p.offsets[s]), int(p.offsets[s + 1])
        sl = slice(b, e)
        ref = orc.leapfrog_scf(p.x[sl], p.y[sl], p.z[sl], p.vx[sl], p.vy[sl], p.vz[sl], p.m[sl],
                               np.array([0, e - b], dtype=np.int64), nmax, lmax, dt, steps)
        dpos = np.sqrt(sum((g[sl] - r) ** 2 for g, r in zip(got[:3], ref[:3])))
        rpos = np.sqrt(sum(r ** 2 for r in ref[:3]))
        dvel = np.sqrt(sum((g[sl] - r) ** 2 for g, r in zip(got[3:], ref[3:])))
        rvel = np.sqrt(sum(r ** 2 for r in ref[3:]))
        ep = acc.summarize(dpos / (1.0 + rpos))  # relative, kept finite next to the centre
        ev = acc.summarize(dvel / (1.0 + rvel))

        def energy(st):
            A, B = orc.scf_coeffs(st[0], st[1], st[2], p.m[sl], nmax, lmax)
            pot = orc.scf_force(st[0], st[1], st[2], nmax, lmax, A, B)[0]
            return 0.5 * np.sum(p.m[sl] * (st[3] ** 2 + st[4] ** 2 + st[5] ** 2)) + 0.5 * np.sum(p.m[sl] * pot)

        e0 = energy((p.x[sl], p.y[sl], p.z[sl], p.vx[sl], p.vy[sl], p.vz[sl]))
        de_ref = energy(ref) / e0 - 1.0
        de_gpu = energy([g[sl] for g in got]) / e0 - 1.0
        print(f"lf prec{prec} sys {s} n={e - b}: pos {ep} vel {ev} dE/E oracle {de_ref:.3e} gpu {de_gpu:.3e}",
              flush=True)
        # measured on MI355X: FP64 position/velocity max 8.6e-16 / 2.5e-15; mixed
        # position median <= 2e-8, max 1.8e-7, velocity median <= 4.4e-8, max 4.5e-7, and
        # the relative energy change within 1.3e-9 of the oracle's
        if prec == FP64:
            assert ep["max"] < 1e-14 and ev["max"] < 3e-14, (s, ep, ev)
        else:
            assert ep["median"] < 2e-7 and ep["max"] < 2e-6, (s, ep, ev)
            assert ev["median"] < 5e-7 and ev["max"] < 5e-6, (s, ep, ev)
            assert abs(de_gpu - de_ref) < 1.5e-8
        worst = max(worst, ep["max"])
    print(f"lf prec{prec}: worst sampled position error {worst:.3e}", flush=True)
