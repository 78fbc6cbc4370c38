"""GPU parity of the SCF path (through the C-ABI) against the FP64 CPU oracle."""
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


def dev(*arrs):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda() for a in arrs]


def host(*ts):
    return [t.cpu().numpy() for t in ts]


def gpu_coeffs(E, p, nmax, lmax, prec):
    x, y, z, m = dev(p.x, p.y, p.z, p.m)
    A, B = E.etics_scf_coeffs(x, y, z, m, nmax, lmax, prec)
    return host(A, B)


def gpu_force(E, p, nmax, lmax, A, B, prec, outputs=3):
    x, y, z = dev(p.x, p.y, p.z)
    dA, dB = dev(A, B)
    r = E.etics_scf_force(x, y, z, nmax, lmax, dA, dB, prec, outputs)
    return [None if t is None else t.cpu().numpy() for t in r]


def report(tag, e):
    s = acc.summarize(e)
    print(f"{tag}: median {s['median']:.3e} p99 {s['p99']:.3e} max {s['max']:.3e}", flush=True)
    return s


# ------------------------------------------------------------------ FP64 parity
@pytest.mark.parametrize("nmax,lmax", [(10, 6), (0, 0), (2, 1), (4, 4), (3, 7), (8, 6), (12, 3), (20, 14)])
def test_fp64_coeffs_match_oracle(E, orc, nmax, lmax):
    p = W.make_config(1, 3001)  # several tiles and a ragged tail
    A, B = gpu_coeffs(E, p, nmax, lmax, FP64)
    rA, rB = orc.scf_coeffs(p.x, p.y, p.z, p.m, nmax, lmax)
    e = acc.coeff_errors(A, B, rA, rB)
    print(nmax, lmax, e, flush=True)
    # measured at most 3.2e-15 over these cutoffs
    assert e["norm_rel"] < 3e-14 and e["max_rel_to_max"] < 3e-14


@pytest.mark.parametrize("nmax,lmax", [(10, 6), (2, 1), (4, 4), (8, 6), (20, 14)])
def test_fp64_force_match_oracle(E, orc, nmax, lmax):
    p = W.make_config(2, 2500)
    rA, rB = orc.scf_coeffs(p.x, p.y, p.z, p.m, nmax, lmax)
    pot, ax, ay, az = gpu_force(E, p, nmax, lmax, rA, rB, FP64)
    pot1 = gpu_force(E, p, nmax, lmax, rA, rB, FP64, outputs=1)[0]
    rp, rx, ry, rz = orc.scf_force(p.x, p.y, p.z, nmax, lmax, rA, rB)
    ef = report(f"fp64 force ({nmax},{lmax})", acc.force_rel_err(ax, ay, az, rx, ry, rz))
    ep = report(f"fp64 pot ({nmax},{lmax})", acc.pot_rel_err(pot, rp))
    ep1 = report(f"fp64 pot-only ({nmax},{lmax})", acc.pot_rel_err(pot1, rp))
    # measured at most 1.1e-14 (force and potential, at (20,14))
    assert ef["max"] < 1e-13 and ep["max"] < 1e-13 and ep1["max"] < 1e-13


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 129, 4099])
def test_fp64_ragged_sizes(E, orc, n):
    p = W.make_config(2, n)
    nmax, lmax = 6, 5
    A, B = gpu_coeffs(E, p, nmax, lmax, FP64)
    rA, rB = orc.scf_coeffs(p.x, p.y, p.z, p.m, nmax, lmax)
    assert acc.coeff_errors(A, B, rA, rB)["norm_rel"] < 3e-14
    pot, ax, ay, az = gpu_force(E, p, nmax, lmax, A, B, FP64)
    rp, rx, ry, rz = orc.scf_force(p.x, p.y, p.z, nmax, lmax, rA, rB)
    assert np.max(acc.force_rel_err(ax, ay, az, rx, ry, rz)) < 1e-13
    assert np.max(acc.pot_rel_err(pot, rp)) < 1e-13


# ---------------------------------------------------------- mixed precision gate
@pytest.mark.parametrize("prec", [MIXED, COMP32])
@pytest.mark.parametrize("cfg,n,nmax,lmax", [(1, 10_000, 10, 6), (2, 30_000, 10, 10), (3, 20_000, 20, 14)])
def test_mixed_force_accuracy(E, orc, prec, cfg, n, nmax, lmax):
    """Force relative error against the FP64 oracle: median <= 1e-5, p99 <= 1e-4."""
    p = W.make_config(cfg, n)
    A, B = gpu_coeffs(E, p, nmax, lmax, prec)
    rA, rB = orc.scf_coeffs(p.x, p.y, p.z, p.m, nmax, lmax)
    ce = acc.coeff_errors(A, B, rA, rB)
    print(f"cfg{cfg} prec{prec} coeff {ce}", flush=True)
    pot, ax, ay, az = gpu_force(E, p, nmax, lmax, A, B, prec)
    pot1 = gpu_force(E, p, nmax, lmax, A, B, prec, outputs=1)[0]
    rp, rx, ry, rz = orc.scf_force(p.x, p.y, p.z, nmax, lmax, rA, rB)
    ef = report(f"cfg{cfg} prec{prec} force", acc.force_rel_err(ax, ay, az, rx, ry, rz))
    ep = report(f"cfg{cfg} prec{prec} pot", acc.pot_rel_err(pot, rp))
    ep1 = report(f"cfg{cfg} prec{prec} pot-only", acc.pot_rel_err(pot1, rp))
    assert ef["median"] <= 1e-5 and ef["p99"] <= 1e-4
    for e in (ep, ep1):
        assert e["median"] <= 1e-5 and e["p99"] <= 1e-4
    assert ce["norm_rel"] < 1e-5


@pytest.mark.parametrize("prec", [MIXED, COMP32])
@pytest.mark.parametrize("nmax,lmax", [(0, 0), (3, 1), (6, 2), (8, 6), (12, 6)])
def test_mixed_small_cutoffs_ragged(E, orc, prec, nmax, lmax):
    """Small cutoffs use tiles of 128 or 256 particles; a ragged N (not a multiple of
    the tile) must still reach the gate."""
    p = W.make_config(2, 5003)
    A, B = gpu_coeffs(E, p, nmax, lmax, prec)
    rA, rB = orc.scf_coeffs(p.x, p.y, p.z, p.m, nmax, lmax)
    assert acc.coeff_errors(A, B, rA, rB)["norm_rel"] < 1e-5
    pot, ax, ay, az = gpu_force(E, p, nmax, lmax, A, B, prec)
    rp, rx, ry, rz = orc.scf_force(p.x, p.y, p.z, nmax, lmax, rA, rB)
    ef = report(f"small ({nmax},{lmax}) prec{prec} force", acc.force_rel_err(ax, ay, az, rx, ry, rz))
    ep = report(f"small ({nmax},{lmax}) prec{prec} pot", acc.pot_rel_err(pot, rp))
    assert ef["median"] <= 1e-5 and ef["p99"] <= 1e-4
    assert ep["median"] <= 1e-5 and ep["p99"] <= 1e-4


def test_cfg2_full_size(E, orc):
    """N = 10^6, (10,10), triaxial Hernquist: the benchmark workload, every particle, in
    both output selections (potential and acceleration; potential only).

    FP64 is compared with the oracle built with long-double running sums, whose result
    differs from the plain oracle only by the plain oracle's own summation rounding
    (printed); the mixed mode with the plain oracle against the accuracy gate."""
    p = W.make_config(2)
    rA, rB = orc.scf_coeffs(p.x, p.y, p.z, p.m, 10, 10)
    rp, rx, ry, rz = orc.scf_force(p.x, p.y, p.z, 10, 10, rA, rB)
    lA, lB = orc.scf_coeffs(p.x, p.y, p.z, p.m, 10, 10, ext=True)
    lp, lx, ly, lz = orc.scf_force(p.x, p.y, p.z, 10, 10, lA, lB, ext=True)
    print(f"cfg2 plain oracle vs long double: coeff {acc.coeff_errors(rA, rB, lA, lB)} "
          f"force {acc.summarize(acc.force_rel_err(rx, ry, rz, lx, ly, lz))} "
          f"pot {acc.summarize(acc.pot_rel_err(rp, lp))}", flush=True)
    for prec in (MIXED, FP64):
        A, B = gpu_coeffs(E, p, 10, 10, prec)
        pot, ax, ay, az = gpu_force(E, p, 10, 10, A, B, prec)
        pot1, nx, _, _ = gpu_force(E, p, 10, 10, A, B, prec, outputs=1)
        assert nx is None
        if prec == FP64:
            ce = acc.coeff_errors(A, B, lA, lB)
            print(f"cfg2 full fp64 coeff vs long double {ce}", flush=True)
            ef = report("cfg2 full fp64 force vs long double", acc.force_rel_err(ax, ay, az, lx, ly, lz))
            ep = report("cfg2 full fp64 pot vs long double", acc.pot_rel_err(pot, lp))
            ep1 = report("cfg2 full fp64 pot-only vs long double", acc.pot_rel_err(pot1, lp))
            # measured: coefficients 3.3e-15 (4.7e-15 max/max), force max 1.8e-15,
            # potential max 1.3e-15
            assert ce["norm_rel"] < 3.5e-14 and ce["max_rel_to_max"] < 5e-14
            assert ef["max"] < 2e-14 and ep["max"] < 2e-14 and ep1["max"] < 2e-14
        else:
            ce = acc.coeff_errors(A, B, rA, rB)
            print(f"cfg2 full mixed coeff {ce}", flush=True)
            ef = report("cfg2 full mixed force", acc.force_rel_err(ax, ay, az, rx, ry, rz))
            ep = report("cfg2 full mixed pot", acc.pot_rel_err(pot, rp))
            ep1 = report("cfg2 full mixed pot-only", acc.pot_rel_err(pot1, rp))
            assert ef["median"] <= 1e-5 and ef["p99"] <= 1e-4 and ce["norm_rel"] < 1e-5
            for e in (ep, ep1):
                assert e["median"] <= 1e-5 and e["p99"] <= 1e-4
            # beyond the gate: every particle of the workload, about 10x the largest
            # error measured on MI355X (force max 9.4e-7, potential max 7.2e-7)
            assert ef["max"] < 1e-5 and ep["max"] < 1e-5 and ep1["max"] < 1e-5


# ------------------------------------------------------------------ edge cases
def test_zero_particles(E):
    import torch
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    A = torch.full((E.etics_coeff_count(4, 3),), 7.0, dtype=torch.float64, device="cuda")
    B = A.clone()
    E.etics_scf_coeffs(e, e, e, e, 4, 3, MIXED, A, B)
    assert float(A.abs().max()) == 0.0 and float(B.abs().max()) == 0.0
    pot, ax, ay, az = E.etics_scf_force(e, e, e, 4, 3, A, B, MIXED)
    assert pot.numel() == 0


def test_deterministic_repeat(E):
    p = W.make_config(2, 50_000)
    for prec in (FP64, MIXED, COMP32):
        A1, B1 = gpu_coeffs(E, p, 10, 10, prec)
        A2, B2 = gpu_coeffs(E, p, 10, 10, prec)
        assert np.array_equal(A1, A2) and np.array_equal(B1, B2)


def test_output_modes_agree(E):
    p = W.make_config(2, 5000)
    A, B = gpu_coeffs(E, p, 8, 6, MIXED)
    both = gpu_force(E, p, 8, 6, A, B, MIXED, 3)
    pot = gpu_force(E, p, 8, 6, A, B, MIXED, 1)
    accel = gpu_force(E, p, 8, 6, A, B, MIXED, 2)
    # separate kernel instantiations may contract FMAs differently: equal to FP32 rounding
    np.testing.assert_allclose(pot[0], both[0], rtol=1e-6)
    for k in (1, 2, 3):
        np.testing.assert_allclose(accel[k], both[k], rtol=1e-6, atol=1e-6 * np.max(np.abs(both[k])))


def test_origin_and_axis_points(E, orc):
    rng = np.random.default_rng(8)
    p = W.make_config(2, 400)
    x, y, z = p.x.copy(), p.y.copy(), p.z.copy()
    x[0] = y[0] = z[0] = 0.0                 # the origin
    x[1] = y[1] = 0.0; z[1] = 0.7            # on the z axis
    x[2] = y[2] = 0.0; z[2] = -2.5
    x[3], y[3], z[3] = 1e-7, -2e-7, 0.4      # next to the axis
    q = W.Particles(x, y, z, p.m)
    nmax, lmax = 6, 6
    rA, rB = orc.scf_coeffs(x, y, z, p.m, nmax, lmax)
    A, B = gpu_coeffs(E, q, nmax, lmax, FP64)
    assert acc.coeff_errors(A, B, rA, rB)["norm_rel"] < 3e-14
    for prec, tol in ((FP64, 1e-13), (MIXED, 1e-4)):
        pot, ax, ay, az = gpu_force(E, q, nmax, lmax, rA, rB, prec)
        rp, rx, ry, rz = orc.scf_force(x, y, z, nmax, lmax, rA, rB)
        assert np.all(np.isfinite(ax)) and np.all(np.isfinite(pot))
        scale = np.max(np.sqrt(rx ** 2 + ry ** 2 + rz ** 2))
        d = np.sqrt((ax - rx) ** 2 + (ay - ry) ** 2 + (az - rz) ** 2)
        assert np.max(d[:4]) < tol * scale
        assert np.max(acc.pot_rel_err(pot[:4], rp[:4])) < tol


def test_cfg1_full_size(E, orc):
    """N = 10^4 Hernquist sphere at (10,6): every coefficient and every particle."""
    p = W.make_config(1)
    rA, rB = orc.scf_coeffs(p.x, p.y, p.z, p.m, 10, 6)
    rp, rx, ry, rz = orc.scf_force(p.x, p.y, p.z, 10, 6, rA, rB)
    for prec in (FP64, MIXED, COMP32):
        A, B = gpu_coeffs(E, p, 10, 6, prec)
        ce = acc.coeff_errors(A, B, rA, rB)
        pot, ax, ay, az = gpu_force(E, p, 10, 6, A, B, prec)
        ef = report(f"cfg1 full prec{prec} force", acc.force_rel_err(ax, ay, az, rx, ry, rz))
        ep = report(f"cfg1 full prec{prec} pot", acc.pot_rel_err(pot, rp))
        if prec == FP64:  # measured: force max 3.4e-15, potential max 3.5e-15
            assert ce["norm_rel"] < 3e-14 and ef["max"] < 5e-14 and ep["max"] < 5e-14
        else:
            assert ef["median"] <= 1e-5 and ef["p99"] <= 1e-4 and ep["median"] <= 1e-5 and ep["p99"] <= 1e-4


def test_cfg3_full_size_sampled(E, orc):
    """N = 10^7 (Hernquist + offset Plummer) at (20,14): the coefficients over all
    particles against the oracle; forces on a seeded 10^5-particle sample."""
    import torch
    p = W.make_config(3)
    n = p.x.shape[0]
    rA, rB = orc.scf_coeffs(p.x, p.y, p.z, p.m, 20, 14)
    idx = np.sort(np.random.default_rng(33).choice(n, 100_000, replace=False))
    rp, rx, ry, rz = orc.scf_force(p.x[idx], p.y[idx], p.z[idx], 20, 14, rA, rB)
    x, y, z, m = dev(p.x, p.y, p.z, p.m)
    for prec in (FP64, COMP32, MIXED):
        A, B = E.etics_scf_coeffs(x, y, z, m, 20, 14, prec)
        pot, ax, ay, az = E.etics_scf_force(x, y, z, 20, 14, A, B, prec)
        A, B = host(A, B)
        ce = acc.coeff_errors(A, B, rA, rB)
        it = torch.from_numpy(idx).cuda()
        pot, ax, ay, az = (t[it].cpu().numpy() for t in (pot, ax, ay, az))
        ef = report(f"cfg3 sampled prec{prec} force", acc.force_rel_err(ax, ay, az, rx, ry, rz))
        ep = report(f"cfg3 sampled prec{prec} pot", acc.pot_rel_err(pot, rp))
        print(f"cfg3 prec{prec} coeff {ce}", flush=True)
        if prec == FP64:  # measured: coefficients 1.4e-14, force max 1.5e-14, pot max 1.2e-14
            assert ce["norm_rel"] < 1.5e-13 and ef["max"] < 1.5e-13 and ep["max"] < 1.5e-13
        else:
            assert ef["median"] <= 1e-5 and ef["p99"] <= 1e-4 and ep["median"] <= 1e-5 and ep["p99"] <= 1e-4
        del pot, ax, ay, az


def test_graph_capture_replays_match_eager(E):
    """etics_scf_coeffs + etics_scf_force captured into a graph (they allocate and
    synchronise nothing): every replay, with eager calls and synchronisations between
    the replays, gives the eager result bit for bit."""
    import torch
    p = W.make_config(2, 20_000)
    x, y, z, m = dev(p.x, p.y, p.z, p.m)
    nmax, lmax, n = 10, 10, p.x.shape[0]
    for prec in (MIXED, FP64):
        K = E.etics_coeff_count(nmax, lmax)
        ws = E.workspace(E.etics_scf_workspace_size(n, nmax, lmax, prec), "cuda")
        A, B = (torch.empty(K, dtype=torch.float64, device="cuda") for _ in range(2))
        outs = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(4)]

        def step():
            E.etics_scf_coeffs(x, y, z, m, nmax, lmax, prec, A, B, ws)
            E.etics_scf_force(x, y, z, nmax, lmax, A, B, prec, E.ETICS_POT_ACC, *outs, ws)

        step()  # eager reference (also sets the kernels' launch attributes before capture)
        torch.cuda.synchronize()
        ref = [t.clone() for t in [A, B, *outs]]
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step()
        for k in range(3):
            for t in [A, B, *outs]:
                t.fill_(float("nan"))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            for got, want in zip([A, B, *outs], ref):
                assert torch.equal(got, want), f"replay {k} differs (prec {prec})"
            step()  # eager work between replays
            torch.cuda.synchronize()
            for got, want in zip([A, B, *outs], ref):
                assert torch.equal(got, want)
