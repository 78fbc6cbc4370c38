"""Pins of the jerk / Hermite oracle (oracle/jerk.py) against things other than itself:
the independent C oracle, finite differences, a closed form and the integrator's order."""
import numpy as np
import pytest
import torch

from paper_1406_4254_amd import workloads as W


@pytest.fixture(scope="module")
def J(orc):
    from oracle import jerk
    return jerk


def rotated_set(n, seed):
    """Triaxial Hernquist sample, rotated and shifted so that no symmetry hides a term,
    with unequal masses."""
    p = W.make_config(2, n)
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    X = np.stack([p.x, p.y, p.z], 1) @ q.T + np.array([0.05, -0.03, 0.02])
    m = rng.uniform(0.5, 1.5, n)
    m /= m.sum()
    v = rng.normal(size=(n, 3)) * 0.4
    return X, v, m


def c_accel(orc, X, m, nmax, lmax):
    A, B = orc.scf_coeffs(X[:, 0], X[:, 1], X[:, 2], m, nmax, lmax)
    _, ax, ay, az = orc.scf_force(X[:, 0], X[:, 1], X[:, 2], nmax, lmax, A, B)
    return np.stack([ax, ay, az], 1), A, B


def test_torch_expansion_equals_c_oracle(orc, J):
    """The plain-torch expansion (coefficients, potential, -grad Phi by autodiff) equals
    the C oracle, an independent implementation (explicit recurrences, analytic force)."""
    X, v, m = rotated_set(700, 1)
    nmax, lmax = 7, 5
    P = torch.from_numpy(X)
    A, B = J.coeffs(P, torch.from_numpy(m), nmax, lmax)
    rA, rB = orc.scf_coeffs(X[:, 0], X[:, 1], X[:, 2], m, nmax, lmax)
    scale = np.max(np.abs(np.concatenate([rA, rB])))
    assert np.max(np.abs(A.numpy().ravel() - rA)) < 1e-13 * scale
    assert np.max(np.abs(B.numpy().ravel() - rB)) < 1e-13 * scale
    pot = J.potential(P, A, B, nmax, lmax).numpy()
    acc = J.acceleration(P, A, B, nmax, lmax).numpy()
    rp, rx, ry, rz = orc.scf_force(X[:, 0], X[:, 1], X[:, 2], nmax, lmax, rA, rB)
    np.testing.assert_allclose(pot, rp, rtol=1e-13)
    ref = np.stack([rx, ry, rz], 1)
    assert np.max(np.linalg.norm(acc - ref, axis=1) / np.linalg.norm(ref, axis=1)) < 1e-12


def test_jerk_equals_finite_differences_along_the_motion(orc, J):
    """j_i = d/dt a_i with every particle moving: fourth-order central differences of
    the C oracle's acceleration (coefficients recomputed at x + v t)."""
    X, v, m = rotated_set(600, 2)
    nmax, lmax = 6, 4
    a, j = J.accel_jerk(torch.from_numpy(X), torch.from_numpy(v), torch.from_numpy(m), nmax, lmax)
    h = 1e-4
    f = lambda t: c_accel(orc, X + v * t, m, nmax, lmax)[0]
    fd = (8.0 * (f(h) - f(-h)) - (f(2 * h) - f(-2 * h))) / (12.0 * h)
    err = np.linalg.norm(j.numpy() - fd, axis=1) / np.linalg.norm(fd, axis=1)
    assert np.median(err) < 1e-10 and np.max(err) < 1e-7
    np.testing.assert_allclose(a.numpy(), f(0.0), rtol=1e-11, atol=1e-13)


def test_coefficient_derivatives_equal_finite_differences(orc, J):
    X, v, m = rotated_set(800, 3)
    nmax, lmax = 8, 6
    A, B, dA, dB = J.coeffs_dot(torch.from_numpy(X), torch.from_numpy(v), torch.from_numpy(m), nmax, lmax)
    h = 1e-4

    def cf(t):
        Y = X + v * t
        return np.concatenate(orc.scf_coeffs(Y[:, 0], Y[:, 1], Y[:, 2], m, nmax, lmax))

    fd = (8.0 * (cf(h) - cf(-h)) - (cf(2 * h) - cf(-2 * h))) / (12.0 * h)
    got = np.concatenate([dA.numpy().ravel(), dB.numpy().ravel()])
    assert np.linalg.norm(got - fd) < 1e-9 * np.linalg.norm(fd)


def test_jerk_of_the_monopole_term_in_closed_form(J):
    """nmax = lmax = 0: a_i = -A(t) x_i / (r_i (1+r_i)^2) with A(t) = 3 sum_k m_k/(1+r_k)
    (Phi = -A/(1+r)), so j_i = -dA/dt x f - A (v f + x f'(r) dr/dt), f = 1/(r(1+r)^2),
    f' = -(1+3r)/(r^2 (1+r)^3), dA/dt = -3 sum m_k (dr_k/dt)/(1+r_k)^2."""
    X, v, m = rotated_set(300, 4)
    a, j = J.accel_jerk(torch.from_numpy(X), torch.from_numpy(v), torch.from_numpy(m), 0, 0)
    r = np.linalg.norm(X, axis=1)
    rd = np.sum(X * v, axis=1) / r
    A = 3.0 * np.sum(m / (1.0 + r))
    Ad = -3.0 * np.sum(m * rd / (1.0 + r) ** 2)
    f = 1.0 / (r * (1.0 + r) ** 2)
    fp = -(1.0 + 3.0 * r) / (r * r * (1.0 + r) ** 3)
    a_ref = -A * X * f[:, None]
    j_ref = -Ad * X * f[:, None] - A * (v * f[:, None] + X * (fp * rd)[:, None])
    np.testing.assert_allclose(a.numpy(), a_ref, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(j.numpy(), j_ref, rtol=1e-12, atol=1e-14 * np.max(np.abs(j_ref)))


def _hermite_energy_error(J, X, v, m, nmax, lmax, T, dt):
    P, V, M = torch.from_numpy(X), torch.from_numpy(v), torch.from_numpy(m)
    e0 = J.energy(P, V, M, nmax, lmax)
    P1, V1 = J.hermite(P, V, M, nmax, lmax, dt, int(round(T / dt)))
    return abs(J.energy(P1, V1, M, nmax, lmax) / e0 - 1.0)


def test_hermite_energy_error_is_fourth_order(J):
    """The SCF forces derive from W = 1/2 sum m Phi, so the energy is conserved in
    continuous time; the Hermite scheme's energy error over a fixed time falls ~16x per
    halving of dt (fourth order), where a second-order scheme would give ~4x."""
    # a cored (Plummer, scale 1.5) sample in the Hernquist-Ostriker expansion, so the
    # shortest orbital time is long against the steps
    rng = np.random.default_rng(7)
    x, y, z = W.sphere(rng, 200, "plummer", 1.5)
    X = np.stack([x, y, z], 1)
    m = np.full(200, 1.0 / 200)
    v = rng.normal(size=X.shape) * 0.3
    errs = [_hermite_energy_error(J, X, v, m, 4, 2, 0.4, dt) for dt in (0.05, 0.025, 0.0125)]
    ratios = [errs[k] / errs[k + 1] for k in range(2)]
    print("hermite energy errors", errs, "ratios", ratios)
    assert errs[-1] < 1e-9
    for q in ratios:
        assert 12.0 < q < 28.0


def test_hermite_one_step_by_hand(J):
    """One step equals the predictor-corrector written out from accelerations and jerks
    of the C-oracle-pinned expansion (checks the stage order and time levels)."""
    X, v, m = rotated_set(150, 9)
    P, V, M = torch.from_numpy(X), torch.from_numpy(v), torch.from_numpy(m)
    dt = 0.03
    a0, j0 = J.accel_jerk(P, V, M, 5, 3)
    Pp = P + V * dt + a0 * dt ** 2 / 2 + j0 * dt ** 3 / 6
    Vp = V + a0 * dt + j0 * dt ** 2 / 2
    a1, j1 = J.accel_jerk(Pp, Vp, M, 5, 3)
    V1 = V + (a0 + a1) * dt / 2 + (j0 - j1) * dt ** 2 / 12
    P1 = P + (V + V1) * dt / 2 + (a0 - a1) * dt ** 2 / 12
    P2, V2 = J.hermite(P, V, M, 5, 3, dt, 1)
    assert torch.equal(P1, P2) and torch.equal(V1, V2)
