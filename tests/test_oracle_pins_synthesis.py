"""Pins of the oracle's SCF synthesis, its leapfrog and its direct summation (CPU only).

The SCF potential is pinned against a brute force that uses no spherical harmonic,
no coefficient array and none of the oracle's code: by the addition theorem
(Section 2.4, eq. scf-phi) the expansion of the field of N particles is

  Phi(x) = sum_k m_k sum_{n,l} Atilde_nl PhiT_nl(r_k) PhiT_nl(r) (2l+1)/(4 pi) P_l(cos g_k),

with g_k the angle between x and particle k and P_l the Legendre polynomial.  Every
sign, (2 - delta_m0) factor and (cos, sin) pairing of the real-form synthesis has to
come out right for the two to agree.  The leapfrog (Section 3.4) is pinned by a
kick-drift-kick composed here from the oracle's coefficient and force calls, and by
the second-order decay of its energy error: SCF forces derive from the potential
energy W = (1/2) sum_i m_i Phi(x_i) = (1/2) sum_nlm (A^2 + B^2) / ((2 - delta_m0)
Atilde_nl), so the total energy of a system is conserved in continuous time.
"""
import math

import numpy as np
import pytest
from scipy import special
from scipy.spatial.transform import Rotation

from paper_1406_4254_amd import accuracy as acc
from paper_1406_4254_amd import workloads as W


def lmi(l, m):
    return l * (l + 1) // 2 + m


def cidx(n, l, m, lmax):
    return n * (lmax + 1) * (lmax + 2) // 2 + lmi(l, m)


# ------------------------------------------------ brute force by the addition theorem
def anl_tilde_closed_form(n, l):
    """1 / I_nl of the Hernquist-Ostriker basis (Section 2.5), from gamma functions."""
    knl = 0.5 * n * (n + 4 * l + 3) + (l + 1) * (2 * l + 1)
    log_i = (math.log(4 * math.pi * knl) - (8 * l + 6) * math.log(2.0) + special.gammaln(n + 4 * l + 3)
             - special.gammaln(n + 1) - math.log(n + 2 * l + 1.5) - 2 * special.gammaln(2 * l + 1.5))
    return -math.exp(-log_i)


def radial_table(r, nmax, lmax):
    """PhiT_nl(r) for an array of radii, shape [nmax+1, lmax+1, len(r)], from scipy's
    Gegenbauer polynomials."""
    r = np.asarray(r, dtype=np.float64)
    xi = (r - 1.0) / (r + 1.0)
    out = np.zeros((nmax + 1, lmax + 1, r.size))
    for l in range(lmax + 1):
        pref = -math.sqrt(4 * math.pi) * r ** l / (1.0 + r) ** (2 * l + 1)
        for n in range(nmax + 1):
            out[n, l] = pref * special.eval_gegenbauer(n, 2 * l + 1.5, xi)
    return out


def brute_potential(src, mass, fld, nmax, lmax):
    """Phi at field points fld [3, nf] of the particles src [3, N] with masses mass."""
    rs = np.linalg.norm(src, axis=0)
    rf = np.linalg.norm(fld, axis=0)
    cosg = (fld.T @ src) / np.outer(rf, rs)
    cosg = np.clip(cosg, -1.0, 1.0)
    ps, pf = radial_table(rs, nmax, lmax), radial_table(rf, nmax, lmax)
    at = np.array([[anl_tilde_closed_form(n, l) for l in range(lmax + 1)] for n in range(nmax + 1)])
    pot = np.zeros(fld.shape[1])
    for l in range(lmax + 1):
        # G_l(f, k) = sum_n Atilde_nl PhiT_nl(r_k) PhiT_nl(r_f)
        g = np.einsum("n,nf,nk->fk", at[:, l], pf[:, l], ps[:, l])
        pot += (2 * l + 1) / (4 * math.pi) * np.sum(g * special.eval_legendre(l, cosg) * mass[None, :],
                                                    axis=1)
    return pot


def _rotated_triaxial(n, seed):
    p = W.triaxial_hernquist(n, seed)
    R = Rotation.random(random_state=seed).as_matrix()
    v = R @ np.vstack([p.x, p.y, p.z]) + np.array([[0.05], [-0.03], [0.02]])
    rng = np.random.default_rng(seed + 1)
    m = p.m * rng.uniform(0.5, 1.5, n)  # unequal masses
    return v, m


def _field_points(seed, nf=40):
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(3, nf))
    d /= np.linalg.norm(d, axis=0)
    return d * 10.0 ** rng.uniform(-1.2, 0.8, nf)


@pytest.mark.parametrize("nmax,lmax", [(0, 3), (4, 4), (6, 7), (3, 10)])
def test_scf_potential_equals_addition_theorem_sum(orc, nmax, lmax):
    """The oracle's coefficients followed by its synthesis give the brute-force sum, at
    field points and at the particles themselves (a rotated, shifted triaxial set with
    unequal masses, so every m and both cos and sin terms are populated)."""
    src, m = _rotated_triaxial(300, 31)
    A, B = orc.scf_coeffs(src[0], src[1], src[2], m, nmax, lmax)
    assert np.max(np.abs(B)) > 1e-3 * np.max(np.abs(A))  # sin terms really present
    for fld in (_field_points(32), src[:, :50]):
        pot = orc.scf_force(fld[0], fld[1], fld[2], nmax, lmax, A, B)[0]
        ref = brute_potential(src, m, fld, nmax, lmax)
        np.testing.assert_allclose(pot, ref, rtol=1e-11, atol=1e-13 * np.max(np.abs(ref)))


def test_scf_force_is_gradient_of_addition_theorem_sum(orc):
    """a = -grad of the brute-force potential (central differences), so the force
    synthesis is pinned without the oracle's own potential."""
    nmax, lmax = 5, 6
    src, m = _rotated_triaxial(250, 33)
    A, B = orc.scf_coeffs(src[0], src[1], src[2], m, nmax, lmax)
    fld = _field_points(34, 25)
    _, ax, ay, az = orc.scf_force(fld[0], fld[1], fld[2], nmax, lmax, A, B)
    got = np.vstack([ax, ay, az])
    h = 1e-5
    for d in range(3):
        fp = fld.copy(); fp[d] += h
        fm = fld.copy(); fm[d] -= h
        fd = -(brute_potential(src, m, fp, nmax, lmax) - brute_potential(src, m, fm, nmax, lmax)) / (2 * h)
        np.testing.assert_allclose(got[d], fd, rtol=2e-7, atol=2e-7 * np.max(np.abs(got)))


def test_scf_energy_identity(orc):
    """sum_i m_i Phi(x_i) = sum_nlm (A^2 + B^2) / ((2 - delta_m0) Atilde_nl): the
    coefficients and the synthesis agree on every (cos, sin) pair and factor."""
    nmax, lmax = 8, 8
    src, m = _rotated_triaxial(2000, 35)
    A, B = orc.scf_coeffs(src[0], src[1], src[2], m, nmax, lmax)
    pot = orc.scf_force(src[0], src[1], src[2], nmax, lmax, A, B)[0]
    lhs = float(np.sum(m * pot))
    rhs = 0.0
    for n in range(nmax + 1):
        for l in range(lmax + 1):
            at = anl_tilde_closed_form(n, l)
            for mm in range(l + 1):
                k = cidx(n, l, mm, lmax)
                rhs += (A[k] ** 2 + B[k] ** 2) / ((1 if mm == 0 else 2) * at)
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_scf_rotation_covariance(orc):
    """Rotating the particles and the field points together leaves Phi unchanged and
    rotates a."""
    nmax, lmax = 6, 8
    src, m = _rotated_triaxial(800, 37)
    fld = _field_points(38, 30)
    A, B = orc.scf_coeffs(src[0], src[1], src[2], m, nmax, lmax)
    p0, *a0 = orc.scf_force(fld[0], fld[1], fld[2], nmax, lmax, A, B)
    R = Rotation.random(random_state=39).as_matrix()
    s2, f2 = R @ src, R @ fld
    A2, B2 = orc.scf_coeffs(s2[0], s2[1], s2[2], m, nmax, lmax)
    p1, *a1 = orc.scf_force(f2[0], f2[1], f2[2], nmax, lmax, A2, B2)
    np.testing.assert_allclose(p1, p0, rtol=1e-11)
    ra = R @ np.vstack(a0)
    np.testing.assert_allclose(np.vstack(a1), ra, rtol=1e-9, atol=1e-11 * np.max(np.abs(ra)))


# --------------------------------------------------------------------- leapfrog
def _small_systems():
    return W.batched_systems(nsys=2, seed=23, nlog=(2.4, 2.6))


def test_leapfrog_equals_kdk_from_oracle_calls(orc):
    """One and two leapfrog steps equal v += dt/2 a(x); x += dt v; v += dt/2 a(x),
    composed here from the oracle's coefficient and force calls, per system."""
    p = _small_systems()
    nmax, lmax, dt = 4, 3, 0.02
    for steps in (1, 2):
        got = orc.leapfrog_scf(p.x, p.y, p.z, p.vx, p.vy, p.vz, p.m, p.offsets, nmax, lmax, dt, steps)
        st = [a.copy() for a in (p.x, p.y, p.z, p.vx, p.vy, p.vz)]
        for s in range(len(p.offsets) - 1):
            sl = slice(p.offsets[s], p.offsets[s + 1])
            x, y, z, vx, vy, vz = (a[sl] for a in st)
            m = p.m[sl]

            def accel():
                A, B = orc.scf_coeffs(x, y, z, m, nmax, lmax)
                return orc.scf_force(x, y, z, nmax, lmax, A, B)[1:]

            for _ in range(steps):
                g = accel()
                for v, gc in zip((vx, vy, vz), g):
                    v += 0.5 * dt * gc
                for q, v in zip((x, y, z), (vx, vy, vz)):
                    q += dt * v
                g = accel()
                for v, gc in zip((vx, vy, vz), g):
                    v += 0.5 * dt * gc
        for a, b in zip(got, st):
            np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-15)


def system_energy(orc, x, y, z, vx, vy, vz, m, nmax, lmax):
    """Kinetic energy plus W = (1/2) sum_i m_i Phi(x_i) of one system."""
    A, B = orc.scf_coeffs(x, y, z, m, nmax, lmax)
    pot = orc.scf_force(x, y, z, nmax, lmax, A, B)[0]
    return 0.5 * np.sum(m * (vx * vx + vy * vy + vz * vz)) + 0.5 * np.sum(m * pot)


def test_leapfrog_energy_error_is_second_order(orc):
    """The energy error after a fixed time falls about fourfold per halving of dt."""
    p = W.batched_systems(nsys=1, seed=25, nlog=(2.7, 2.7))
    nmax, lmax, T = 4, 2, 0.32
    e0 = system_energy(orc, p.x, p.y, p.z, p.vx, p.vy, p.vz, p.m, nmax, lmax)
    errs = []
    for dt in (0.04, 0.02, 0.01, 0.005):
        s = orc.leapfrog_scf(p.x, p.y, p.z, p.vx, p.vy, p.vz, p.m, p.offsets, nmax, lmax, dt,
                             int(round(T / dt)))
        errs.append(abs(system_energy(orc, *s, p.m, nmax, lmax) - e0) / abs(e0))
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    print("energy errors", errs, "ratios", ratios)
    assert errs[-1] < 1e-4
    for q in ratios[1:]:
        assert 3.0 < q < 5.5


# ------------------------------------------------------------------ direct summation
def test_direct_force_is_minus_gradient(orc):
    """The direct-summation force on particle i is -grad of its potential with respect
    to its own position (central differences, the other particles fixed)."""
    p = W.plummer_hernquist_mix(200, 43)
    pot, ax, ay, az = orc.direct(p.x, p.y, p.z, p.m)
    got = np.vstack([ax, ay, az])
    for i in (0, 17, 99, 150):
        h = 1e-6 * max(1e-3, math.sqrt(p.x[i] ** 2 + p.y[i] ** 2 + p.z[i] ** 2))
        fd = []
        for d, arr in enumerate((p.x, p.y, p.z)):
            vals = []
            for sgn in (1, -1):
                q = [p.x.copy(), p.y.copy(), p.z.copy()]
                q[d][i] += sgn * h
                vals.append(orc.direct(q[0], q[1], q[2], p.m)[0][i])
            fd.append(-(vals[0] - vals[1]) / (2 * h))
        np.testing.assert_allclose(got[:, i], fd, rtol=1e-6, atol=1e-6 * np.linalg.norm(got[:, i]))


def test_direct_potential_of_a_pair_and_a_triangle(orc):
    """Closed forms: two unit-separated particles, and an equilateral triangle."""
    pot, ax, ay, az = orc.direct(np.array([0.0, 1.0]), np.zeros(2), np.zeros(2), np.array([2.0, 3.0]))
    np.testing.assert_allclose(pot, [-3.0, -2.0], rtol=1e-15)
    np.testing.assert_allclose(ax, [3.0, -2.0], rtol=1e-15)
    s = 0.7
    x = np.array([0.0, s, s / 2])
    y = np.array([0.0, 0.0, s * math.sqrt(3) / 2])
    pot, ax, ay, az = orc.direct(x, y, np.zeros(3), np.ones(3))
    np.testing.assert_allclose(pot, -2.0 / s, rtol=1e-14)
    c = np.array([s / 2, s * math.sqrt(3) / 6])
    for i in range(3):
        d = c - np.array([x[i], y[i]])
        np.testing.assert_allclose([ax[i], ay[i]], math.sqrt(3) / s ** 2 * d / np.linalg.norm(d), rtol=1e-13)


# ------------------------------------------------- rounding of the oracle's own sums
def test_long_double_sums_agree_with_plain_oracle(orc):
    """The oracle built with long-double running sums is the same computation: at small
    N both agree to a few units of FP64 rounding, so the long-double build measures only the rounding of
    the plain oracle's sequential sums."""
    p = W.make_config(4, 500)
    a = orc.mex_force(p.x, p.y, p.z, p.m, 8)
    b = orc.mex_force(p.x, p.y, p.z, p.m, 8, ext=True)
    assert np.max(acc.force_rel_err(*a[1:], *b[1:])) < 1e-14
    assert np.max(acc.pot_rel_err(a[0], b[0])) < 1e-14
    q = W.make_config(2, 500)
    A, B = orc.scf_coeffs(q.x, q.y, q.z, q.m, 10, 10)
    A2, B2 = orc.scf_coeffs(q.x, q.y, q.z, q.m, 10, 10, ext=True)
    assert acc.coeff_errors(A, B, A2, B2)["norm_rel"] < 1e-14
    f = orc.scf_force(q.x, q.y, q.z, 10, 10, A2, B2)
    g = orc.scf_force(q.x, q.y, q.z, 10, 10, A2, B2, ext=True)
    assert np.max(acc.force_rel_err(*f[1:], *g[1:])) < 1e-13


@pytest.mark.slow
def test_oracle_mex_rounding_grows_with_n(orc):
    """The plain oracle's MEX sums are sequential over all particles, so their rounding
    grows with N: measured against the long-double build (numbers kept as the basis
    of the FP64 GPU parity bounds)."""
    out = {}
    for n in (10_000, 100_000):
        p = W.make_config(4, n)
        a = orc.mex_force(p.x, p.y, p.z, p.m, 10)
        b = orc.mex_force(p.x, p.y, p.z, p.m, 10, ext=True)
        out[n] = acc.summarize(acc.force_rel_err(*a[1:], *b[1:]))
    print(out)
    assert out[100_000]["max"] < 5e-12
    assert out[100_000]["median"] > out[10_000]["median"]
