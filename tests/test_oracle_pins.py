"""Pins of the FP64 oracle to things other than itself (CPU only).

Each test checks a part of the oracle against a closed form, a library routine,
an exact identity, an invariant or brute force, chosen so that a dropped term, a
wrong sign or index, or a transposed operand in that part fails here.
"""
import json
import math
import os

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg
from scipy import special
from scipy.spatial.transform import Rotation

from paper_1406_4254_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def lmi(l, m):
    return l * (l + 1) // 2 + m


def cidx(n, l, m, lmax):
    return n * (lmax + 1) * (lmax + 2) // 2 + lmi(l, m)


# ----------------------------------------------------------------- Gegenbauer
@pytest.mark.parametrize("alpha", [0.5, 1.5, 2.5, 21.5, 29.5])
def test_gegenbauer_closed_forms(orc, alpha):
    a = alpha
    for x in np.linspace(-1.0, 1.0, 11):
        c = orc.gegenbauer(3, a, x)
        ref = [1.0, 2 * a * x, 2 * a * (a + 1) * x ** 2 - a,
               4.0 / 3.0 * a * (a + 1) * (a + 2) * x ** 3 - 2 * a * (a + 1) * x]
        scale = max(1.0, np.max(np.abs(ref)))
        np.testing.assert_allclose(c, ref, rtol=1e-13, atol=1e-13 * scale)


@pytest.mark.parametrize("alpha", [1.5, 9.5, 21.5, 29.5])
def test_gegenbauer_at_one_is_binomial(orc, alpha):
    c = orc.gegenbauer(20, alpha, 1.0)
    ref = [math.exp(math.lgamma(n + 2 * alpha) - math.lgamma(n + 1) - math.lgamma(2 * alpha))
           for n in range(21)]
    np.testing.assert_allclose(c, ref, rtol=1e-12)


def test_gegenbauer_half_is_legendre(orc):
    for x in np.linspace(-1, 1, 13):
        c = orc.gegenbauer(12, 0.5, x)
        ref = [npleg.legval(x, [0] * n + [1]) for n in range(13)]
        np.testing.assert_allclose(c, ref, rtol=1e-12, atol=1e-14)


def test_gegenbauer_matches_scipy(orc):
    rng = np.random.default_rng(11)
    for _ in range(40):
        a = 2 * rng.integers(0, 15) + 1.5
        x = rng.uniform(-1, 1)
        c = orc.gegenbauer(20, a, x)
        ref = np.array([special.eval_gegenbauer(n, a, x) for n in range(21)])
        np.testing.assert_allclose(c, ref, rtol=1e-10, atol=1e-10 * np.max(np.abs(ref)))


# ------------------------------------------------------------------- Legendre
def test_ylm_closed_forms(orc):
    for th in [0.1, 0.7, 1.3, 2.0, 3.0]:
        Y = orc.ylm(2, th)
        s, c = math.sin(th), math.cos(th)
        assert Y[lmi(0, 0)] == pytest.approx(1 / math.sqrt(4 * math.pi), rel=1e-15)
        assert Y[lmi(1, 0)] == pytest.approx(math.sqrt(3 / (4 * math.pi)) * c, rel=1e-14, abs=1e-16)
        assert Y[lmi(1, 1)] == pytest.approx(-math.sqrt(3 / (8 * math.pi)) * s, rel=1e-14)  # CS phase
        assert Y[lmi(2, 0)] == pytest.approx(math.sqrt(5 / (4 * math.pi)) * (3 * c * c - 1) / 2,
                                             rel=1e-13, abs=1e-16)
        assert Y[lmi(2, 2)] == pytest.approx(math.sqrt(15 / (32 * math.pi)) * s * s, rel=1e-13)


def test_ylm_matches_scipy(orc):
    for th in np.linspace(1e-4, math.pi - 1e-4, 17):
        Y = orc.ylm(14, th)
        for l in range(15):
            for m in range(l + 1):
                ref = special.sph_harm_y(l, m, th, 0.0).real
                assert abs(Y[lmi(l, m)] - ref) <= 1e-12 * max(1.0, abs(ref)), (l, m, th)


def test_unsold(orc):
    for th in np.linspace(0.0, math.pi, 9):
        Y = orc.ylm(14, th)
        for l in range(15):
            s = sum((1 if m == 0 else 2) * Y[lmi(l, m)] ** 2 for m in range(l + 1))
            assert s == pytest.approx((2 * l + 1) / (4 * math.pi), rel=1e-12)


def test_ylm_orthonormal_quadrature(orc):
    L = 12
    mu, w = npleg.leggauss(40)
    Ys = np.array([orc.ylm(L, math.acos(x)) for x in mu])
    for m in range(L + 1):
        for l in range(m, L + 1):
            for l2 in range(m, L + 1):
                v = 2 * math.pi * np.sum(w * Ys[:, lmi(l, m)] * Ys[:, lmi(l2, m)])
                assert v == pytest.approx(1.0 if l == l2 else 0.0, abs=1e-12)


def test_paper_m_recursion_pins_phase(orc):
    """The azimuthal recursion printed in Section 4.2 (read as one sum) holds for the
    oracle's unnormalised functions only with the Condon-Shortley phase."""
    L = 10
    for th in [0.4, 1.1, 2.2]:
        Y = orc.ylm(L, th)
        P = {}
        for l in range(L + 1):
            for m in range(l + 1):
                N = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m) / math.factorial(l + m))
                P[l, m] = Y[lmi(l, m)] / N
        cot = math.cos(th) / math.sin(th)
        for l in range(2, L + 1):
            for m in range(2, l + 1):
                rhs = -2 * (m - 1) * cot * P[l, m - 1] - (l + m - 1) * (l - m + 2) * P[l, m - 2]
                assert P[l, m] == pytest.approx(rhs, rel=1e-10, abs=1e-10 * abs(P[l, m - 2]))


def test_ylm_derivatives_fd(orc):
    L = 12
    h = 1e-6
    for th in [1e-3, 0.3, 1.0, 1.9, 3.1]:
        Y, dY, mYs = orc.ylm_deriv(L, th)
        Yp, Ym = orc.ylm(L, th + h), orc.ylm(L, th - h)
        np.testing.assert_allclose(dY, (Yp - Ym) / (2 * h), rtol=1e-6, atol=1e-8)
        for l in range(L + 1):
            for m in range(l + 1):
                assert mYs[lmi(l, m)] == pytest.approx(m * Y[lmi(l, m)] / math.sin(th), rel=1e-9,
                                                       abs=1e-12)


# --------------------------------------------------------------- radial basis
def test_anl_tilde_00_is_minus_three(orc):
    assert orc.anl_tilde(0, 0) == pytest.approx(-3.0, rel=1e-14)


@pytest.mark.parametrize("r", [0.05, 0.4, 1.0, 3.0, 17.0])
def test_radial_derivative_fd(orc, r):
    h = 1e-6 * r
    phi, dphi = orc.phi_nl(10, 10, r)
    pp, _ = orc.phi_nl(10, 10, r + h)
    pm, _ = orc.phi_nl(10, 10, r - h)
    np.testing.assert_allclose(dphi, (pp - pm) / (2 * h), rtol=1e-6,
                               atol=1e-8 * np.max(np.abs(dphi)))


@pytest.mark.parametrize("r", [0.1, 0.7, 2.0, 6.0])
def test_poisson_pairs(orc, r):
    """(1/r^2) d/dr (r^2 PhiT') - l(l+1) PhiT / r^2 = 4 pi rhoT for every (n, l)."""
    nmax, lmax = 8, 8
    h = 1e-5 * r
    phi, _ = orc.phi_nl(nmax, lmax, r)
    _, dp = orc.phi_nl(nmax, lmax, r + h)
    _, dm = orc.phi_nl(nmax, lmax, r - h)
    d2 = ((r + h) ** 2 * dp - (r - h) ** 2 * dm) / (2 * h) / r ** 2
    ls = np.arange(lmax + 1)[None, :]
    lap = d2 - ls * (ls + 1) * phi / r ** 2
    rho = orc.rho_nl(nmax, lmax, r)
    np.testing.assert_allclose(lap, 4 * math.pi * rho, rtol=2e-6,
                               atol=1e-7 * np.max(np.abs(4 * math.pi * rho)))


def test_biorthogonality_quadrature(orc):
    """int rhoT_nl PhiT_n'l r^2 dr = delta_nn' / Atilde_nl, by Gauss-Legendre in xi."""
    nmax, lmax = 10, 10
    xi, w = npleg.leggauss(60)
    rho = np.zeros((len(xi), nmax + 1, lmax + 1))
    phi = np.zeros_like(rho)
    jac = np.zeros(len(xi))
    for k, x in enumerate(xi):
        r = (1 + x) / (1 - x)
        rho[k] = orc.rho_nl(nmax, lmax, r)
        phi[k] = orc.phi_nl(nmax, lmax, r)[0]
        jac[k] = w[k] * r * r * 2.0 / (1 - x) ** 2
    for l in range(lmax + 1):
        for n in range(nmax + 1):
            for n2 in range(nmax + 1):
                v = np.sum(jac * rho[:, n, l] * phi[:, n2, l])
                if n == n2:
                    assert v * orc.anl_tilde(n, l) == pytest.approx(1.0, rel=1e-11)
                else:
                    assert abs(v * orc.anl_tilde(n, l)) < 1e-11


# ------------------------------------------------------- coefficient pipeline
@pytest.mark.parametrize("target", [(0, 0, 0, "c"), (2, 1, 1, "c"), (1, 2, 1, "s"), (3, 3, 3, "s"),
                                    (4, 4, 2, "c"), (0, 3, 0, "c"), (2, 4, 4, "c")])
def test_unit_coefficient_quadrature(orc, target):
    """Signed masses that sample rhoT_{n0 l0} Ybar_{l0 m0} cos/sin(m0 phi) exactly by
    quadrature return exactly one unit coefficient and zero for all others."""
    n0, l0, m0, cs = target
    nmax = lmax = 4
    xi, wx = npleg.leggauss(24)
    mu, wm = npleg.leggauss(12)
    nph = 12
    ph = 2 * math.pi * np.arange(nph) / nph
    X, Y, Z, M = [], [], [], []
    for a, x in enumerate(xi):
        r = (1 + x) / (1 - x)
        jr = wx[a] * r * r * 2.0 / (1 - x) ** 2 * orc.rho_nl(nmax, lmax, r)[n0, l0]
        for b, c in enumerate(mu):
            th = math.acos(c)
            yl = orc.ylm(lmax, th)[lmi(l0, m0)]
            s = math.sqrt(1 - c * c)
            for p in ph:
                trig = math.cos(m0 * p) if cs == "c" else math.sin(m0 * p)
                X.append(r * s * math.cos(p)); Y.append(r * s * math.sin(p)); Z.append(r * c)
                M.append(jr * wm[b] * (2 * math.pi / nph) * yl * trig)
    A, B = orc.scf_coeffs(np.array(X), np.array(Y), np.array(Z), np.array(M), nmax, lmax)
    k = cidx(n0, l0, m0, lmax)
    ea, eb = np.zeros_like(A), np.zeros_like(B)
    (ea if cs == "c" else eb)[k] = 1.0
    np.testing.assert_allclose(A, ea, atol=1e-11)
    np.testing.assert_allclose(B, eb, atol=1e-11)


def test_hernquist_00_exact(orc):
    """nmax = lmax = 0: A_000 = 3 sum m/(1+r); Phi = -A/(1+r); a = -A x / (r (1+r)^2)."""
    p = W.hernquist_sphere(2000, 101)
    r = np.sqrt(p.x ** 2 + p.y ** 2 + p.z ** 2)
    A, B = orc.scf_coeffs(p.x, p.y, p.z, p.m, 0, 0)
    a0 = 3.0 * np.sum(p.m / (1 + r))
    assert A[0] == pytest.approx(a0, rel=1e-13)
    assert B[0] == 0.0
    pot, ax, ay, az = orc.scf_force(p.x, p.y, p.z, 0, 0, A, B)
    np.testing.assert_allclose(pot, -A[0] / (1 + r), rtol=1e-13)
    f = -A[0] / (r * (1 + r) ** 2)
    np.testing.assert_allclose(ax, f * p.x, rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(ay, f * p.y, rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(az, f * p.z, rtol=1e-12, atol=1e-300)


def test_hernquist_stratified_monopole(orc):
    """Stratified Hernquist radii: A_000 -> M = 1 with O(N^-1.5) error and A_n00 -> 0
    for n >= 1 (biorthogonality of the basis against its zeroth density)."""
    n = 10000
    u = (np.arange(n) + 0.5) / n
    r = W.hernquist_radii(u)
    rng = np.random.default_rng(3)
    ct = rng.uniform(-1, 1, n)
    ph = rng.uniform(0, 2 * math.pi, n)
    st = np.sqrt(1 - ct * ct)
    x, y, z = r * st * np.cos(ph), r * st * np.sin(ph), r * ct
    A, B = orc.scf_coeffs(x, y, z, np.full(n, 1.0 / n), 6, 0)
    assert abs(A[0] - 1.0) < 5 * n ** -1.5
    assert np.all(np.abs(A[1:]) < 2e-5)


def _odd_l_mask(nmax, lmax, pred):
    mask = np.zeros((nmax + 1) * (lmax + 1) * (lmax + 2) // 2, dtype=bool)
    for n in range(nmax + 1):
        for l in range(lmax + 1):
            for m in range(l + 1):
                mask[cidx(n, l, m, lmax)] = pred(l, m)
    return mask


def test_mirror_symmetries(orc):
    nmax, lmax = 4, 6
    p = W.triaxial_hernquist(300, 7)
    x, y, z, m = p.x, p.y, p.z, p.m
    cat = np.concatenate
    A0, _ = orc.scf_coeffs(x, y, z, m, nmax, lmax)
    tol = 1e-14 * np.max(np.abs(A0))
    # point reflection: odd l vanish
    A, B = orc.scf_coeffs(cat([x, -x]), cat([y, -y]), cat([z, -z]), cat([m, m]), nmax, lmax)
    odd = _odd_l_mask(nmax, lmax, lambda l, mm: l % 2 == 1)
    assert np.all(np.abs(A[odd]) < tol) and np.all(np.abs(B[odd]) < tol)
    assert np.max(np.abs(A[~odd])) > 1e3 * tol
    # z mirror: l + m odd vanish
    A, B = orc.scf_coeffs(cat([x, x]), cat([y, y]), cat([z, -z]), cat([m, m]), nmax, lmax)
    lm_odd = _odd_l_mask(nmax, lmax, lambda l, mm: (l + mm) % 2 == 1)
    assert np.all(np.abs(A[lm_odd]) < tol) and np.all(np.abs(B[lm_odd]) < tol)
    # y mirror: every B vanishes
    A, B = orc.scf_coeffs(cat([x, x]), cat([y, -y]), cat([z, z]), cat([m, m]), nmax, lmax)
    assert np.all(np.abs(B) < tol)
    # x mirror: odd m vanish in A, even m vanish in B
    A, B = orc.scf_coeffs(cat([x, -x]), cat([y, y]), cat([z, z]), cat([m, m]), nmax, lmax)
    m_odd = _odd_l_mask(nmax, lmax, lambda l, mm: mm % 2 == 1)
    assert np.all(np.abs(A[m_odd]) < tol) and np.all(np.abs(B[~m_odd]) < tol)


def _power(A, B, nmax, lmax):
    P = np.zeros((nmax + 1, lmax + 1))
    for n in range(nmax + 1):
        for l in range(lmax + 1):
            k0 = cidx(n, l, 0, lmax)
            P[n, l] = A[k0] ** 2 + 0.5 * np.sum(A[k0 + 1:k0 + l + 1] ** 2 + B[k0 + 1:k0 + l + 1] ** 2)
    return P


def test_rotation_invariant_power(orc):
    nmax, lmax = 6, 8
    p = W.triaxial_hernquist(2000, 9)
    P0 = _power(*orc.scf_coeffs(p.x, p.y, p.z, p.m, nmax, lmax), nmax, lmax)
    R = Rotation.random(random_state=4).as_matrix()
    v = R @ np.vstack([p.x, p.y, p.z])
    P1 = _power(*orc.scf_coeffs(v[0], v[1], v[2], p.m, nmax, lmax), nmax, lmax)
    np.testing.assert_allclose(P1, P0, rtol=1e-10, atol=1e-14 * np.max(P0))


# -------------------------------------------------------------- force synthesis
def _random_coeffs(rng, nmax, lmax):
    K = (nmax + 1) * (lmax + 1) * (lmax + 2) // 2
    A = rng.normal(size=K)
    B = rng.normal(size=K)
    for n in range(nmax + 1):
        for l in range(lmax + 1):
            B[cidx(n, l, 0, lmax)] = 0.0
    return A, B


def test_force_is_minus_gradient(orc):
    rng = np.random.default_rng(5)
    nmax, lmax = 5, 6
    A, B = _random_coeffs(rng, nmax, lmax)
    pts = rng.normal(size=(3, 25)) * rng.uniform(0.05, 4.0, size=25)
    pts[:, 0] = [1e-9, 2e-9, 0.7]     # next to the z axis
    pts[:, 1] = [0.0, 0.0, -1.3]      # on the z axis
    pot, ax, ay, az = orc.scf_force(pts[0], pts[1], pts[2], nmax, lmax, A, B)
    acc = np.vstack([ax, ay, az])
    for d in range(3):
        h = 1e-6
        pp = pts.copy(); pp[d] += h
        pm = pts.copy(); pm[d] -= h
        fd = -(orc.scf_force(*pp, nmax, lmax, A, B)[0] - orc.scf_force(*pm, nmax, lmax, A, B)[0]) / (2 * h)
        np.testing.assert_allclose(acc[d], fd, rtol=1e-6, atol=1e-6 * np.max(np.abs(acc)))


def test_force_at_origin_convention(orc):
    """At r = 0 the l = 0 radial force has no direction and is 0; l = 1 gives a finite
    uniform field, equal to the limit from nearby points."""
    rng = np.random.default_rng(6)
    nmax, lmax = 3, 3
    A, B = _random_coeffs(rng, nmax, lmax)
    for n in range(nmax + 1):
        A[cidx(n, 0, 0, lmax)] = 0.0       # remove the cusp of the l = 0 terms
    o = orc.scf_force(np.zeros(1), np.zeros(1), np.zeros(1), nmax, lmax, A, B)
    e = 1e-9
    near = orc.scf_force(np.array([e]), np.array([0.3 * e]), np.array([-0.2 * e]), nmax, lmax, A, B)
    assert o[0][0] == 0.0 and abs(near[0][0]) < 1e-6
    for k in range(1, 4):
        assert o[k][0] == pytest.approx(near[k][0], rel=1e-6, abs=1e-12)


# ------------------------------------------------------------------------ MEX
@pytest.mark.parametrize("lmax", [0, 3, 8])
def test_mex_equals_legendre_sum(orc, lmax):
    p = W.plummer_hernquist_mix(300, 12)
    pot = orc.mex_force(p.x, p.y, p.z, p.m, lmax)[0]
    ref = orc.mex_brute(p.x, p.y, p.z, p.m, lmax)
    np.testing.assert_allclose(pot, ref, rtol=1e-12, atol=1e-14 * np.max(np.abs(ref)))


def test_mex_monopole_is_gauss_law(orc):
    p = W.plummer_hernquist_mix(500, 13)
    key = (p.x * p.x + p.y * p.y) + p.z * p.z
    order = np.lexsort((np.arange(p.n), key))
    assert np.array_equal(order, orc.mex_order(p.x, p.y, p.z))
    r = np.sqrt(key)
    min_ = np.zeros(p.n)
    mout = np.zeros(p.n)
    ms = p.m[order]
    rs = r[order]
    min_[order] = np.concatenate([[0.0], np.cumsum(ms)[:-1]])
    mout[order] = np.concatenate([np.cumsum((ms / rs)[::-1])[::-1][1:], [0.0]])
    pot, ax, ay, az = orc.mex_force(p.x, p.y, p.z, p.m, 0)
    np.testing.assert_allclose(pot, -(min_ / r + mout), rtol=1e-12)
    g = -min_ / r ** 3
    np.testing.assert_allclose(ax, g * p.x, rtol=1e-10, atol=1e-14)
    np.testing.assert_allclose(az, g * p.z, rtol=1e-10, atol=1e-14)


def test_mex_force_is_gradient_of_field(orc):
    """The MEX force on particle i equals -grad of the truncated expansion of all other
    particles, evaluated at field points around x_i (no shell is crossed)."""
    p = W.plummer_hernquist_mix(400, 14)
    lmax = 6
    _, ax, ay, az = orc.mex_force(p.x, p.y, p.z, p.m, lmax)
    r = np.sqrt(p.x ** 2 + p.y ** 2 + p.z ** 2)
    for i in [3, 50, 171, 333]:
        keep = np.arange(p.n) != i
        h = 1e-7 * r[i]
        gaps = np.abs(r[keep] - r[i])
        assert np.min(gaps) > 10 * h
        fd = []
        for d in range(3):
            f = np.array([[p.x[i]], [p.y[i]], [p.z[i]]]).repeat(2, axis=1)
            f[d, 0] += h
            f[d, 1] -= h
            v = orc.mex_brute(p.x[keep], p.y[keep], p.z[keep], p.m[keep], lmax, f[0], f[1], f[2])
            fd.append(-(v[0] - v[1]) / (2 * h))
        got = np.array([ax[i], ay[i], az[i]])
        np.testing.assert_allclose(got, fd, rtol=2e-6, atol=2e-6 * np.max(np.abs(got)))


def test_mex_tends_to_direct_sum(orc):
    p = W.plummer_hernquist_mix(400, 15)
    direct = orc.direct(p.x, p.y, p.z, p.m)[0]
    errs = [np.median(np.abs(orc.mex_force(p.x, p.y, p.z, p.m, L)[0] / direct - 1)) for L in (0, 4, 12, 24)]
    assert errs[0] > errs[1] > errs[2] > errs[3]


# ------------------------------------------------------------------- leapfrog
def test_leapfrog_time_reversible(orc):
    p = W.batched_systems(nsys=2, seed=21, nlog=(2.5, 2.7))
    nmax, lmax, dt, steps = 4, 2, 0.01, 20
    s1 = orc.leapfrog_scf(p.x, p.y, p.z, p.vx, p.vy, p.vz, p.m, p.offsets, nmax, lmax, dt, steps)
    x, y, z, vx, vy, vz = s1
    s2 = orc.leapfrog_scf(x, y, z, -vx, -vy, -vz, p.m, p.offsets, nmax, lmax, dt, steps)
    for a, b in zip(s2[:3], (p.x, p.y, p.z)):
        np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-9)
    for a, b in zip(s2[3:], (p.vx, p.vy, p.vz)):
        np.testing.assert_allclose(-a, b, rtol=1e-8, atol=1e-9)


# --------------------------------------------------------------- paper values
def test_paper_coefficient_counts(orc):
    with open(os.path.join(GOLDEN, "paper_values.json")) as f:
        g = json.load(f)
    for case in g["scf_complex_coefficients"]:
        assert orc.coeff_count(case["nmax"], case["lmax"]) == case["count"]
    for case in g["mex_function_pairs"]:
        assert (case["lmax"] + 1) * (case["lmax"] + 2) // 2 == case["count"]
