"""Pins of the Ferrers n=1 "real" force (the reference of the accuracy study,
Section 4.1) and of the direct-summation oracle, against closed forms, Poisson's
equation, the far field and brute force (CPU only)."""
import math

import numpy as np
import pytest

from paper_1406_4254_amd import workloads as W
from oracle import ferrers as F


def test_sphere_limit_closed_form():
    """a = b = c = R: the enclosed mass is M [(5/2) s^3 - (3/2) s^5], s = r/R, and
    the force -M(<r) x / r^3 inside and out."""
    R = 1.3
    rng = np.random.default_rng(3)
    r = np.concatenate([rng.uniform(1e-3, R, 50), rng.uniform(R, 20.0, 50)])
    d = rng.normal(size=(3, 100))
    d /= np.linalg.norm(d, axis=0)
    x, y, z = r * d
    got = F.force(x, y, z, (R, R, R))
    s = np.minimum(r / R, 1.0)
    menc = np.where(r < R, 2.5 * s ** 3 - 1.5 * s ** 5, 1.0)
    for g, xk in zip(got, (x, y, z)):
        np.testing.assert_allclose(g, -menc * xk / r ** 3, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("model", ["model1", "model2"])
def test_poisson_inside(model):
    """div F = -4 pi rho at interior points (central differences, h = 1e-4)."""
    axes = W.FERRERS_MODELS[model]
    p = W.ferrers1(40, 11, axes)
    h = 1e-4
    div = np.zeros(p.n)
    for k in range(3):
        pts = [p.x.copy(), p.y.copy(), p.z.copy()]
        pts[k] = pts[k] + h
        fp = F.force(*pts, axes)[k]
        pts[k] = pts[k] - 2 * h
        fm = F.force(*pts, axes)[k]
        div += (fp - fm) / (2 * h)
    rho = F.density(p.x, p.y, p.z, axes)
    keep = rho > 0.05 * rho.max()  # away from the surface, where rho has a kink
    np.testing.assert_allclose(div[keep], -4 * math.pi * rho[keep], rtol=2e-6)


def test_far_field_and_surface_continuity():
    axes = W.FERRERS_MODELS["model2"]
    # far field: |F| r^2 -> M (quadrupole correction ~ (a/r)^2)
    d = np.array([[0.3, -0.5, 0.81]]).T / np.linalg.norm([0.3, -0.5, 0.81])
    x, y, z = d * 1e3
    f = np.sqrt(sum(g ** 2 for g in F.force(x, y, z, axes)))
    assert abs(f[0] * 1e6 - 1.0) < 1e-5
    # continuity across the surface mu = a along a ray
    base = np.array([0.4, 0.5, 0.6])
    mu = math.sqrt((base[0] / axes[0]) ** 2 + (base[1] / axes[1]) ** 2 + (base[2] / axes[2]) ** 2)
    pin = base / mu * (1 - 1e-10)
    pout = base / mu * (1 + 1e-10)
    fi = np.array(F.force(*[np.array([v]) for v in pin], axes))
    fo = np.array(F.force(*[np.array([v]) for v in pout], axes))
    np.testing.assert_allclose(fi, fo, rtol=1e-8)


def test_quadrature_converged():
    axes = W.FERRERS_MODELS["model2"]
    p = W.ferrers1(200, 5, axes)
    x = np.concatenate([p.x, 3 * p.x])
    y = np.concatenate([p.y, 3 * p.y])
    z = np.concatenate([p.z, 3 * p.z])
    a = F.force(x, y, z, axes, nodes=96)
    b = F.force(x, y, z, axes, nodes=160)
    for u, v in zip(a, b):
        np.testing.assert_allclose(u, v, rtol=1e-12, atol=1e-14)


def test_sampler_density_profile():
    """mu/a of the drawn points follows p(s) = 15/2 s^2 (1 - s^2) on [0, 1]."""
    axes = W.FERRERS_MODELS["model2"]
    p = W.ferrers1(200_000, 1, axes)
    s = np.sqrt((p.x / axes[0]) ** 2 + (p.y / axes[1]) ** 2 + (p.z / axes[2]) ** 2)
    assert s.max() <= 1.0
    hist, edges = np.histogram(s, bins=20, range=(0, 1))
    cdf = lambda v: 7.5 * (v ** 3 / 3 - v ** 5 / 5)  # noqa: E731
    expect = p.n * (cdf(edges[1:]) - cdf(edges[:-1]))
    assert np.all(np.abs(hist - expect) < 5 * np.sqrt(expect) + 5)
    assert abs(np.sum(p.m) - 1.0) < 1e-12


def test_direct_sum_brute_force_and_momentum(orc):
    """The oracle's direct sum against a plain double loop, and sum m_i a_i = 0."""
    p = W.ferrers1(60, 2, W.FERRERS_MODELS["model1"])
    pot, ax, ay, az = orc.direct(p.x, p.y, p.z, p.m)
    for i in (0, 17, 59):
        e = np.zeros(4)
        for j in range(p.n):
            if j == i:
                continue
            d = np.array([p.x[j] - p.x[i], p.y[j] - p.y[i], p.z[j] - p.z[i]])
            r = math.sqrt(d @ d)
            e[0] -= p.m[j] / r
            e[1:] += p.m[j] * d / r ** 3
        np.testing.assert_allclose([pot[i], ax[i], ay[i], az[i]], e, rtol=1e-13)
    mom = np.array([np.sum(p.m * ax), np.sum(p.m * ay), np.sum(p.m * az)])
    assert np.all(np.abs(mom) < 1e-14 * np.sum(p.m * np.sqrt(ax ** 2 + ay ** 2 + az ** 2)))
