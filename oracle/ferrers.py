"""The "real" (smooth, infinite-N) force of a Ferrers ellipsoid of index 1, the
reference of the accuracy study in Section 4.1.  TEST INFRASTRUCTURE ONLY, like the
rest of this package.  Plain numpy, FP64.

Density (G = 1, total mass M, axes a1 >= a2 >= a3 not required):
    rho = rho0 (1 - m^2)  for m^2 = x^2/a1^2 + y^2/a2^2 + z^2/a3^2 <= 1, else 0,
    rho0 = 15 M / (8 pi a1 a2 a3).
The field of a stratified ellipsoid follows from the one-dimensional integral of
Binney & Tremaine, Galactic Dynamics, Section 2.5 (the paper's reference for these
models): with m^2(u) = sum_k x_k^2 / (a_k^2 + u) and
Delta(u) = sqrt((a1^2 + u)(a2^2 + u)(a3^2 + u)),
    F_k(x) = -2 pi rho0 a1 a2 a3 x_k  int_lambda^inf  (1 - m^2(u)) du / ((a_k^2 + u) Delta(u)),
where lambda = 0 inside the body and m^2(lambda) = 1 outside (the density factor
vanishes for u < lambda).  This is -grad of the potential of that section for
rho(m^2) = rho0 (1 - m^2); the paper fits the same force as a polynomial instead.

Quadrature: u = lambda + s0 (1/t^2 - 1), t in (0, 1], s0 = max_k a_k^2 + lambda, so
the integrand (which decays like u^(-5/2)) becomes a smooth function of t that vanishes
like t^2 at t = 0; Gauss-Legendre nodes on [0, 1] (numpy's leggauss) then converge
fast.  lambda by bisection on the decreasing function m^2(lambda) - 1.
"""
from __future__ import annotations

import numpy as np


def _lambda(x, y, z, a2):
    """lambda per point: 0 inside the body, else the root of m^2(lambda) = 1."""
    m2 = x * x / a2[0] + y * y / a2[1] + z * z / a2[2]
    lam = np.zeros_like(x)
    out = m2 > 1.0
    if np.any(out):
        xo, yo, zo = x[out], y[out], z[out]
        lo = np.zeros_like(xo)
        hi = xo * xo + yo * yo + zo * zo  # m^2(r^2) < 1 since every a_k^2 > 0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            f = xo * xo / (a2[0] + mid) + yo * yo / (a2[1] + mid) + zo * zo / (a2[2] + mid) - 1.0
            lo = np.where(f > 0.0, mid, lo)
            hi = np.where(f > 0.0, hi, mid)
        lam[out] = 0.5 * (lo + hi)
    return lam


def force(x, y, z, axes, mass=1.0, nodes=96, chunk=20000):
    """Acceleration (ax, ay, az) of the Ferrers n=1 ellipsoid at the given points."""
    x, y, z = (np.ascontiguousarray(v, dtype=np.float64) for v in (x, y, z))
    a2 = np.array([float(v) ** 2 for v in axes])
    abc = float(axes[0]) * float(axes[1]) * float(axes[2])
    rho0 = 15.0 * mass / (8.0 * np.pi * abc)
    t, w = np.polynomial.legendre.leggauss(nodes)
    t = 0.5 * (t + 1.0)
    w = 0.5 * w
    out = [np.empty_like(x) for _ in range(3)]
    for s in range(0, x.size, chunk):
        xs, ys, zs = x[s:s + chunk], y[s:s + chunk], z[s:s + chunk]
        lam = _lambda(xs, ys, zs, a2)
        s0 = a2.max() + lam
        u = lam[:, None] + s0[:, None] * (1.0 / (t * t) - 1.0)[None, :]
        du = (2.0 * s0[:, None] / (t * t * t)[None, :]) * w[None, :]
        d = [a2[k] + u for k in range(3)]
        delta = np.sqrt(d[0] * d[1] * d[2])
        m2 = xs[:, None] ** 2 / d[0] + ys[:, None] ** 2 / d[1] + zs[:, None] ** 2 / d[2]
        common = (1.0 - m2) * du / delta
        for k, xk in enumerate((xs, ys, zs)):
            out[k][s:s + chunk] = -2.0 * np.pi * rho0 * abc * xk * np.sum(common / d[k], axis=1)
    return tuple(out)


def density(x, y, z, axes, mass=1.0):
    """rho at the given points (0 outside the body)."""
    a, b, c = (float(v) for v in axes)
    rho0 = 15.0 * mass / (8.0 * np.pi * a * b * c)
    m2 = (np.asarray(x) / a) ** 2 + (np.asarray(y) / b) ** 2 + (np.asarray(z) / c) ** 2
    return np.where(m2 <= 1.0, rho0 * (1.0 - m2), 0.0)
