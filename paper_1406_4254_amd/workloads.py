"""Seeded synthetic particle sets for the SCF / MEX force calculation.

This module only draws inputs; it holds none of the expansion arithmetic, and both
the GPU path and the CPU oracle are fed from it.  All draws use numpy's PCG64
(``numpy.random.default_rng(seed)``) in FP64 on the host.  The paper measures on
synthetic models (a Hernquist sphere for its timing and single-precision study,
Sections 3.4 and 4.2); there is no dataset to stand in for.

Per spherical component of n particles the draw order is fixed:
``u = rng.random(n)`` (mass fraction), ``cos(theta) = rng.uniform(-1, 1, n)``,
``phi = rng.uniform(0, 2 pi, n)``; components are drawn in the order listed.
Radii invert the cumulative mass profile (total mass 1, G = 1):
  Hernquist (scale a):  M(<r) = r^2/(r+a)^2      ->  r = a sqrt(u) / (1 - sqrt(u))
  Plummer   (scale b):  M(<r) = r^3/(r^2+b^2)^1.5 ->  r = b / sqrt(u^(-2/3) - 1)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Particles:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    m: np.ndarray
    vx: np.ndarray | None = None
    vy: np.ndarray | None = None
    vz: np.ndarray | None = None
    offsets: np.ndarray | None = None  # int64 [nsys+1] for batched sets
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def _sphere_dirs(rng, n):
    ct = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * math.pi, n)
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    return st * np.cos(ph), st * np.sin(ph), ct


def hernquist_radii(u, a=1.0):
    s = np.sqrt(u)
    return a * s / (1.0 - s)


def plummer_radii(u, b=1.0):
    return b / np.sqrt(u ** (-2.0 / 3.0) - 1.0)


def sphere(rng, n, kind="hernquist", scale=1.0):
    """n positions of an isotropic Hernquist or Plummer sphere centred at the origin."""
    u = rng.random(n)
    dx, dy, dz = _sphere_dirs(rng, n)
    r = hernquist_radii(u, scale) if kind == "hernquist" else plummer_radii(u, scale)
    return r * dx, r * dy, r * dz


def hernquist_sphere(n, seed, scale=1.0):
    """Config 1 form: equal-mass (1/n) isotropic Hernquist sphere."""
    rng = np.random.default_rng(seed)
    x, y, z = sphere(rng, n, "hernquist", scale)
    return Particles(x, y, z, np.full(n, 1.0 / n),
                     meta={"model": "hernquist", "a": scale, "seed": seed})


def triaxial_hernquist(n, seed, axes=(1.0, 0.8, 0.6)):
    """Config 2 form: Hernquist sphere with x, y, z scaled by axes (l > 0 terms populated)."""
    rng = np.random.default_rng(seed)
    x, y, z = sphere(rng, n, "hernquist", 1.0)
    return Particles(x * axes[0], y * axes[1], z * axes[2], np.full(n, 1.0 / n),
                     meta={"model": "triaxial_hernquist", "axes": list(axes), "seed": seed})


def triaxial_plummer(n, seed, b=1.0, axes=(1.0, 0.8, 0.6)):
    """Plummer sphere (scale b, m = 1/n) with x, y, z scaled by axes: the cored model
    that the Clutton-Brock radial basis expands from its zeroth order."""
    rng = np.random.default_rng(seed)
    x, y, z = sphere(rng, n, "plummer", b)
    return Particles(x * axes[0], y * axes[1], z * axes[2], np.full(n, 1.0 / n),
                     meta={"model": "triaxial_plummer", "b": b, "axes": list(axes), "seed": seed})


def hernquist_plummer_offset(n, seed, b=0.3, offset=(0.5, 0.0, 0.0)):
    """Config 3 form: n/2 Hernquist (a=1) at the origin + n/2 Plummer (b) centred at offset."""
    rng = np.random.default_rng(seed)
    n1 = n // 2
    n2 = n - n1
    x1, y1, z1 = sphere(rng, n1, "hernquist", 1.0)
    x2, y2, z2 = sphere(rng, n2, "plummer", b)
    x = np.concatenate([x1, x2 + offset[0]])
    y = np.concatenate([y1, y2 + offset[1]])
    z = np.concatenate([z1, z2 + offset[2]])
    return Particles(x, y, z, np.full(n, 1.0 / n),
                     meta={"model": "hernquist+offset_plummer", "b": b, "offset": list(offset),
                           "seed": seed})


def plummer_hernquist_mix(n, seed, b=1.0, a=1.0):
    """Config 4 form: n/2 Plummer (b) + n/2 Hernquist (a), both at the origin."""
    rng = np.random.default_rng(seed)
    n1 = n // 2
    n2 = n - n1
    x1, y1, z1 = sphere(rng, n1, "plummer", b)
    x2, y2, z2 = sphere(rng, n2, "hernquist", a)
    return Particles(np.concatenate([x1, x2]), np.concatenate([y1, y2]), np.concatenate([z1, z2]),
                     np.full(n, 1.0 / n), meta={"model": "plummer+hernquist", "seed": seed})


# ---------------------------------------------------------------- velocities
def _jeans_sigma2_table(kind, scale, rmin=1e-6, rmax=1e8, npts=4000):
    """Isotropic Jeans radial dispersion sigma_r^2(r) = (1/rho) int_r^inf rho M / r'^2 dr'
    (G = M = 1) tabulated on a log grid by trapezoidal quadrature."""
    lr = np.linspace(math.log(rmin), math.log(rmax), npts)
    r = np.exp(lr)
    if kind == "hernquist":
        rho = scale / (2.0 * math.pi * r * (r + scale) ** 3)
        M = r * r / (r + scale) ** 2
    else:
        rho = 3.0 / (4.0 * math.pi * scale ** 3) * (1.0 + (r / scale) ** 2) ** -2.5
        M = r ** 3 / (r * r + scale * scale) ** 1.5
    f = rho * M / (r * r) * r  # integrand in d(ln r)
    seg = 0.5 * (f[1:] + f[:-1]) * np.diff(lr)
    tail = np.concatenate([np.cumsum(seg[::-1])[::-1], [0.0]])
    return lr, np.log(np.maximum(tail / rho, 1e-300))


def jeans_velocities(rng, x, y, z, kind, scale):
    """Isotropic Gaussian velocities with the local Jeans dispersion of the system's own profile."""
    lr, ls2 = _jeans_sigma2_table(kind, scale)
    r = np.sqrt(x * x + y * y + z * z)
    s = np.sqrt(np.exp(np.interp(np.log(np.maximum(r, 1e-6)), lr, ls2)))
    v = rng.standard_normal((3, r.shape[0]))
    return v[0] * s, v[1] * s, v[2] * s


def batched_systems(nsys=256, seed=5, nlog=(3.0, 5.0), scale_range=(0.5, 2.0)):
    """Config 5 form: nsys independent spheres in one CSR set (offsets[nsys+1]).

    System s draws from ``default_rng(seed).spawn(nsys)[s]`` in this order: log10 N_s
    ~ U(nlog), kind (Hernquist if U < 1/2 else Plummer), log10 scale ~ U(log10 range),
    positions (sphere draw order above), velocities (3 x N_s standard normals)."""
    children = np.random.default_rng(seed).spawn(nsys)
    xs, ys, zs, ms, vxs, vys, vzs = [], [], [], [], [], [], []
    sizes, kinds, scales = [], [], []
    for s in range(nsys):
        rng = children[s]
        ns = int(round(10.0 ** rng.uniform(*nlog)))
        kind = "hernquist" if rng.random() < 0.5 else "plummer"
        scale = 10.0 ** rng.uniform(math.log10(scale_range[0]), math.log10(scale_range[1]))
        x, y, z = sphere(rng, ns, kind, scale)
        vx, vy, vz = jeans_velocities(rng, x, y, z, kind, scale)
        xs.append(x); ys.append(y); zs.append(z)
        ms.append(np.full(ns, 1.0 / ns))
        vxs.append(vx); vys.append(vy); vzs.append(vz)
        sizes.append(ns); kinds.append(kind); scales.append(scale)
    offsets = np.zeros(nsys + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    cat = np.concatenate
    return Particles(cat(xs), cat(ys), cat(zs), cat(ms), cat(vxs), cat(vys), cat(vzs), offsets,
                     meta={"model": "batched_spheres", "nsys": nsys, "seed": seed,
                           "kinds": kinds, "scales": scales})


# ------------------------------------------------------------- named configs
CONFIGS = {
    1: dict(name="scf_hernquist_n1e4_n10_l6", n=10_000, nmax=10, lmax=6, seed=1,
            make=lambda n, seed: hernquist_sphere(n, seed)),
    2: dict(name="scf_triaxial_hernquist_n1e6_n10_l10", n=1_000_000, nmax=10, lmax=10, seed=2,
            make=lambda n, seed: triaxial_hernquist(n, seed)),
    3: dict(name="scf_hernquist_plummer_n1e7_n20_l14", n=10_000_000, nmax=20, lmax=14, seed=3,
            make=lambda n, seed: hernquist_plummer_offset(n, seed)),
    4: dict(name="mex_plummer_hernquist_n1e6_l10", n=1_000_000, nmax=None, lmax=10, seed=4,
            make=lambda n, seed: plummer_hernquist_mix(n, seed)),
    5: dict(name="batched_256_spheres_n8_l6", n=None, nmax=8, lmax=6, seed=5,
            make=lambda n, seed: batched_systems(256 if n is None else n, seed)),
}


# Ferrers ellipsoids of index 1 (the accuracy study of Section 4.1): density
# rho0 (1 - mu^2/a^2) inside the ellipsoid mu <= a, mu^2 = x^2 + (a/b)^2 y^2 + (a/c)^2 z^2.
# model1 is the 10:10:9 oblate spheroid, model2 the 3:2:1 triaxial ellipsoid; a = 1,
# total mass 1.
FERRERS_MODELS = {"model1": (1.0, 1.0, 0.9), "model2": (1.0, 2.0 / 3.0, 1.0 / 3.0)}


def ferrers1(n, seed, axes=(1.0, 1.0, 0.9)):
    """n particles of mass 1/n drawn from a Ferrers n=1 ellipsoid with the given axes.

    The unit-ball variable s = mu/a has density proportional to s^2 (1 - s^2): s is
    drawn as u^(1/3) (uniform ball) and kept with probability 1 - s^2 (rejection, in
    rounds of draws until n are kept); directions are isotropic; the point is then
    stretched by the axes."""
    rng = np.random.default_rng(seed)
    kept = []
    have = 0
    while have < n:
        k = max(2 * (n - have) + 64, 1024)
        s = rng.random(k) ** (1.0 / 3.0)
        keep = rng.random(k) < 1.0 - s * s
        kept.append(s[keep])
        have += int(keep.sum())
    s = np.concatenate(kept)[:n]
    dx, dy, dz = _sphere_dirs(rng, n)
    a, b, c = axes
    x, y, z = a * s * dx, b * s * dy, c * s * dz
    return Particles(x, y, z, np.full(n, 1.0 / n), meta=dict(model="ferrers1", axes=tuple(axes)))


def make_config(cfg: int, n: int | None = None) -> Particles:
    """Particles of a named configuration; n overrides the size (same recipe and seed)."""
    c = CONFIGS[cfg]
    return c["make"](c["n"] if n is None else n, c["seed"])
