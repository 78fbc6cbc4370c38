"""FP64 CPU oracle for the SCF jerk and the fourth-order Hermite integrator.

TEST INFRASTRUCTURE ONLY: used by the test suite and nothing in the GPU library.

The paper notes that Hernquist's SCF code computes the jerk, the time derivative of
the acceleration, for a fourth-order Hermite integrator (Section 3.4, Performance), and
names that integrator as the next step for SCF, not for MEX, whose force derivative is
discontinuous at shell crossings (Section 5.4).  Here, for particles x_k moving with
velocities v_k:

  * the SCF coefficients A_nlm(t), B_nlm(t) are those of eq. scf-phi (Section 2.4, the
    Hernquist-Ostriker basis of Section 2.5) at the positions x_k + v_k t, and their time
    derivatives dA/dt, dB/dt are the t-derivatives at t = 0;
  * the acceleration of particle i is a_i = -grad Phi(x_i; A, B), and its jerk is the
    total time derivative j_i = d/dt a(x_i + v_i t; A(t), B(t)) at t = 0 -- the field
    point and every particle that makes the field move;
  * the integrator is the Hermite predictor-corrector of Makino & Aarseth (1992), one
    shared step dt:
      predict  x_p = x + v dt + a dt^2/2 + j dt^3/6,   v_p = v + a dt + j dt^2/2,
      evaluate a_1, j_1 at (x_p, v_p),
      correct  v_1 = v + (a + a_1) dt/2 + (j - j_1) dt^2/12,
               x_1 = x + (v + v_1) dt/2 + (a - a_1) dt^2/12.

The expansion is written out directly in plain PyTorch FP64 CPU tensors: the
Gegenbauer three-term recurrence, the textbook associated-Legendre recurrence
normalised by factorials, cos/sin(m phi) from atan2, the coefficient sums and the
synthesis.  The acceleration is -grad Phi by reverse-mode differentiation of that
potential and the time derivatives are forward-mode derivatives along the motion
(torch.func), so both are exact to rounding, with no finite differences.  Atilde_nl
comes from the C oracle.  Points exactly on the z axis are outside its domain (the
azimuth has no derivative there).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from oracle import anl_tilde

F64 = torch.float64


def _lm_tables(lmax):
    ls, ms = [], []
    for l in range(lmax + 1):
        for m in range(l + 1):
            ls.append(l)
            ms.append(m)
    return torch.tensor(ls), torch.tensor(ms)


def _spherical(p):
    """r, cos(theta), sin(theta), phi of points p [P, 3]."""
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    R = torch.sqrt(x * x + y * y)
    r = torch.sqrt(R * R + z * z)
    return r, z / r, R / r, torch.atan2(y, x)


def _radial(r, nmax, lmax):
    """PhiT_nl(r) [P, nmax+1, lmax+1]: -sqrt(4 pi) r^l/(1+r)^(2l+1) C_n^(2l+3/2)(xi)."""
    xi = (r - 1.0) / (r + 1.0)
    cols = []
    for l in range(lmax + 1):
        a = 2.0 * l + 1.5
        c = [torch.ones_like(r)]
        if nmax >= 1:
            c.append(2.0 * a * xi)
        for n in range(2, nmax + 1):
            c.append((2.0 * (n + a - 1.0) * xi * c[n - 1] - (n + 2.0 * a - 2.0) * c[n - 2]) / n)
        f = -math.sqrt(4.0 * math.pi) * r ** l / (1.0 + r) ** (2 * l + 1)
        cols.append(torch.stack(c, dim=1) * f[:, None])
    return torch.stack(cols, dim=2)


def _ylm(ct, st, lmax):
    """Orthonormal Ybar_lm(theta) [P, (lmax+1)(lmax+2)/2] (Condon-Shortley phase), from
    P_m^m = (-1)^m (2m-1)!! sin^m, P_{m+1}^m = (2m+1) cos P_m^m,
    (l-m) P_l^m = (2l-1) cos P_{l-1}^m - (l+m-1) P_{l-2}^m, times
    sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)."""
    P = {}
    for m in range(lmax + 1):
        dfact = 1.0
        for k in range(1, 2 * m, 2):
            dfact *= k
        P[(m, m)] = (-1.0) ** m * dfact * st ** m
        if m + 1 <= lmax:
            P[(m + 1, m)] = (2 * m + 1) * ct * P[(m, m)]
        for l in range(m + 2, lmax + 1):
            P[(l, m)] = ((2 * l - 1) * ct * P[(l - 1, m)] - (l + m - 1) * P[(l - 2, m)]) / (l - m)
    out = []
    for l in range(lmax + 1):
        for m in range(l + 1):
            norm = math.sqrt((2 * l + 1) / (4.0 * math.pi) * math.factorial(l - m) / math.factorial(l + m))
            out.append(norm * P[(l, m)])
    return torch.stack(out, dim=1)


def _basis(p, nmax, lmax):
    r, ct, st, ph = _spherical(p)
    ls, ms = _lm_tables(lmax)
    G = _radial(r, nmax, lmax)[:, :, ls]          # [P, n, lm]
    Y = _ylm(ct, st, lmax)                        # [P, lm]
    c = torch.cos(ms[None, :].to(F64) * ph[:, None])
    s = torch.sin(ms[None, :].to(F64) * ph[:, None])
    return G, Y, c, s


def coeffs(p, mass, nmax, lmax):
    """A, B [nmax+1, (lmax+1)(lmax+2)/2] of particles p [N, 3] with masses [N]."""
    G, Y, c, s = _basis(p, nmax, lmax)
    ls, ms = _lm_tables(lmax)
    at = torch.tensor([[anl_tilde(n, l) for l in range(lmax + 1)] for n in range(nmax + 1)], dtype=F64)
    scale = at[:, ls] * torch.where(ms == 0, 1.0, 2.0).to(F64)[None, :]
    w = mass[:, None] * Y
    A = scale * torch.einsum("knj,kj->nj", G, w * c)
    B = scale * torch.einsum("knj,kj->nj", G, w * s)
    return A, B


def potential(points, A, B, nmax, lmax):
    """Phi at points [P, 3] from coefficients A, B:
    sum_nlm PhiT_nl(r) Ybar_lm(theta) (A cos m phi + B sin m phi)."""
    G, Y, c, s = _basis(points, nmax, lmax)
    return torch.einsum("pnj,nj,pj->p", G, A, Y * c) + torch.einsum("pnj,nj,pj->p", G, B, Y * s)


def acceleration(points, A, B, nmax, lmax):
    """a = -grad Phi at points [P, 3] (each point's potential depends on that point only)."""
    return -torch.func.grad(lambda q: potential(q, A, B, nmax, lmax).sum())(points)


def coeffs_dot(p, v, mass, nmax, lmax):
    """(A, B) and their time derivatives along the motion x_k + v_k t."""
    (A, B), (dA, dB) = torch.func.jvp(lambda t: coeffs(p + v * t, mass, nmax, lmax),
                                      (torch.zeros((), dtype=F64),), (torch.ones((), dtype=F64),))
    return A, B, dA, dB


def accel_jerk(p, v, mass, nmax, lmax):
    """Acceleration and jerk of every particle of one system [N, 3] each."""
    def acc_t(t):
        q = p + v * t
        A, B = coeffs(q, mass, nmax, lmax)
        return acceleration(q, A, B, nmax, lmax)
    a, j = torch.func.jvp(acc_t, (torch.zeros((), dtype=F64),), (torch.ones((), dtype=F64),))
    return a, j


def energy(p, v, mass, nmax, lmax):
    """Kinetic energy plus half the mass-weighted SCF potential (W = 1/2 sum m Phi)."""
    A, B = coeffs(p, mass, nmax, lmax)
    return float(0.5 * torch.sum(mass * torch.sum(v * v, dim=1)) +
                 0.5 * torch.sum(mass * potential(p, A, B, nmax, lmax)))


def hermite(p, v, mass, nmax, lmax, dt, nsteps):
    """nsteps shared Hermite steps of one system; returns the final (p, v)."""
    a, j = accel_jerk(p, v, mass, nmax, lmax)
    for _ in range(nsteps):
        pp = p + v * dt + a * (dt * dt / 2.0) + j * (dt ** 3 / 6.0)
        vp = v + a * dt + j * (dt * dt / 2.0)
        a1, j1 = accel_jerk(pp, vp, mass, nmax, lmax)
        v1 = v + (a + a1) * (dt / 2.0) + (j - j1) * (dt * dt / 12.0)
        p = p + (v + v1) * (dt / 2.0) + (a - a1) * (dt * dt / 12.0)
        v, a, j = v1, a1, j1
    return p, v


def as_rows(x, y, z):
    return torch.from_numpy(np.stack([np.asarray(x, dtype=np.float64), np.asarray(y, dtype=np.float64),
                                      np.asarray(z, dtype=np.float64)], axis=1))


def hermite_systems(x, y, z, vx, vy, vz, m, offsets, nmax, lmax, dt, nsteps):
    """Hermite steps of independent systems in CSR layout; returns (x, y, z, vx, vy, vz)."""
    out = [np.array(a, dtype=np.float64, copy=True) for a in (x, y, z, vx, vy, vz)]
    for s in range(len(offsets) - 1):
        b, e = int(offsets[s]), int(offsets[s + 1])
        if e <= b:
            continue
        p = as_rows(x[b:e], y[b:e], z[b:e])
        v = as_rows(vx[b:e], vy[b:e], vz[b:e])
        p, v = hermite(p, v, torch.from_numpy(np.asarray(m[b:e], dtype=np.float64)), nmax, lmax, dt, nsteps)
        for k in range(3):
            out[k][b:e] = p[:, k].numpy()
            out[3 + k][b:e] = v[:, k].numpy()
    return tuple(out)
