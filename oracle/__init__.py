"""FP64 CPU oracle for the SCF / MEX expansion force calculation.

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package; the GPU library and
its Python binding never do.  The oracle shares no code with the GPU path.

The arithmetic lives in ``etics_oracle.c`` (plain C, FP64, compiled without
fast-math and without FMA contraction); this module only builds it with gcc and
marshals numpy arrays through ctypes.  Each wrapped function names the part of
the paper it follows in the C source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "etics_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# the same source with long-double running sums: measures the rounding of the plain
# oracle's own sequential sums (each term is still formed in double)
_LIB_EXT = os.path.join(_HERE, "liboracle_ld.so")
_lib = None
_lib_ext = None

_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)


def _build_one(out: str, extra) -> None:
    cmd = [
        "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
        "-ffp-contract=off", "-fno-fast-math", "-Wall", *extra,
        _SRC, "-o", out + ".tmp", "-lm",
    ]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)


def build() -> str:
    """Compile etics_oracle.c into liboracle.so (gcc, -O2, OpenMP, no fast-math) and
    into liboracle_ld.so (the same with long-double running sums)."""
    _build_one(_LIB, [])
    _build_one(_LIB_EXT, ["-DORACLE_ACC=long double"])
    return _LIB


def _stale(path: str) -> bool:
    return not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC)


def lib(ext: bool = False):
    """The oracle library; ext=True: the build with long-double running sums."""
    global _lib, _lib_ext
    if (_lib_ext if ext else _lib) is None:
        if _stale(_LIB) or _stale(_LIB_EXT):
            build()
        L = ctypes.CDLL(_LIB_EXT if ext else _LIB)
        L.oracle_gegenbauer.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, _D]
        L.oracle_ylm.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, _D]
        L.oracle_ylm_deriv.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, _D, _D, _D]
        L.oracle_knl.argtypes = [ctypes.c_int, ctypes.c_int]
        L.oracle_knl.restype = ctypes.c_double
        L.oracle_anl_tilde.argtypes = [ctypes.c_int, ctypes.c_int]
        L.oracle_anl_tilde.restype = ctypes.c_double
        L.oracle_phi_nl.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _D, _D]
        L.oracle_rho_nl.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _D]
        L.oracle_knl_cb.argtypes = [ctypes.c_int, ctypes.c_int]
        L.oracle_knl_cb.restype = ctypes.c_double
        L.oracle_anl_tilde_basis.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.oracle_anl_tilde_basis.restype = ctypes.c_double
        L.oracle_phi_nl_basis.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, _D, _D]
        L.oracle_rho_nl_basis.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, _D]
        L.oracle_scf_coeffs_basis.argtypes = [ctypes.c_int, _D, _D, _D, _D, ctypes.c_int64, ctypes.c_int,
                                              ctypes.c_int, _D, _D]
        L.oracle_scf_force_basis.argtypes = [ctypes.c_int, _D, _D, _D, ctypes.c_int64, ctypes.c_int,
                                             ctypes.c_int, _D, _D, _D, _D, _D, _D]
        L.oracle_coeff_count.argtypes = [ctypes.c_int, ctypes.c_int]
        L.oracle_coeff_count.restype = ctypes.c_int
        L.oracle_scf_coeffs.argtypes = [_D, _D, _D, _D, ctypes.c_int64, ctypes.c_int, ctypes.c_int, _D, _D]
        L.oracle_scf_force.argtypes = [_D, _D, _D, ctypes.c_int64, ctypes.c_int, ctypes.c_int, _D, _D,
                                       _D, _D, _D, _D]
        L.oracle_r2_key.argtypes = [ctypes.c_double] * 3
        L.oracle_r2_key.restype = ctypes.c_double
        L.oracle_mex_order.argtypes = [_D, _D, _D, ctypes.c_int64, _I64]
        L.oracle_mex_force.argtypes = [_D, _D, _D, _D, ctypes.c_int64, ctypes.c_int, _D, _D, _D, _D]
        L.oracle_mex_brute.argtypes = [_D, _D, _D, _D, ctypes.c_int64, ctypes.c_int, _D, _D, _D,
                                       ctypes.c_int64, ctypes.c_int, _D]
        L.oracle_direct.argtypes = [_D, _D, _D, _D, ctypes.c_int64, _D, _D, _D, _D]
        L.oracle_leapfrog_scf.argtypes = [_D, _D, _D, _D, _D, _D, _D, _I64, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_double, ctypes.c_int]
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        if ext:
            _lib_ext = L
        else:
            _lib = L
    return _lib_ext if ext else _lib


def _dp(a):
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return lib().oracle_num_threads()


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


def coeff_count(nmax: int, lmax: int) -> int:
    return lib().oracle_coeff_count(nmax, lmax)


def gegenbauer(nmax: int, alpha: float, x: float) -> np.ndarray:
    out = np.zeros(nmax + 1)
    lib().oracle_gegenbauer(nmax, alpha, x, _dp(out))
    return out


def ylm(lmax: int, theta: float) -> np.ndarray:
    """Orthonormal Ybar_lm(theta), index l(l+1)/2 + m."""
    out = np.zeros((lmax + 1) * (lmax + 2) // 2)
    lib().oracle_ylm(lmax, np.cos(theta), np.sin(theta), _dp(out))
    return out


def ylm_deriv(lmax: int, theta: float):
    n = (lmax + 1) * (lmax + 2) // 2
    Y, dY, mYs = np.zeros(n), np.zeros(n), np.zeros(n)
    lib().oracle_ylm_deriv(lmax, np.cos(theta), np.sin(theta), _dp(Y), _dp(dY), _dp(mYs))
    return Y, dY, mYs


# radial bases: 0 = Hernquist-Ostriker (the paper's), 1 = Clutton-Brock
BASIS_HO, BASIS_CB = 0, 1


def knl(n: int, l: int, basis: int = BASIS_HO) -> float:
    return lib().oracle_knl_cb(n, l) if basis == BASIS_CB else lib().oracle_knl(n, l)


def anl_tilde(n: int, l: int, basis: int = BASIS_HO) -> float:
    return lib().oracle_anl_tilde_basis(basis, n, l)


def phi_nl(nmax: int, lmax: int, r: float, basis: int = BASIS_HO):
    """(PhiT, dPhiT/dr) arrays shaped [nmax+1, lmax+1]."""
    phi = np.zeros((nmax + 1) * (lmax + 1))
    dphi = np.zeros_like(phi)
    lib().oracle_phi_nl_basis(basis, nmax, lmax, float(r), _dp(phi), _dp(dphi))
    return phi.reshape(nmax + 1, lmax + 1), dphi.reshape(nmax + 1, lmax + 1)


def rho_nl(nmax: int, lmax: int, r: float, basis: int = BASIS_HO) -> np.ndarray:
    rho = np.zeros((nmax + 1) * (lmax + 1))
    lib().oracle_rho_nl_basis(basis, nmax, lmax, float(r), _dp(rho))
    return rho.reshape(nmax + 1, lmax + 1)


def scf_coeffs(x, y, z, m, nmax: int, lmax: int, ext: bool = False, basis: int = BASIS_HO):
    """ext=True: the same sums with long-double accumulators."""
    x, y, z, m = _f64(x), _f64(y), _f64(z), _f64(m)
    K = coeff_count(nmax, lmax)
    A, B = np.zeros(K), np.zeros(K)
    lib(ext).oracle_scf_coeffs_basis(basis, _dp(x), _dp(y), _dp(z), _dp(m), len(x), nmax, lmax,
                                     _dp(A), _dp(B))
    return A, B


def scf_force(x, y, z, nmax: int, lmax: int, A, B, ext: bool = False, basis: int = BASIS_HO):
    x, y, z, A, B = _f64(x), _f64(y), _f64(z), _f64(A), _f64(B)
    n = len(x)
    pot, ax, ay, az = (np.zeros(n) for _ in range(4))
    lib(ext).oracle_scf_force_basis(basis, _dp(x), _dp(y), _dp(z), n, nmax, lmax, _dp(A), _dp(B),
                                    _dp(pot), _dp(ax), _dp(ay), _dp(az))
    return pot, ax, ay, az


def r2_key(x: float, y: float, z: float) -> float:
    return lib().oracle_r2_key(x, y, z)


def mex_order(x, y, z) -> np.ndarray:
    x, y, z = _f64(x), _f64(y), _f64(z)
    order = np.zeros(len(x), dtype=np.int64)
    lib().oracle_mex_order(_dp(x), _dp(y), _dp(z), len(x), order.ctypes.data_as(_I64))
    return order


def mex_force(x, y, z, m, lmax: int, ext: bool = False):
    x, y, z, m = _f64(x), _f64(y), _f64(z), _f64(m)
    n = len(x)
    pot, ax, ay, az = (np.zeros(n) for _ in range(4))
    lib(ext).oracle_mex_force(_dp(x), _dp(y), _dp(z), _dp(m), n, lmax,
                           _dp(pot), _dp(ax), _dp(ay), _dp(az))
    return pot, ax, ay, az


def mex_brute(x, y, z, m, lmax: int, fx=None, fy=None, fz=None):
    """Truncated Laplace expansion summed directly over sources (addition-theorem form).

    Without field points, the field points are the particles themselves and self
    terms are skipped."""
    x, y, z, m = _f64(x), _f64(y), _f64(z), _f64(m)
    skip = fx is None
    if skip:
        fx, fy, fz = x, y, z
    fx, fy, fz = _f64(fx), _f64(fy), _f64(fz)
    pot = np.zeros(len(fx))
    lib().oracle_mex_brute(_dp(x), _dp(y), _dp(z), _dp(m), len(x), lmax, _dp(fx), _dp(fy), _dp(fz),
                           len(fx), 1 if skip else 0, _dp(pot))
    return pot


def direct(x, y, z, m):
    x, y, z, m = _f64(x), _f64(y), _f64(z), _f64(m)
    n = len(x)
    pot, ax, ay, az = (np.zeros(n) for _ in range(4))
    lib().oracle_direct(_dp(x), _dp(y), _dp(z), _dp(m), n, _dp(pot), _dp(ax), _dp(ay), _dp(az))
    return pot, ax, ay, az


def leapfrog_scf(x, y, z, vx, vy, vz, m, offsets, nmax: int, lmax: int, dt: float, nsteps: int):
    """KDK leapfrog of independent systems; returns updated copies (x,y,z,vx,vy,vz)."""
    arrs = [np.array(a, dtype=np.float64, copy=True) for a in (x, y, z, vx, vy, vz)]
    m = _f64(m)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    lib().oracle_leapfrog_scf(*[_dp(a) for a in arrs], _dp(m), offsets.ctypes.data_as(_I64),
                              len(offsets) - 1, nmax, lmax, float(dt), int(nsteps))
    return tuple(arrs)
