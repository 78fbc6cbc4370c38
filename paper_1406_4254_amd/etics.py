"""Thin Python binding of libetics.so (the C-ABI in include/etics.h).

Argument marshalling only: every step of the force calculation runs in the HIP
kernels behind the C-ABI.  Tensors must be FP64, contiguous and on the GPU; the
functions allocate outputs and workspace with torch when they are not given, and
enqueue on torch's current stream.  There is no CPU fallback: if the library is not
built, or a call fails, an exception is raised.

torch is imported before the library is loaded, so that libetics.so binds to the HIP
runtime (libamdhip64.so.7) that torch has already loaded.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libetics.so")

ETICS_FP64 = 0
ETICS_MIXED_FP64ACC = 1
ETICS_MIXED_COMP32 = 2
ETICS_POT = 1
ETICS_ACC = 2
ETICS_POT_ACC = 3
ETICS_LEAPFROG_EAGER = 1
ETICS_NMAX_CAP = 20
ETICS_LMAX_CAP = 14

PRECISIONS = {"fp64": ETICS_FP64, "mixed": ETICS_MIXED_FP64ACC, "comp32": ETICS_MIXED_COMP32}

EXPORTED = [
    "etics_coeff_count", "etics_scf_workspace_size", "etics_scf_coeffs", "etics_scf_force",
    "etics_mex_workspace_size", "etics_mex_force", "etics_batched_workspace_size",
    "etics_scf_coeffs_batched", "etics_scf_force_batched", "etics_leapfrog_scf_batched",
    "etics_direct_force", "etics_set_timing_events", "etics_last_error", "etics_version",
]


class EticsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"etics error {code}: {msg}")
        self.code = code


_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_int = ctypes.c_int
_sz = ctypes.c_size_t


def lib():
    """Load libetics.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        L.etics_coeff_count.argtypes = [_int, _int]
        L.etics_coeff_count.restype = _int
        L.etics_scf_workspace_size.argtypes = [_i64, _int, _int, _int]
        L.etics_scf_workspace_size.restype = _sz
        L.etics_scf_coeffs.argtypes = [_vp, _vp, _vp, _vp, _i64, _int, _int, _int, _vp, _vp, _vp, _sz, _vp]
        L.etics_scf_coeffs.restype = _int
        L.etics_scf_force.argtypes = [_vp, _vp, _vp, _i64, _int, _int, _vp, _vp, _int, _int,
                                      _vp, _vp, _vp, _vp, _vp, _sz, _vp]
        L.etics_scf_force.restype = _int
        L.etics_mex_workspace_size.argtypes = [_i64, _int, _int]
        L.etics_mex_workspace_size.restype = _sz
        L.etics_mex_force.argtypes = [_vp, _vp, _vp, _vp, _i64, _int, _int, _int, _vp, _vp, _vp, _vp,
                                      _vp, _sz, _vp]
        L.etics_mex_force.restype = _int
        L.etics_batched_workspace_size.argtypes = [_i64, _int, _int, _int, _int]
        L.etics_batched_workspace_size.restype = _sz
        L.etics_scf_coeffs_batched.argtypes = [_vp, _vp, _vp, _vp, _vp, _int, _i64, _int, _int, _int,
                                               _vp, _vp, _vp, _sz, _vp]
        L.etics_scf_coeffs_batched.restype = _int
        L.etics_scf_force_batched.argtypes = [_vp, _vp, _vp, _vp, _int, _i64, _int, _int, _vp, _vp,
                                              _int, _int, _vp, _vp, _vp, _vp, _vp, _sz, _vp]
        L.etics_scf_force_batched.restype = _int
        L.etics_leapfrog_scf_batched.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _int, _i64,
                                                 _int, _int, _int, ctypes.c_double, _int, _int, _vp, _sz,
                                                 _vp]
        L.etics_leapfrog_scf_batched.restype = _int
        L.etics_direct_force.argtypes = [_vp, _vp, _vp, _vp, _i64, _int, _vp, _vp, _vp, _vp, _vp]
        L.etics_direct_force.restype = _int
        L.etics_set_timing_events.argtypes = [_vp, _vp]
        L.etics_set_timing_events.restype = _int
        L.etics_last_error.restype = ctypes.c_char_p
        L.etics_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise EticsError(rc, lib().etics_last_error().decode())


def _prec(p) -> int:
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def _dev(t, name, dtype=torch.float64):
    if t is None:
        return None
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TypeError(f"{name}: expected a contiguous {dtype} CUDA tensor")
    return t


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def workspace(nbytes: int, device) -> torch.Tensor:
    """Device workspace (torch's allocator returns 512-byte aligned blocks)."""
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def etics_version() -> str:
    return lib().etics_version().decode()


def etics_set_timing_events(before, after) -> None:
    """Record two torch.cuda.Event objects around the main kernel of every later
    compute call of this thread (None, None: stop).  The events must already exist on
    the device (record each once before passing it)."""
    if (before is None) != (after is None):
        raise ValueError("pass both events or neither")
    hb = None if before is None else ctypes.c_void_p(before.cuda_event)
    ha = None if after is None else ctypes.c_void_p(after.cuda_event)
    if before is not None and not (before.cuda_event and after.cuda_event):
        raise ValueError("record the events once before passing them")
    _check(lib().etics_set_timing_events(hb, ha))


def etics_coeff_count(nmax: int, lmax: int) -> int:
    return lib().etics_coeff_count(nmax, lmax)


def etics_scf_workspace_size(n: int, nmax: int, lmax: int, precision=ETICS_MIXED_FP64ACC) -> int:
    return lib().etics_scf_workspace_size(n, nmax, lmax, _prec(precision))


def etics_mex_workspace_size(n: int, lmax: int, precision=ETICS_MIXED_FP64ACC) -> int:
    return lib().etics_mex_workspace_size(n, lmax, _prec(precision))


def etics_batched_workspace_size(ntotal: int, nsys: int, nmax: int, lmax: int,
                                 precision=ETICS_MIXED_FP64ACC) -> int:
    return lib().etics_batched_workspace_size(ntotal, nsys, nmax, lmax, _prec(precision))


def etics_scf_coeffs(x, y, z, m, nmax: int, lmax: int, precision=ETICS_MIXED_FP64ACC,
                     A=None, B=None, ws=None, stream=None):
    """SCF coefficients (A, B) of the particles (x, y, z, m)."""
    p = _prec(precision)
    for t, nm in ((x, "x"), (y, "y"), (z, "z"), (m, "m")):
        _dev(t, nm)
    n = x.numel()
    K = etics_coeff_count(nmax, lmax)
    if K < 0:
        raise EticsError(-1, "nmax/lmax outside the caps")
    A = torch.empty(K, dtype=torch.float64, device=x.device) if A is None else _dev(A, "A")
    B = torch.empty(K, dtype=torch.float64, device=x.device) if B is None else _dev(B, "B")
    need = etics_scf_workspace_size(n, nmax, lmax, p)
    ws = workspace(need, x.device) if ws is None else ws
    _check(lib().etics_scf_coeffs(_ptr(x), _ptr(y), _ptr(z), _ptr(m), n, nmax, lmax, p, _ptr(A), _ptr(B),
                                  _ptr(ws), ws.numel(), _stream(stream)))
    return A, B


def etics_scf_force(x, y, z, nmax: int, lmax: int, A, B, precision=ETICS_MIXED_FP64ACC,
                    outputs=ETICS_POT_ACC, pot=None, ax=None, ay=None, az=None, ws=None, stream=None):
    """SCF potential and acceleration at (x, y, z) from coefficients A, B."""
    p = _prec(precision)
    for t, nm in ((x, "x"), (y, "y"), (z, "z"), (A, "A"), (B, "B")):
        _dev(t, nm)
    n = x.numel()
    mk = lambda: torch.empty(n, dtype=torch.float64, device=x.device)
    if outputs & ETICS_POT:
        pot = mk() if pot is None else _dev(pot, "pot")
    if outputs & ETICS_ACC:
        ax = mk() if ax is None else _dev(ax, "ax")
        ay = mk() if ay is None else _dev(ay, "ay")
        az = mk() if az is None else _dev(az, "az")
    need = etics_scf_workspace_size(n, nmax, lmax, p)
    ws = workspace(need, x.device) if ws is None else ws
    _check(lib().etics_scf_force(_ptr(x), _ptr(y), _ptr(z), n, nmax, lmax, _ptr(A), _ptr(B), p, outputs,
                                 _ptr(pot), _ptr(ax), _ptr(ay), _ptr(az), _ptr(ws), ws.numel(),
                                 _stream(stream)))
    return pot, ax, ay, az


def etics_mex_force(x, y, z, m, lmax: int, precision=ETICS_MIXED_FP64ACC, outputs=ETICS_POT_ACC,
                    pot=None, ax=None, ay=None, az=None, ws=None, stream=None):
    """MEX potential and acceleration of every particle from all the others."""
    p = _prec(precision)
    for t, nm in ((x, "x"), (y, "y"), (z, "z"), (m, "m")):
        _dev(t, nm)
    n = x.numel()
    mk = lambda: torch.empty(n, dtype=torch.float64, device=x.device)
    if outputs & ETICS_POT:
        pot = mk() if pot is None else _dev(pot, "pot")
    if outputs & ETICS_ACC:
        ax = mk() if ax is None else _dev(ax, "ax")
        ay = mk() if ay is None else _dev(ay, "ay")
        az = mk() if az is None else _dev(az, "az")
    need = etics_mex_workspace_size(n, lmax, p)
    ws = workspace(need, x.device) if ws is None else ws
    _check(lib().etics_mex_force(_ptr(x), _ptr(y), _ptr(z), _ptr(m), n, lmax, p, outputs,
                                 _ptr(pot), _ptr(ax), _ptr(ay), _ptr(az), _ptr(ws), ws.numel(),
                                 _stream(stream)))
    return pot, ax, ay, az


def etics_direct_force(x, y, z, m, outputs=ETICS_POT_ACC, pot=None, ax=None, ay=None, az=None,
                       stream=None):
    """Unsoftened FP64 direct-summation potential and acceleration (O(n^2))."""
    for t, nm in ((x, "x"), (y, "y"), (z, "z"), (m, "m")):
        _dev(t, nm)
    n = x.numel()
    mk = lambda: torch.empty(n, dtype=torch.float64, device=x.device)
    if outputs & ETICS_POT:
        pot = mk() if pot is None else _dev(pot, "pot")
    if outputs & ETICS_ACC:
        ax = mk() if ax is None else _dev(ax, "ax")
        ay = mk() if ay is None else _dev(ay, "ay")
        az = mk() if az is None else _dev(az, "az")
    _check(lib().etics_direct_force(_ptr(x), _ptr(y), _ptr(z), _ptr(m), n, outputs, _ptr(pot), _ptr(ax),
                                    _ptr(ay), _ptr(az), _stream(stream)))
    return pot, ax, ay, az


def etics_scf_coeffs_batched(x, y, z, m, offsets, nmax: int, lmax: int, precision=ETICS_MIXED_FP64ACC,
                             A=None, B=None, ws=None, stream=None):
    p = _prec(precision)
    _dev(offsets, "offsets", torch.int64)
    nsys = offsets.numel() - 1
    n = x.numel()
    K = etics_coeff_count(nmax, lmax)
    A = torch.empty(nsys * K, dtype=torch.float64, device=x.device) if A is None else _dev(A, "A")
    B = torch.empty(nsys * K, dtype=torch.float64, device=x.device) if B is None else _dev(B, "B")
    need = etics_batched_workspace_size(n, nsys, nmax, lmax, p)
    ws = workspace(need, x.device) if ws is None else ws
    _check(lib().etics_scf_coeffs_batched(_ptr(x), _ptr(y), _ptr(z), _ptr(m), _ptr(offsets), nsys, n,
                                          nmax, lmax, p, _ptr(A), _ptr(B), _ptr(ws), ws.numel(),
                                          _stream(stream)))
    return A, B


def etics_scf_force_batched(x, y, z, offsets, nmax: int, lmax: int, A, B, precision=ETICS_MIXED_FP64ACC,
                            outputs=ETICS_POT_ACC, pot=None, ax=None, ay=None, az=None, ws=None,
                            stream=None):
    p = _prec(precision)
    _dev(offsets, "offsets", torch.int64)
    nsys = offsets.numel() - 1
    n = x.numel()
    for t, nm in ((x, "x"), (y, "y"), (z, "z"), (A, "A"), (B, "B")):
        _dev(t, nm)
    mk = lambda: torch.empty(n, dtype=torch.float64, device=x.device)
    if outputs & ETICS_POT:
        pot = mk() if pot is None else _dev(pot, "pot")
    if outputs & ETICS_ACC:
        ax = mk() if ax is None else _dev(ax, "ax")
        ay = mk() if ay is None else _dev(ay, "ay")
        az = mk() if az is None else _dev(az, "az")
    need = etics_batched_workspace_size(n, nsys, nmax, lmax, p)
    ws = workspace(need, x.device) if ws is None else ws
    _check(lib().etics_scf_force_batched(_ptr(x), _ptr(y), _ptr(z), _ptr(offsets), nsys, n, nmax, lmax,
                                         _ptr(A), _ptr(B), p, outputs, _ptr(pot), _ptr(ax), _ptr(ay),
                                         _ptr(az), _ptr(ws), ws.numel(), _stream(stream)))
    return pot, ax, ay, az


def etics_leapfrog_scf_batched(x, y, z, vx, vy, vz, m, offsets, nmax: int, lmax: int, dt: float,
                               nsteps: int, precision=ETICS_MIXED_FP64ACC, flags: int = 0, ws=None,
                               stream=None):
    """Advance x..vz in place by nsteps KDK steps (one captured graph replayed)."""
    p = _prec(precision)
    _dev(offsets, "offsets", torch.int64)
    nsys = offsets.numel() - 1
    n = x.numel()
    need = etics_batched_workspace_size(n, nsys, nmax, lmax, p)
    ws = workspace(need, x.device) if ws is None else ws
    _check(lib().etics_leapfrog_scf_batched(_ptr(x), _ptr(y), _ptr(z), _ptr(vx), _ptr(vy), _ptr(vz),
                                            _ptr(m), _ptr(offsets), nsys, n, nmax, lmax, p, float(dt),
                                            int(nsteps), int(flags), _ptr(ws), ws.numel(), _stream(stream)))
