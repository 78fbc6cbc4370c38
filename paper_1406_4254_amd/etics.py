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
ETICS_BASIS_HO = 0
ETICS_BASIS_CB = 1
ETICS_NMAX_CAP = 20
ETICS_LMAX_CAP = 14

PRECISIONS = {"fp64": ETICS_FP64, "mixed": ETICS_MIXED_FP64ACC, "comp32": ETICS_MIXED_COMP32}

EXPORTED = [
    "etics_coeff_count", "etics_scf_workspace_size", "etics_scf_coeffs", "etics_scf_force",
    "etics_mex_workspace_size", "etics_mex_force", "etics_batched_workspace_size",
    "etics_scf_coeffs_noalloc", "etics_scf_coeffs_basis", "etics_scf_force_basis",
    "etics_scf_coeffs_batched", "etics_scf_force_batched", "etics_leapfrog_scf_batched",
    "etics_direct_force", "etics_set_timing_events", "etics_last_error", "etics_version",
    "etics_tuning_load", "etics_tuning_set", "etics_tuning_clear", "etics_plan_info",
    "etics_scf_coeffs_dot", "etics_scf_jerk", "etics_hermite_workspace_size", "etics_hermite_scf_batched",
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
        L.etics_scf_coeffs_noalloc.argtypes = [_vp, _vp, _vp, _vp, _i64, _int, _int, _int, _vp, _vp, _vp]
        L.etics_scf_coeffs_noalloc.restype = _int
        L.etics_scf_coeffs_basis.argtypes = [_vp, _vp, _vp, _vp, _i64, _int, _int, _int, _int, _vp, _vp,
                                             _vp, _sz, _vp]
        L.etics_scf_coeffs_basis.restype = _int
        L.etics_scf_force_basis.argtypes = [_vp, _vp, _vp, _i64, _int, _int, _vp, _vp, _int, _int, _int,
                                            _vp, _vp, _vp, _vp, _vp, _sz, _vp]
        L.etics_scf_force_basis.restype = _int
        L.etics_tuning_load.argtypes = [ctypes.c_char_p]
        L.etics_tuning_load.restype = _int
        L.etics_tuning_set.argtypes = [_int, _int, _int, _int, _int, _i64, ctypes.POINTER(_int), _int]
        L.etics_tuning_set.restype = _int
        L.etics_tuning_clear.argtypes = []
        L.etics_tuning_clear.restype = _int
        L.etics_plan_info.argtypes = [_int, _i64, _int, _int, _int, _int, ctypes.POINTER(_int), _int]
        L.etics_plan_info.restype = _int
        L.etics_scf_coeffs_dot.argtypes = [_vp] * 7 + [_i64, _int, _int, _int, _vp, _vp, _vp, _sz, _vp]
        L.etics_scf_coeffs_dot.restype = _int
        L.etics_scf_jerk.argtypes = [_vp] * 6 + [_i64, _int, _int] + [_vp] * 4 + [_int] + [_vp] * 7 + [_sz, _vp]
        L.etics_scf_jerk.restype = _int
        L.etics_hermite_workspace_size.argtypes = [_i64, _int, _int, _int, _int]
        L.etics_hermite_workspace_size.restype = _sz
        L.etics_hermite_scf_batched.argtypes = [_vp] * 8 + [_int, _i64, _int, _int, _int, ctypes.c_double, _int,
                                                            _int, _vp, _sz, _vp]
        L.etics_hermite_scf_batched.restype = _int
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


def _validate(items):
    """Check every array argument before anything is launched.

    items: (tensor or None, name, count, dtype, exact).  Sizes are checked first
    (ValueError: a tensor with `exact` must hold exactly `count` elements, otherwise at
    least `count`), then type, layout and device (TypeError): FP64 (int64 for offsets,
    any type for the workspace), contiguous, on one GPU.  The library only sees
    pointers, so a short array here would otherwise become out-of-bounds device
    accesses."""
    for t, name, count, _, exact in items:
        if t is None:
            continue
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name}: expected a torch tensor")
        k = t.numel() if name != "ws" else t.numel() * t.element_size()
        if exact and k != count:
            raise ValueError(f"{name}: {k} elements, expected {count}")
        if not exact and k < count:
            what = "bytes" if name == "ws" else "elements"
            raise ValueError(f"{name}: {k} {what}, at least {count} needed")
    device = None
    for t, name, _, dtype, _ in items:
        if t is None:
            continue
        if dtype is None:
            if not (t.is_cuda and t.is_contiguous()):
                raise TypeError(f"{name}: expected a contiguous CUDA tensor")
        else:
            _dev(t, name, dtype)
        if device is None:
            device = t.device
        elif t.device != device:
            raise TypeError(f"{name}: on {t.device}, the other arrays are on {device}")


def _nbytes(t) -> int:
    return t.numel() * t.element_size()


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


PLAN_FIELDS = ("nw", "tp", "streams", "grid_mult", "unit", "split", "phase2")


def etics_tuning_load(path: str) -> int:
    """Replace the library's tuned-plan table with the plans of a JSON file."""
    rc = lib().etics_tuning_load(os.fsencode(path))
    _check(rc if rc < 0 else 0)
    return rc


def etics_tuning_set(nmax: int, lmax: int, precision, n: int, plan: dict, batched=False,
                     basis=ETICS_BASIS_HO) -> None:
    """Add or replace one tuned plan (missing fields keep the fixed rules' values)."""
    vals = (_int * 7)(*[int(plan.get(k, 0)) for k in PLAN_FIELDS])
    _check(lib().etics_tuning_set(int(bool(batched)), nmax, lmax, _prec(precision), int(basis), int(n), vals, 7))


def etics_tuning_clear() -> None:
    _check(lib().etics_tuning_clear())


def etics_plan_info(n: int, nmax: int, lmax: int, precision, batched=False, basis=ETICS_BASIS_HO) -> dict:
    """The tile plan a coefficient call over n particles would use."""
    out = (_int * 9)()
    _check(lib().etics_plan_info(int(bool(batched)), int(n), nmax, lmax, _prec(precision), int(basis), out, 9))
    d = dict(zip(PLAN_FIELDS, out[:7]))
    d["tuned"] = bool(out[7])
    d["grid"] = out[8]
    return d


def etics_coeff_count(nmax: int, lmax: int) -> int:
    return lib().etics_coeff_count(nmax, lmax)


def etics_scf_workspace_size(n: int, nmax: int, lmax: int, precision=ETICS_MIXED_FP64ACC) -> int:
    return lib().etics_scf_workspace_size(n, nmax, lmax, _prec(precision))


def etics_mex_workspace_size(n: int, lmax: int, precision=ETICS_MIXED_FP64ACC) -> int:
    return lib().etics_mex_workspace_size(n, lmax, _prec(precision))


def etics_batched_workspace_size(ntotal: int, nsys: int, nmax: int, lmax: int,
                                 precision=ETICS_MIXED_FP64ACC) -> int:
    return lib().etics_batched_workspace_size(ntotal, nsys, nmax, lmax, _prec(precision))


F64 = torch.float64
I64 = torch.int64


def _outputs(outputs, n, device, pot, ax, ay, az):
    mk = lambda: torch.empty(n, dtype=F64, device=device)
    if outputs & ETICS_POT:
        pot = mk() if pot is None else pot
    if outputs & ETICS_ACC:
        ax = mk() if ax is None else ax
        ay = mk() if ay is None else ay
        az = mk() if az is None else az
    return pot, ax, ay, az


def _out_items(outputs, n, pot, ax, ay, az):
    if outputs not in (ETICS_POT, ETICS_ACC, ETICS_POT_ACC):
        raise ValueError("outputs must be ETICS_POT, ETICS_ACC or ETICS_POT_ACC")
    items = []
    if outputs & ETICS_POT:
        items.append((pot, "pot", n, F64, False))
    if outputs & ETICS_ACC:
        items += [(ax, "ax", n, F64, False), (ay, "ay", n, F64, False), (az, "az", n, F64, False)]
    return items


def _coeff_count_checked(nmax: int, lmax: int) -> int:
    K = etics_coeff_count(nmax, lmax)
    if K < 0:
        raise EticsError(-1, "nmax/lmax outside the caps")
    return K


def _first_tensor(x):
    if not isinstance(x, torch.Tensor):
        raise TypeError("x: expected a torch tensor")
    return x.numel(), x.device


def etics_scf_coeffs(x, y, z, m, nmax: int, lmax: int, precision=ETICS_MIXED_FP64ACC,
                     A=None, B=None, ws=None, stream=None):
    """SCF coefficients (A, B) of the particles (x, y, z, m)."""
    p = _prec(precision)
    n, device = _first_tensor(x)
    K = _coeff_count_checked(nmax, lmax)
    need = etics_scf_workspace_size(n, nmax, lmax, p)
    _validate([(x, "x", n, F64, True), (y, "y", n, F64, True), (z, "z", n, F64, True),
               (m, "m", n, F64, True), (A, "A", K, F64, False), (B, "B", K, F64, False),
               (ws, "ws", need, None, False)])
    A = torch.empty(K, dtype=F64, device=device) if A is None else A
    B = torch.empty(K, dtype=F64, device=device) if B is None else B
    ws = workspace(need, device) if ws is None else ws
    _check(lib().etics_scf_coeffs(_ptr(x), _ptr(y), _ptr(z), _ptr(m), n, nmax, lmax, p, _ptr(A), _ptr(B),
                                  _ptr(ws), _nbytes(ws), _stream(stream)))
    return A, B


def etics_scf_coeffs_noalloc(x, y, z, m, nmax: int, lmax: int, precision=ETICS_MIXED_FP64ACC,
                             A=None, B=None, stream=None):
    """SCF coefficients through the allocation-free entry point (the library's fixed
    device scratch instead of a workspace)."""
    p = _prec(precision)
    n, device = _first_tensor(x)
    K = _coeff_count_checked(nmax, lmax)
    _validate([(x, "x", n, F64, True), (y, "y", n, F64, True), (z, "z", n, F64, True),
               (m, "m", n, F64, True), (A, "A", K, F64, False), (B, "B", K, F64, False)])
    A = torch.empty(K, dtype=F64, device=device) if A is None else A
    B = torch.empty(K, dtype=F64, device=device) if B is None else B
    _check(lib().etics_scf_coeffs_noalloc(_ptr(x), _ptr(y), _ptr(z), _ptr(m), n, nmax, lmax, p, _ptr(A),
                                          _ptr(B), _stream(stream)))
    return A, B


def etics_scf_force(x, y, z, nmax: int, lmax: int, A, B, precision=ETICS_MIXED_FP64ACC,
                    outputs=ETICS_POT_ACC, pot=None, ax=None, ay=None, az=None, ws=None, stream=None):
    """SCF potential and acceleration at (x, y, z) from coefficients A, B."""
    p = _prec(precision)
    n, device = _first_tensor(x)
    K = _coeff_count_checked(nmax, lmax)
    need = etics_scf_workspace_size(n, nmax, lmax, p)
    if A is None or B is None:
        raise TypeError("A and B are required")
    _validate([(x, "x", n, F64, True), (y, "y", n, F64, True), (z, "z", n, F64, True),
               (A, "A", K, F64, False), (B, "B", K, F64, False), (ws, "ws", need, None, False)]
              + _out_items(outputs, n, pot, ax, ay, az))
    pot, ax, ay, az = _outputs(outputs, n, device, pot, ax, ay, az)
    ws = workspace(need, device) if ws is None else ws
    _check(lib().etics_scf_force(_ptr(x), _ptr(y), _ptr(z), n, nmax, lmax, _ptr(A), _ptr(B), p, outputs,
                                 _ptr(pot), _ptr(ax), _ptr(ay), _ptr(az), _ptr(ws), _nbytes(ws),
                                 _stream(stream)))
    return pot, ax, ay, az


def etics_scf_coeffs_basis(x, y, z, m, nmax: int, lmax: int, precision=ETICS_MIXED_FP64ACC,
                           basis=ETICS_BASIS_HO, A=None, B=None, ws=None, stream=None):
    """SCF coefficients (A, B) in radial basis `basis` (ETICS_BASIS_HO or ETICS_BASIS_CB)."""
    p = _prec(precision)
    n, device = _first_tensor(x)
    K = _coeff_count_checked(nmax, lmax)
    need = etics_scf_workspace_size(n, nmax, lmax, p)
    _validate([(x, "x", n, F64, True), (y, "y", n, F64, True), (z, "z", n, F64, True),
               (m, "m", n, F64, True), (A, "A", K, F64, False), (B, "B", K, F64, False),
               (ws, "ws", need, None, False)])
    A = torch.empty(K, dtype=F64, device=device) if A is None else A
    B = torch.empty(K, dtype=F64, device=device) if B is None else B
    ws = workspace(need, device) if ws is None else ws
    _check(lib().etics_scf_coeffs_basis(_ptr(x), _ptr(y), _ptr(z), _ptr(m), n, nmax, lmax, p, int(basis),
                                        _ptr(A), _ptr(B), _ptr(ws), _nbytes(ws), _stream(stream)))
    return A, B


def etics_scf_force_basis(x, y, z, nmax: int, lmax: int, A, B, precision=ETICS_MIXED_FP64ACC,
                          basis=ETICS_BASIS_HO, outputs=ETICS_POT_ACC, pot=None, ax=None, ay=None, az=None,
                          ws=None, stream=None):
    """SCF potential and acceleration from coefficients A, B of radial basis `basis`."""
    p = _prec(precision)
    n, device = _first_tensor(x)
    K = _coeff_count_checked(nmax, lmax)
    need = etics_scf_workspace_size(n, nmax, lmax, p)
    if A is None or B is None:
        raise TypeError("A and B are required")
    _validate([(x, "x", n, F64, True), (y, "y", n, F64, True), (z, "z", n, F64, True),
               (A, "A", K, F64, False), (B, "B", K, F64, False), (ws, "ws", need, None, False)]
              + _out_items(outputs, n, pot, ax, ay, az))
    pot, ax, ay, az = _outputs(outputs, n, device, pot, ax, ay, az)
    ws = workspace(need, device) if ws is None else ws
    _check(lib().etics_scf_force_basis(_ptr(x), _ptr(y), _ptr(z), n, nmax, lmax, _ptr(A), _ptr(B), p,
                                       int(basis), outputs, _ptr(pot), _ptr(ax), _ptr(ay), _ptr(az),
                                       _ptr(ws), _nbytes(ws), _stream(stream)))
    return pot, ax, ay, az


def etics_mex_force(x, y, z, m, lmax: int, precision=ETICS_MIXED_FP64ACC, outputs=ETICS_POT_ACC,
                    pot=None, ax=None, ay=None, az=None, ws=None, stream=None):
    """MEX potential and acceleration of every particle from all the others."""
    p = _prec(precision)
    n, device = _first_tensor(x)
    need = etics_mex_workspace_size(n, lmax, p)
    _validate([(x, "x", n, F64, True), (y, "y", n, F64, True), (z, "z", n, F64, True),
               (m, "m", n, F64, True), (ws, "ws", need, None, False)]
              + _out_items(outputs, n, pot, ax, ay, az))
    pot, ax, ay, az = _outputs(outputs, n, device, pot, ax, ay, az)
    ws = workspace(need, device) if ws is None else ws
    _check(lib().etics_mex_force(_ptr(x), _ptr(y), _ptr(z), _ptr(m), n, lmax, p, outputs,
                                 _ptr(pot), _ptr(ax), _ptr(ay), _ptr(az), _ptr(ws), _nbytes(ws),
                                 _stream(stream)))
    return pot, ax, ay, az


def etics_direct_force(x, y, z, m, outputs=ETICS_POT_ACC, pot=None, ax=None, ay=None, az=None,
                       stream=None):
    """Unsoftened FP64 direct-summation potential and acceleration (O(n^2))."""
    n, device = _first_tensor(x)
    _validate([(x, "x", n, F64, True), (y, "y", n, F64, True), (z, "z", n, F64, True),
               (m, "m", n, F64, True)] + _out_items(outputs, n, pot, ax, ay, az))
    pot, ax, ay, az = _outputs(outputs, n, device, pot, ax, ay, az)
    _check(lib().etics_direct_force(_ptr(x), _ptr(y), _ptr(z), _ptr(m), n, outputs, _ptr(pot), _ptr(ax),
                                    _ptr(ay), _ptr(az), _stream(stream)))
    return pot, ax, ay, az


def _nsys_of(offsets) -> int:
    if not isinstance(offsets, torch.Tensor):
        raise TypeError("offsets: expected a torch tensor")
    nsys = offsets.numel() - 1
    if nsys < 1:
        raise ValueError("offsets: needs nsys + 1 >= 2 entries")
    return nsys


def etics_scf_coeffs_batched(x, y, z, m, offsets, nmax: int, lmax: int, precision=ETICS_MIXED_FP64ACC,
                             A=None, B=None, ws=None, stream=None):
    """Coefficients of nsys systems stored back to back (offsets: int64 [nsys+1])."""
    p = _prec(precision)
    n, device = _first_tensor(x)
    nsys = _nsys_of(offsets)
    K = _coeff_count_checked(nmax, lmax)
    need = etics_batched_workspace_size(n, nsys, nmax, lmax, p)
    _validate([(x, "x", n, F64, True), (y, "y", n, F64, True), (z, "z", n, F64, True),
               (m, "m", n, F64, True), (offsets, "offsets", nsys + 1, I64, True),
               (A, "A", nsys * K, F64, False), (B, "B", nsys * K, F64, False),
               (ws, "ws", need, None, False)])
    A = torch.empty(nsys * K, dtype=F64, device=device) if A is None else A
    B = torch.empty(nsys * K, dtype=F64, device=device) if B is None else B
    ws = workspace(need, device) if ws is None else ws
    _check(lib().etics_scf_coeffs_batched(_ptr(x), _ptr(y), _ptr(z), _ptr(m), _ptr(offsets), nsys, n,
                                          nmax, lmax, p, _ptr(A), _ptr(B), _ptr(ws), _nbytes(ws),
                                          _stream(stream)))
    return A, B


def etics_scf_force_batched(x, y, z, offsets, nmax: int, lmax: int, A, B, precision=ETICS_MIXED_FP64ACC,
                            outputs=ETICS_POT_ACC, pot=None, ax=None, ay=None, az=None, ws=None,
                            stream=None):
    """Potential and acceleration of nsys systems, each from its own coefficients."""
    p = _prec(precision)
    n, device = _first_tensor(x)
    nsys = _nsys_of(offsets)
    K = _coeff_count_checked(nmax, lmax)
    need = etics_batched_workspace_size(n, nsys, nmax, lmax, p)
    if A is None or B is None:
        raise TypeError("A and B are required")
    _validate([(x, "x", n, F64, True), (y, "y", n, F64, True), (z, "z", n, F64, True),
               (offsets, "offsets", nsys + 1, I64, True), (A, "A", nsys * K, F64, False),
               (B, "B", nsys * K, F64, False), (ws, "ws", need, None, False)]
              + _out_items(outputs, n, pot, ax, ay, az))
    pot, ax, ay, az = _outputs(outputs, n, device, pot, ax, ay, az)
    ws = workspace(need, device) if ws is None else ws
    _check(lib().etics_scf_force_batched(_ptr(x), _ptr(y), _ptr(z), _ptr(offsets), nsys, n, nmax, lmax,
                                         _ptr(A), _ptr(B), p, outputs, _ptr(pot), _ptr(ax), _ptr(ay),
                                         _ptr(az), _ptr(ws), _nbytes(ws), _stream(stream)))
    return pot, ax, ay, az


def etics_leapfrog_scf_batched(x, y, z, vx, vy, vz, m, offsets, nmax: int, lmax: int, dt: float,
                               nsteps: int, precision=ETICS_MIXED_FP64ACC, flags: int = 0, ws=None,
                               stream=None):
    """Advance x..vz in place by nsteps KDK steps (one captured graph replayed)."""
    p = _prec(precision)
    n, device = _first_tensor(x)
    nsys = _nsys_of(offsets)
    _coeff_count_checked(nmax, lmax)
    need = etics_batched_workspace_size(n, nsys, nmax, lmax, p)
    _validate([(x, "x", n, F64, True), (y, "y", n, F64, True), (z, "z", n, F64, True),
               (vx, "vx", n, F64, True), (vy, "vy", n, F64, True), (vz, "vz", n, F64, True),
               (m, "m", n, F64, True), (offsets, "offsets", nsys + 1, I64, True),
               (ws, "ws", need, None, False)])
    ws = workspace(need, device) if ws is None else ws
    _check(lib().etics_leapfrog_scf_batched(_ptr(x), _ptr(y), _ptr(z), _ptr(vx), _ptr(vy), _ptr(vz),
                                            _ptr(m), _ptr(offsets), nsys, n, nmax, lmax, p, float(dt),
                                            int(nsteps), int(flags), _ptr(ws), _nbytes(ws), _stream(stream)))


def etics_scf_coeffs_dot(x, y, z, vx, vy, vz, m, nmax: int, lmax: int, precision=ETICS_MIXED_FP64ACC,
                         Adot=None, Bdot=None, ws=None, stream=None):
    """Time derivatives dA/dt, dB/dt of the coefficients along the velocities."""
    p = _prec(precision)
    n, device = _first_tensor(x)
    K = _coeff_count_checked(nmax, lmax)
    need = etics_scf_workspace_size(n, nmax, lmax, p)
    _validate([(x, "x", n, F64, True), (y, "y", n, F64, True), (z, "z", n, F64, True),
               (vx, "vx", n, F64, True), (vy, "vy", n, F64, True), (vz, "vz", n, F64, True),
               (m, "m", n, F64, True), (Adot, "Adot", K, F64, False), (Bdot, "Bdot", K, F64, False),
               (ws, "ws", need, None, False)])
    Adot = torch.empty(K, dtype=F64, device=device) if Adot is None else Adot
    Bdot = torch.empty(K, dtype=F64, device=device) if Bdot is None else Bdot
    ws = workspace(need, device) if ws is None else ws
    _check(lib().etics_scf_coeffs_dot(_ptr(x), _ptr(y), _ptr(z), _ptr(vx), _ptr(vy), _ptr(vz), _ptr(m), n, nmax,
                                      lmax, p, _ptr(Adot), _ptr(Bdot), _ptr(ws), _nbytes(ws), _stream(stream)))
    return Adot, Bdot


def etics_scf_jerk(x, y, z, vx, vy, vz, nmax: int, lmax: int, A, B, Adot, Bdot, precision=ETICS_MIXED_FP64ACC,
                   out=None, ws=None, stream=None):
    """Acceleration and jerk (ax, ay, az, jx, jy, jz) at points moving with (vx, vy, vz)."""
    p = _prec(precision)
    n, device = _first_tensor(x)
    K = _coeff_count_checked(nmax, lmax)
    need = etics_scf_workspace_size(n, nmax, lmax, p)
    out = [None] * 6 if out is None else list(out)
    _validate([(x, "x", n, F64, True), (y, "y", n, F64, True), (z, "z", n, F64, True),
               (vx, "vx", n, F64, True), (vy, "vy", n, F64, True), (vz, "vz", n, F64, True),
               (A, "A", K, F64, False), (B, "B", K, F64, False), (Adot, "Adot", K, F64, False),
               (Bdot, "Bdot", K, F64, False), (ws, "ws", need, None, False)]
              + [(o, f"out[{k}]", n, F64, False) for k, o in enumerate(out)])
    out = [torch.empty(n, dtype=F64, device=device) if o is None else o for o in out]
    ws = workspace(need, device) if ws is None else ws
    _check(lib().etics_scf_jerk(_ptr(x), _ptr(y), _ptr(z), _ptr(vx), _ptr(vy), _ptr(vz), n, nmax, lmax, _ptr(A),
                                _ptr(B), _ptr(Adot), _ptr(Bdot), p, *[_ptr(o) for o in out], _ptr(ws), _nbytes(ws),
                                _stream(stream)))
    return tuple(out)


def etics_hermite_workspace_size(ntotal: int, nsys: int, nmax: int, lmax: int,
                                 precision=ETICS_MIXED_FP64ACC) -> int:
    return lib().etics_hermite_workspace_size(ntotal, nsys, nmax, lmax, _prec(precision))


def etics_hermite_scf_batched(x, y, z, vx, vy, vz, m, offsets, nmax: int, lmax: int, dt: float,
                              nsteps: int, precision=ETICS_MIXED_FP64ACC, flags: int = 0, ws=None,
                              stream=None):
    """Advance x..vz in place by nsteps fourth-order Hermite steps (one captured graph replayed)."""
    p = _prec(precision)
    n, device = _first_tensor(x)
    nsys = _nsys_of(offsets)
    _coeff_count_checked(nmax, lmax)
    need = etics_hermite_workspace_size(n, nsys, nmax, lmax, p)
    _validate([(x, "x", n, F64, True), (y, "y", n, F64, True), (z, "z", n, F64, True),
               (vx, "vx", n, F64, True), (vy, "vy", n, F64, True), (vz, "vz", n, F64, True),
               (m, "m", n, F64, True), (offsets, "offsets", nsys + 1, I64, True),
               (ws, "ws", need, None, False)])
    ws = workspace(need, device) if ws is None else ws
    _check(lib().etics_hermite_scf_batched(_ptr(x), _ptr(y), _ptr(z), _ptr(vx), _ptr(vy), _ptr(vz), _ptr(m),
                                           _ptr(offsets), nsys, n, nmax, lmax, p, float(dt), int(nsteps),
                                           int(flags), _ptr(ws), _nbytes(ws), _stream(stream)))
