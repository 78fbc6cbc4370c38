"""Host-side checks of the C-ABI library: it loads, exports every symbol that
include/etics.h declares, and rejects invalid arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "etics.h")
LIBPATH = os.path.join(ROOT, "paper_1406_4254_amd", "libetics.so")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIBPATH):
        from paper_1406_4254_amd import build
        build.build()
    return ctypes.CDLL(LIBPATH)


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(etics_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_three_named_calls():
    d = declared()
    for name in ("etics_scf_coeffs", "etics_scf_force", "etics_mex_force"):
        assert name in d


def test_every_declared_symbol_is_exported(L):
    for name in declared():
        assert hasattr(L, name), name


def test_binding_covers_header():
    from paper_1406_4254_amd import etics
    assert sorted(etics.EXPORTED) == declared()


def test_coeff_count(L):
    assert L.etics_coeff_count(10, 6) == 308   # Section 2.4: 308 coefficients at (10,6)
    assert L.etics_coeff_count(10, 10) == 726
    assert L.etics_coeff_count(20, 14) == 2520
    assert L.etics_coeff_count(21, 6) == -1
    assert L.etics_coeff_count(4, 15) == -1
    assert L.etics_coeff_count(-1, 2) == -1


def test_workspace_sizes(L):
    f = L.etics_scf_workspace_size
    f.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    f.restype = ctypes.c_size_t
    for prec in (0, 1, 2):
        for nmax, lmax in ((0, 0), (10, 6), (10, 10), (20, 14), (8, 6)):
            assert f(1_000_000, nmax, lmax, prec) > 0
    assert f(-1, 10, 6, 1) == 0
    assert f(100, 10, 6, 7) == 0
    assert f(100, 30, 6, 1) == 0


def test_invalid_arguments_rejected_without_device_work(L):
    c = L.etics_scf_coeffs
    c.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_size_t, ctypes.c_void_p]
    L.etics_last_error.restype = ctypes.c_char_p
    fake = ctypes.c_void_p(0x1000)
    # n < 0
    assert c(fake, fake, fake, fake, -5, 4, 4, 1, fake, fake, fake, 1 << 20, None) == -1
    # cutoffs
    assert c(fake, fake, fake, fake, 10, 21, 4, 1, fake, fake, fake, 1 << 20, None) == -1
    # precision
    assert c(fake, fake, fake, fake, 10, 4, 4, 9, fake, fake, fake, 1 << 20, None) == -1
    # NULL outputs / inputs
    assert c(fake, fake, fake, fake, 10, 4, 4, 1, None, fake, fake, 1 << 20, None) == -1
    assert c(None, fake, fake, fake, 10, 4, 4, 1, fake, fake, fake, 1 << 20, None) == -1
    assert b"NULL" in L.etics_last_error()
    # workspace too small
    assert c(fake, fake, fake, fake, 10, 4, 4, 1, fake, fake, fake, 16, None) == -2
    assert b"workspace" in L.etics_last_error()
    f = L.etics_scf_force
    f.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_int, ctypes.c_int] + \
                 [ctypes.c_void_p] * 5 + [ctypes.c_size_t, ctypes.c_void_p]
    # outputs out of range, missing pot, missing acc
    assert f(fake, fake, fake, 10, 4, 4, fake, fake, 1, 0, fake, fake, fake, fake, fake, 1 << 20, None) == -1
    assert f(fake, fake, fake, 10, 4, 4, fake, fake, 1, 1, None, fake, fake, fake, fake, 1 << 20, None) == -1
    assert f(fake, fake, fake, 10, 4, 4, fake, fake, 1, 2, fake, None, fake, fake, fake, 1 << 20, None) == -1
    # misaligned workspace
    assert f(fake, fake, fake, 10, 4, 4, fake, fake, 1, 3, fake, fake, fake, fake,
             ctypes.c_void_p(0x1008), 1 << 30, None) == -1


def test_direct_force_arguments_rejected_without_device_work(L):
    d = L.etics_direct_force
    d.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int64, ctypes.c_int] + [ctypes.c_void_p] * 5
    L.etics_last_error.restype = ctypes.c_char_p
    fake = ctypes.c_void_p(0x1000)
    assert d(fake, fake, fake, fake, -1, 3, fake, fake, fake, fake, None) == -1
    assert d(fake, fake, fake, fake, 1 << 31, 3, fake, fake, fake, fake, None) == -1
    assert d(fake, fake, fake, fake, 10, 0, fake, fake, fake, fake, None) == -1
    assert d(fake, fake, fake, None, 10, 3, fake, fake, fake, fake, None) == -1
    assert d(fake, fake, fake, fake, 10, 1, None, None, None, None, None) == -1
    assert d(fake, fake, fake, fake, 10, 2, None, fake, None, fake, None) == -1
    assert b"NULL" in L.etics_last_error()
    # n = 0 is valid and does nothing (no device work, NULL arrays allowed)
    assert d(None, None, None, None, 0, 3, None, None, None, None, None) == 0


def test_version(L):
    L.etics_version.restype = ctypes.c_char_p
    assert b"gfx950" in L.etics_version()


def test_timing_events_need_both_or_neither(L):
    t = L.etics_set_timing_events
    t.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    L.etics_last_error.restype = ctypes.c_char_p
    assert t(ctypes.c_void_p(0x1000), None) == -1
    assert b"timing" in L.etics_last_error()
    assert t(None, ctypes.c_void_p(0x1000)) == -1
    assert t(None, None) == 0  # off: stores nothing, touches no device


# ------------------------------------------------ binding: sizes checked before launch
def _cpu(n, dtype=None):
    import torch
    return torch.zeros(n, dtype=torch.float64 if dtype is None else dtype)


def test_binding_rejects_mismatched_sizes_before_any_launch():
    """Every array argument is size-checked on the host (ValueError) before its type or
    device (TypeError), so these CPU tensors never reach the library."""
    import torch

    from paper_1406_4254_amd import etics as E
    n = 100
    x, y, z, m = _cpu(n), _cpu(n), _cpu(n), _cpu(n)
    K = E.etics_coeff_count(4, 3)
    with pytest.raises(ValueError, match="y"):
        E.etics_scf_coeffs(x, _cpu(n - 1), z, m, 4, 3)
    with pytest.raises(ValueError, match="m"):
        E.etics_scf_coeffs(x, y, z, _cpu(n + 1), 4, 3)
    with pytest.raises(ValueError, match="A"):
        E.etics_scf_coeffs(x, y, z, m, 4, 3, A=_cpu(K - 1))
    with pytest.raises(ValueError, match="ws"):
        E.etics_scf_coeffs(x, y, z, m, 4, 3, ws=torch.zeros(16, dtype=torch.uint8))
    with pytest.raises(ValueError, match="B"):
        E.etics_scf_force(x, y, z, 4, 3, _cpu(K), _cpu(K - 2))
    with pytest.raises(ValueError, match="pot"):
        E.etics_scf_force(x, y, z, 4, 3, _cpu(K), _cpu(K), outputs=E.ETICS_POT, pot=_cpu(n - 1))
    with pytest.raises(ValueError, match="az"):
        E.etics_scf_force(x, y, z, 4, 3, _cpu(K), _cpu(K), outputs=E.ETICS_ACC, ax=_cpu(n), ay=_cpu(n),
                          az=_cpu(3))
    with pytest.raises(ValueError, match="outputs"):
        E.etics_scf_force(x, y, z, 4, 3, _cpu(K), _cpu(K), outputs=0)
    with pytest.raises(ValueError, match="z"):
        E.etics_mex_force(x, y, _cpu(n - 1), m, 6)
    with pytest.raises(ValueError, match="ax"):
        E.etics_mex_force(x, y, z, m, 6, ax=_cpu(1), ay=_cpu(n), az=_cpu(n))
    with pytest.raises(ValueError, match="m"):
        E.etics_direct_force(x, y, z, _cpu(n - 1))
    off = torch.tensor([0, 40, 100], dtype=torch.int64)
    with pytest.raises(ValueError, match="A"):
        E.etics_scf_coeffs_batched(x, y, z, m, off, 4, 3, A=_cpu(K))  # needs nsys * K
    with pytest.raises(ValueError, match="offsets"):
        E.etics_scf_coeffs_batched(x, y, z, m, torch.zeros(1, dtype=torch.int64), 4, 3)
    with pytest.raises(ValueError, match="B"):
        E.etics_scf_force_batched(x, y, z, off, 4, 3, _cpu(2 * K), _cpu(2 * K - 1))
    with pytest.raises(ValueError, match="vy"):
        E.etics_leapfrog_scf_batched(x, y, z, _cpu(n), _cpu(n - 1), _cpu(n), m, off, 4, 3, 0.01, 2)
    with pytest.raises(ValueError, match="m"):
        E.etics_leapfrog_scf_batched(x, y, z, _cpu(n), _cpu(n), _cpu(n), _cpu(7), off, 4, 3, 0.01, 2)


def test_binding_rejects_host_and_wrong_typed_tensors():
    import torch

    from paper_1406_4254_amd import etics as E
    n = 50
    x, y, z, m = _cpu(n), _cpu(n), _cpu(n), _cpu(n)
    with pytest.raises(TypeError, match="CUDA"):
        E.etics_scf_coeffs(x, y, z, m, 4, 3)  # right sizes, but host memory
    with pytest.raises(TypeError):
        E.etics_mex_force(x, y, z, _cpu(n, torch.float32), 6)
    off = torch.tensor([0, 50], dtype=torch.int32)
    with pytest.raises(TypeError):
        E.etics_scf_coeffs_batched(x, y, z, m, off, 4, 3)
    with pytest.raises(TypeError):
        E.etics_scf_coeffs([0.0], y, z, m, 4, 3)
    with pytest.raises(EticsErrorType()):
        E.etics_scf_coeffs(x, y, z, m, 30, 3)  # cutoffs outside the caps


def EticsErrorType():
    from paper_1406_4254_amd import etics as E
    return E.EticsError
