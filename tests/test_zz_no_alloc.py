"""The allocation-free coefficient entry point (etics_scf_coeffs_noalloc) against the
workspace entry point (etics_scf_coeffs), through the C-ABI."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_1406_4254_amd import workloads as W  # noqa: E402

FP64, MIXED, COMP32 = 0, 1, 2


@pytest.fixture(scope="module")
def E():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1406_4254_amd import etics
    etics.lib()
    return etics


def dev(p):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (p.x, p.y, p.z, p.m)]


@pytest.mark.parametrize("prec", [FP64, MIXED, COMP32])
@pytest.mark.parametrize("nmax,lmax", [(10, 10), (20, 14), (8, 6)])
def test_noalloc_equals_workspace_call(E, prec, nmax, lmax):
    """Two calls in a row, the second with fewer particles: both equal the workspace
    entry point's result bit for bit (same kernels, same plan, same summation order),
    so the shared scratch keeps nothing from the first call that the second reads."""
    import torch
    for n in (200_003, 7_001):
        p = W.make_config(2, n)
        x, y, z, m = dev(p)
        A0, B0 = E.etics_scf_coeffs(x, y, z, m, nmax, lmax, prec)
        A1, B1 = E.etics_scf_coeffs_noalloc(x, y, z, m, nmax, lmax, prec)
        torch.cuda.synchronize()
        print(f"noalloc ({nmax},{lmax}) prec{prec} n={n}: max |dA| {float((A1 - A0).abs().max()):.3e}",
              flush=True)
        assert torch.equal(A0, A1) and torch.equal(B0, B1)


def test_noalloc_zero_particles_and_errors(E):
    import torch
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    K = E.etics_coeff_count(4, 3)
    A = torch.full((K,), 7.0, dtype=torch.float64, device="cuda")
    B = A.clone()
    E.etics_scf_coeffs_noalloc(e, e, e, e, 4, 3, MIXED, A, B)
    assert float(A.abs().max()) == 0.0 and float(B.abs().max()) == 0.0
    # arguments outside the caps are rejected by the library before any device work
    L = E.lib()
    assert L.etics_scf_coeffs_noalloc(None, None, None, None, 0, 4, 30, MIXED, A.data_ptr(), B.data_ptr(),
                                      None) == -1
    assert L.etics_scf_coeffs_noalloc(None, None, None, None, 10, 4, 3, MIXED, A.data_ptr(), B.data_ptr(),
                                      None) == -1
