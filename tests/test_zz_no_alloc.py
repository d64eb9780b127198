"""The allocation-free butterfly product (bfmf_bf_apply_noalloc) against the
allocating one (bfmf_bf_apply), through the C ABI: equal bit for bit on two
calls in a row (the second smaller), no device allocation by the library
during the calls, and a clear error for a product larger than the fixed
scratch array."""
import numpy as np
import pytest

from workloads import rng_for

pytestmark = pytest.mark.gpu


def _fourier(m, n):
    x = (np.arange(m) + 0.5) / m
    xi = np.arange(n) - n / 2
    return np.exp(2j * np.pi * np.outer(x, xi) * 0.25)


def _dev(torch, A):
    """A (rows x cols, complex128) as a column-major device array: a (cols, rows) torch tensor."""
    return torch.from_numpy(np.ascontiguousarray(np.asarray(A).T)).to("cuda")


def test_noalloc_product_equals_the_allocating_product(gpu_lib):
    import torch
    K = _fourier(300, 280)
    b, shape = gpu_lib.bfmf_bf_compress_dense(K, 3, 1e-6, method=1, samples=32, seed=5)
    try:
        rng = rng_for("test", "rhs", (300, 280))
        cases = []
        for nrhs in (17, 5):  # the second call smaller than the first
            for adjoint in (False, True):
                nin = shape[0] if adjoint else shape[1]
                X = rng.standard_normal((nin, nrhs)) + 1j * rng.standard_normal((nin, nrhs))
                cases.append((adjoint, X, gpu_lib.bfmf_bf_apply(b, shape, X, adjoint=adjoint)))
        devs = [(_dev(torch, X), torch.zeros((X.shape[1], Y.shape[0]), dtype=torch.complex128, device="cuda"))
                for _, X, Y in cases]
        torch.cuda.synchronize()
        before = gpu_lib.bfmf_device_allocation_count()
        for (adjoint, X, Y), (dX, dY) in zip(cases, devs):
            print(f"noalloc product: adjoint {adjoint} nrhs {X.shape[1]}", flush=True)
            st = gpu_lib.bfmf_bf_apply_noalloc(b, adjoint, X.shape[1], dX.data_ptr(), X.shape[0], dY.data_ptr(),
                                               Y.shape[0])
            assert st == gpu_lib.BFMF_OK, gpu_lib.bfmf_last_error(None)
            got = dY.cpu().numpy().T
            assert np.array_equal(got, Y), np.abs(got - Y).max()
        assert gpu_lib.bfmf_device_allocation_count() == before
    finally:
        gpu_lib.bfmf_bf_destroy(b)


def test_noalloc_product_refuses_more_than_the_fixed_scratch(gpu_lib):
    import torch
    K = _fourier(256, 256)
    b, shape = gpu_lib.bfmf_bf_compress_dense(K, 2, 1e-6, method=1, samples=32, seed=5)
    try:
        nrhs = 40000  # inter-level workspace of about 2 x 256 x nrhs x 16 bytes > 64 MiB
        dX = torch.zeros((nrhs, 256), dtype=torch.complex128, device="cuda")
        dY = torch.zeros((nrhs, 256), dtype=torch.complex128, device="cuda")
        st = gpu_lib.bfmf_bf_apply_noalloc(b, False, nrhs, dX.data_ptr(), 256, dY.data_ptr(), 256)
        assert st == gpu_lib.BFMF_E_INVAL
        assert "scratch" in gpu_lib.bfmf_last_error(None)
    finally:
        gpu_lib.bfmf_bf_destroy(b)
