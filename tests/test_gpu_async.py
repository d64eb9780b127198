"""bfmf_solve_async: the direct solve X = M^-1 B queued on the caller's stream.

X must equal bfmf_solve's direct solve (max_iter < 0) bit for bit, and work
queued on the same stream after the call must see the finished X (the output
buffer starts as NaN, so reading it early would show).  GMRES options are
refused with E_INVAL."""
import numpy as np
import pytest

from workloads import make_problem, rng_for

pytestmark = pytest.mark.gpu


def test_solve_async_equals_the_direct_solve_in_stream_order(gpu_lib):
    import torch
    p = make_problem("helmholtz24")
    rng = rng_for("test", "rhs", (24, 3))
    B = rng.standard_normal((p.n, 3)) + 1j * rng.standard_normal((p.n, 3))
    s = gpu_lib.Solver(0).analyze(p.rowptr, p.colind, p.values, dims=p.dims)
    try:
        s.factor(tol=1e-6, n_min=256, batched=True)
        X_ref, info = s.solve(B, max_iter=-1)
        assert info["iters"] == 0
        dB = torch.from_numpy(np.ascontiguousarray(B.T)).to("cuda")
        torch.cuda.synchronize()
        stream = torch.cuda.Stream()
        outs = []
        with torch.cuda.stream(stream):
            for _ in range(2):  # the second call reuses the workspaces of the first
                dX = torch.full((3, p.n), complex(float("nan"), 0), dtype=torch.complex128, device="cuda")
                o = gpu_lib.bfmf_solve_async(s.h, dB.data_ptr(), p.n, dX.data_ptr(), p.n, 3, stream.cuda_stream)
                assert o.iters_max == 0 and o.relres_max == -1
                outs.append(dX.clone())  # queued after the solve on the same stream
        stream.synchronize()
        for out in outs:
            X = out.cpu().numpy().T
            assert np.array_equal(X, X_ref), np.nanmax(np.abs(X - X_ref))
        o = gpu_lib.bfmf_default_solve_opts()  # GMRES is not queued without the host
        st = gpu_lib._lib.bfmf_solve_async(s.h, 3, gpu_lib.C.c_void_p(dB.data_ptr()), p.n,
                                           gpu_lib.C.c_void_p(outs[0].data_ptr()), p.n, None, gpu_lib.C.byref(o))
        assert st == gpu_lib.BFMF_E_INVAL
    finally:
        s.close()
