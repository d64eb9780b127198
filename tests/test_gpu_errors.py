"""Error conventions of the C ABI on the GPU (bfmf.h, bfmf_factor and bfmf_solve):
  * E_NOMEM when the HBM budget is too small, both for the level workspaces
    and dense factors (checked before the factorization starts) and for the
    growth of the compressed fronts' butterfly pool and scratch (checked
    during the factorization); either way the handle is back in the analyzed
    state and a later factorization within budget succeeds;
  * E_NOCONV when GMRES reaches max_iter, with X holding the last iterate
    and relres_max its largest true relative residual."""
import re

import numpy as np
import pytest

from workloads import make_problem
from oracle import nd
from oracle import multifrontal as mf

pytestmark = pytest.mark.gpu


def test_budget_too_small_returns_nomem_and_rolls_back(gpu_lib):
    p = make_problem("helmholtz24")
    s = gpu_lib.Solver(0).analyze(p.rowptr, p.colind, p.values, dims=p.dims)
    try:
        with pytest.raises(gpu_lib.BfmfError) as e:
            s.factor(tol=1e-3, n_min=256, batched=True, hbm_budget=1 << 20)
        assert e.value.status == gpu_lib.BFMF_E_NOMEM
        need = int(re.search(r"need (\d+) bytes", str(e.value)).group(1))
        # enough for the workspaces and dense factors, not for the butterflies of the compressed fronts
        with pytest.raises(gpu_lib.BfmfError) as e:
            s.factor(tol=1e-3, n_min=256, batched=True, hbm_budget=need + (1 << 20))
        assert e.value.status == gpu_lib.BFMF_E_NOMEM
        assert "budget" in str(e.value)
        with pytest.raises(gpu_lib.BfmfError) as e:  # analyzed, not factored
            s.solve(p.rhs)
        assert e.value.status == gpu_lib.BFMF_E_STATE
        s.factor(tol=1e-3, n_min=256, batched=True)
        X, info = s.solve(p.rhs, true_rtol=1e-3)
        od = nd.nd_grid(p.dims, leaf_max=512, sep_leaf=64)
        x_or = mf.solve(mf.factor(p.rowptr, p.colind, p.values, od), p.rhs)
        err = np.linalg.norm(X - x_or) / np.linalg.norm(x_or)
        assert info["status"] == 0 and err <= 1e-2, (err, info)
    finally:
        s.close()


def test_max_iter_returns_noconv_with_the_last_iterate(gpu_lib):
    p = make_problem("helmholtz24")
    s = gpu_lib.Solver(0).analyze(p.rowptr, p.colind, p.values, dims=p.dims)
    try:
        s.factor(tol=3e-1, n_min=256, batched=True)  # a poor preconditioner: one iteration is not enough
        X, info = s.solve(p.rhs, max_iter=1, true_rtol=1e-8)
        assert info["status"] == gpu_lib.BFMF_E_NOCONV and info["iters"] == 1, info
        res = mf.rel_residual(p.rowptr, p.colind, p.values, X, p.rhs)
        assert np.all(np.isfinite(X)) and np.linalg.norm(X) > 0
        assert abs(res.max() - info["relres"]) <= 1e-6 * res.max(), (res, info)
        assert info["relres"] > 1e-8
    finally:
        s.close()
