"""GPU parity on the other workload shapes: the Yee curl-curl operator
(indefinite, piecewise permittivity, edge nested dissection), the Helmholtz
operator with a heterogeneous Gaussian-random-field velocity, and the
27-point visco-acoustic operator with absorbing layers.

Compressed fronts in both precisions against the exact FP64 oracle: the
GMRES solution within 10 tol and a true residual at most 1e-3."""
import numpy as np
import pytest

from workloads import make_problem, rng_for
from workloads.maxwell import yee_curlcurl, block_permittivity
from oracle import nd
from oracle import multifrontal as mf

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_maxwell_yee_compressed(gpu_lib, precision):
    cells = 10
    eps = block_permittivity(cells, 4, rng_for("test", "coef", (cells,)))
    rp, ci, v, meta = yee_curlcurl(cells, 0.03, eps_cells=eps)
    n = rp.shape[0] - 1
    rng = rng_for("test", "rhs", (cells,))
    B = np.zeros((n, 3), dtype=np.complex128)
    B[rng.choice(n, 3, replace=False), np.arange(3)] = 1.0
    od = nd.nd_yee(cells, meta["coords"], leaf_max=64, sep_leaf=32)
    x_or = mf.solve(mf.factor(rp, ci, v, od), B)
    s = gpu_lib.Solver(0).analyze(rp, ci, v, coords=meta["coords"], cells=cells, leaf_max=64, sep_leaf=32)
    prec = gpu_lib.BFMF_C128 if precision == "c128" else gpu_lib.BFMF_C64_MIXED
    s.factor(tol=1e-3, n_min=100, batched=True, precision=prec)
    st = s.stats()
    assert st["compressed_fronts"] >= 1
    X, info = s.solve(B, true_rtol=1e-3)
    err = np.linalg.norm(X - x_or) / np.linalg.norm(x_or)
    res = mf.rel_residual(rp, ci, v, X, B).max()
    assert info["status"] == 0 and err <= 1e-2 and res <= 1e-3, (err, res, info, st["compressed_fronts"])
    s.close()


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_grf_velocity_compressed(gpu_lib, precision):
    p = make_problem("helmholtz128grf", n=16, nrhs=4)
    # the velocity from the diagonal 6 - (omega h / c)^2 (1 + i delta): heterogeneous, within [1, 2]
    A = mf.csr_matrix(p.rowptr, p.colind, p.values)
    c = p.meta["omega"] * p.meta["h"] / np.sqrt(6.0 - A.diagonal().real)
    assert c.min() >= 1.0 - 1e-9 and c.max() <= 2.0 + 1e-9 and c.max() - c.min() > 0.2
    od = nd.nd_grid(p.dims, leaf_max=64, sep_leaf=32)
    x_or = mf.solve(mf.factor(p.rowptr, p.colind, p.values, od), p.rhs)
    s = gpu_lib.Solver(0).analyze(p.rowptr, p.colind, p.values, dims=p.dims, leaf_max=64, sep_leaf=32)
    prec = gpu_lib.BFMF_C128 if precision == "c128" else gpu_lib.BFMF_C64_MIXED
    s.factor(tol=1e-3, n_min=60, batched=True, precision=prec)
    assert s.stats()["compressed_fronts"] >= 3
    X, info = s.solve(p.rhs, true_rtol=1e-3)
    err = np.linalg.norm(X - x_or) / np.linalg.norm(x_or)
    res = mf.rel_residual(p.rowptr, p.colind, p.values, X, p.rhs).max()
    assert info["status"] == 0 and err <= 1e-2 and res <= 1e-3, (err, res, info)
    s.close()


def test_poisson_compressed(gpu_lib):
    """omega = 0 (3D Poisson) on the same path, beside the Helmholtz operator of the same grid:
    both compressed solves within the bound."""
    for name in ("poisson100", "helmholtz100"):
        p = make_problem(name, n=20, nrhs=2)
        od = nd.nd_grid(p.dims, leaf_max=64, sep_leaf=32)
        x_or = mf.solve(mf.factor(p.rowptr, p.colind, p.values, od), p.rhs)
        s = gpu_lib.Solver(0).analyze(p.rowptr, p.colind, p.values, dims=p.dims, leaf_max=64, sep_leaf=32)
        s.factor(tol=1e-3, n_min=100, batched=True, precision=gpu_lib.BFMF_C64_MIXED)
        st = s.stats()
        assert st["compressed_fronts"] >= 3
        X, info = s.solve(p.rhs, true_rtol=1e-3)
        err = np.linalg.norm(X - x_or) / np.linalg.norm(x_or)
        res = mf.rel_residual(p.rowptr, p.colind, p.values, X, p.rhs).max()
        assert info["status"] == 0 and err <= 1e-2 and res <= 1e-3, (name, err, res, info)
        s.close()


def _acoustic_small(n, pml):
    from workloads import acoustic_27pt, grf_velocity
    dims = (n, n, n)
    c = grf_velocity(dims, rng_for("test", "coef", (n, pml)))
    rp, ci, v, _ = acoustic_27pt(dims, c=c, pml=pml)
    N = rp.shape[0] - 1
    rng = rng_for("test", "rhs", (n, pml))
    B = np.zeros((N, 3), dtype=np.complex128)
    B[rng.choice(N, 3, replace=False), np.arange(3)] = 1.0
    return dims, rp, ci, v, B


def test_acoustic27_exact_matches_oracle(gpu_lib):
    """27-point visco-acoustic operator with absorbing layers, no compression:
    the GPU's multifrontal solve equals the oracle's (Alg. 1) to rounding."""
    dims, rp, ci, v, B = _acoustic_small(16, 3)
    od = nd.nd_grid(dims, leaf_max=64, sep_leaf=32)
    x_or = mf.solve(mf.factor(rp, ci, v, od), B)
    s = gpu_lib.Solver(0).analyze(rp, ci, v, dims=dims, leaf_max=64, sep_leaf=32)
    s.factor(tol=1e-3, n_min=1 << 30, batched=True, precision=gpu_lib.BFMF_C128)
    assert s.stats()["compressed_fronts"] == 0
    X, info = s.solve(B, true_rtol=1e-10)
    assert info["status"] == 0
    assert np.linalg.norm(X - x_or) <= 1e-10 * np.linalg.norm(x_or)
    s.close()


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_acoustic27_compressed(gpu_lib, precision):
    """Compressed separator fronts on the 27-point operator (GRF velocity, 4
    absorbing layers per face) against the exact FP64 oracle."""
    dims, rp, ci, v, B = _acoustic_small(20, 4)
    od = nd.nd_grid(dims, leaf_max=64, sep_leaf=32)
    x_or = mf.solve(mf.factor(rp, ci, v, od), B)
    s = gpu_lib.Solver(0).analyze(rp, ci, v, dims=dims, leaf_max=64, sep_leaf=32)
    prec = gpu_lib.BFMF_C128 if precision == "c128" else gpu_lib.BFMF_C64_MIXED
    s.factor(tol=1e-3, n_min=100, batched=True, precision=prec)
    st = s.stats()
    assert st["compressed_fronts"] >= 3
    X, info = s.solve(B, true_rtol=1e-3)
    err = np.linalg.norm(X - x_or) / np.linalg.norm(x_or)
    res = mf.rel_residual(rp, ci, v, X, B).max()
    assert info["status"] == 0 and err <= 1e-2 and res <= 1e-3, (err, res, info, st["compressed_fronts"])
    s.close()


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_parallel_separators_compressed(gpu_lib, precision):
    """Separator variant (Sec. 6 remark): the top two levels of the dissection
    cut across one axis; the compressed solve on that ordering against the
    exact FP64 oracle on the same ordering."""
    p = make_problem("helmholtz100", n=20, nrhs=2)
    od = nd.nd_grid(p.dims, leaf_max=64, sep_leaf=32, parallel_levels=2)
    x_or = mf.solve(mf.factor(p.rowptr, p.colind, p.values, od), p.rhs)
    s = gpu_lib.Solver(0).analyze(p.rowptr, p.colind, p.values, dims=p.dims, leaf_max=64, sep_leaf=32,
                                  parallel_levels=2)
    sy = gpu_lib.bfmf_get_symbolic(s.h)
    assert np.array_equal(sy["perm"], od.perm)
    prec = gpu_lib.BFMF_C128 if precision == "c128" else gpu_lib.BFMF_C64_MIXED
    s.factor(tol=1e-3, n_min=100, batched=True, precision=prec)
    st = s.stats()
    assert st["compressed_fronts"] >= 3
    X, info = s.solve(p.rhs, true_rtol=1e-3)
    err = np.linalg.norm(X - x_or) / np.linalg.norm(x_or)
    res = mf.rel_residual(p.rowptr, p.colind, p.values, X, p.rhs).max()
    assert info["status"] == 0 and err <= 1e-2 and res <= 1e-3, (err, res, info)
    s.close()
