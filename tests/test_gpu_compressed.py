"""GPU parity of the compressed-front path (Alg. 5) through the C ABI.

The oracle is the exact multifrontal solution (Alg. 1, FP64, CPU).  With
butterfly tolerance eps the compressed factorization preconditions GMRES; the
GMRES solution must match the oracle to 10 eps with a true relative residual
at most 1e-3 (1e-2 / 1e-3 at eps = 1e-3).
"""
import numpy as np
import pytest

from workloads import make_problem, helmholtz_7pt, rng_for
from oracle import nd
from oracle import multifrontal as mf

pytestmark = pytest.mark.gpu


def oracle_solution(p, leaf=512, sep_leaf=64):
    od = nd.nd_grid(p.dims, leaf_max=leaf, sep_leaf=sep_leaf)
    fac = mf.factor(p.rowptr, p.colind, p.values, od)
    return mf.solve_refined(p.rowptr, p.colind, p.values, fac, p.rhs, steps=1)


@pytest.mark.parametrize("batched", [False, True])
def test_helmholtz24_compressed_top_fronts(gpu_lib, batched):
    p = make_problem("helmholtz24")
    x_or = oracle_solution(p)
    s = gpu_lib.Solver(0).analyze(p.rowptr, p.colind, p.values, dims=p.dims)
    s.factor(tol=1e-3, n_min=256, batched=batched)
    st = s.stats()
    assert st["compressed_fronts"] == 3 and st["dense_fronts"] == 60
    assert 0 < st["max_rank"] < 576
    X, info = s.solve(p.rhs, true_rtol=1e-3)
    assert info["status"] == 0
    err = np.linalg.norm(X - x_or) / np.linalg.norm(x_or)
    res = mf.rel_residual(p.rowptr, p.colind, p.values, X, p.rhs).max()
    assert err <= 1e-2 and res <= 1e-3, (err, res, info)
    s.close()


def test_nested_compressed_fronts_and_tolerance_trend(gpu_lib):
    """Compressed fronts whose children are compressed; tighter eps -> fewer iterations."""
    dims = (16, 16, 16)
    rp, ci, v, _ = helmholtz_7pt(dims, 0.05)
    rng = rng_for("test", "rhs", (16,))
    b = rng.standard_normal((rp.shape[0] - 1, 2)) + 1j * rng.standard_normal((rp.shape[0] - 1, 2))
    od = nd.nd_grid(dims, leaf_max=64, sep_leaf=32)
    fac = mf.factor(rp, ci, v, od)
    x_or = mf.solve(fac, b)
    iters = []
    for tol in (1e-2, 1e-5):
        s = gpu_lib.Solver(0).analyze(rp, ci, v, dims=dims, leaf_max=64, sep_leaf=32)
        s.factor(tol=tol, n_min=60, batched=True)
        st = s.stats()
        assert st["compressed_fronts"] >= 3  # the root and both its children at least
        X, info = s.solve(b, true_rtol=1e-6, rtol=1e-9)
        err = np.linalg.norm(X - x_or) / np.linalg.norm(x_or)
        assert info["status"] == 0 and err <= 1e-4, (tol, err, info)
        iters.append(info["iters"])
        # the preconditioner alone: error of the order of eps times the
        # amplification of the indefinite operator (a few hundred here)
        Mx = s.precondition(b)
        assert np.linalg.norm(Mx - x_or) / np.linalg.norm(x_or) <= 1000 * tol
        s.close()
    assert iters[1] <= iters[0]


@pytest.mark.parametrize("batched", [False, True])
def test_helmholtz24_mixed_precision(gpu_lib, batched):
    """Complex64 butterflies and sketches, FP64 pivot blocks and GMRES: the same
    bound against the FP64 oracle, and the preconditioner within a small factor
    of the complex128 one."""
    p = make_problem("helmholtz24")
    x_or = oracle_solution(p)
    pre = {}
    for prec in (gpu_lib.BFMF_C128, gpu_lib.BFMF_C64_MIXED):
        s = gpu_lib.Solver(0).analyze(p.rowptr, p.colind, p.values, dims=p.dims)
        s.factor(tol=1e-3, n_min=256, batched=batched, precision=prec)
        st = s.stats()
        assert st["compressed_fronts"] == 3
        X, info = s.solve(p.rhs, true_rtol=1e-3)
        assert info["status"] == 0
        err = np.linalg.norm(X - x_or) / np.linalg.norm(x_or)
        res = mf.rel_residual(p.rowptr, p.colind, p.values, X, p.rhs).max()
        assert err <= 1e-2 and res <= 1e-3, (prec, err, res, info)
        Mx = s.precondition(p.rhs)
        pre[prec] = np.linalg.norm(Mx - x_or) / np.linalg.norm(x_or)
        if prec == gpu_lib.BFMF_C64_MIXED:
            # complex64 factors take half the bytes of complex128 ones, and less than the dense fronts
            assert st["factor_bytes"] < st["dense_factor_bytes"]
        s.close()
    assert pre[gpu_lib.BFMF_C64_MIXED] <= 3 * pre[gpu_lib.BFMF_C128] + 1e-5, pre


def test_nested_compressed_mixed_precision(gpu_lib):
    """Nested compressed fronts in the complex64 form converge to the FP64 solution."""
    dims = (16, 16, 16)
    rp, ci, v, _ = helmholtz_7pt(dims, 0.05)
    rng = rng_for("test", "rhs", (16,))
    b = rng.standard_normal((rp.shape[0] - 1, 2)) + 1j * rng.standard_normal((rp.shape[0] - 1, 2))
    od = nd.nd_grid(dims, leaf_max=64, sep_leaf=32)
    fac = mf.factor(rp, ci, v, od)
    x_or = mf.solve(fac, b)
    s = gpu_lib.Solver(0).analyze(rp, ci, v, dims=dims, leaf_max=64, sep_leaf=32)
    s.factor(tol=1e-3, n_min=60, batched=True, precision=gpu_lib.BFMF_C64_MIXED)
    assert s.stats()["compressed_fronts"] >= 3
    X, info = s.solve(b, true_rtol=1e-6, rtol=1e-9)
    err = np.linalg.norm(X - x_or) / np.linalg.norm(x_or)
    assert info["status"] == 0 and err <= 1e-4, (err, info)
    s.close()


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_autotuned_tiles_match_a_fixed_tile(gpu_lib, precision):
    """Factor and preconditioner with autotuned grouped-GEMM tile shapes equal those
    with the 64 x 64 shape forced for every launch, bit for bit."""
    dims = (16, 16, 16)
    rp, ci, v, _ = helmholtz_7pt(dims, 0.05)
    b = rng_for("test", "rhs", (16,)).standard_normal((rp.shape[0] - 1, 3)) + 0j
    prec = gpu_lib.BFMF_C128 if precision == "c128" else gpu_lib.BFMF_C64_MIXED
    out, used = [], []
    try:
        for cfg in (-1, 0):
            gpu_lib.bfmf_set_gemm_tile(cfg)
            s = gpu_lib.Solver(0).analyze(rp, ci, v, dims=dims, leaf_max=64, sep_leaf=32)
            gpu_lib.bfmf_reset_kernel_stats(s.h)
            s.factor(tol=1e-3, n_min=60, batched=True, precision=prec)
            out.append(s.precondition(b))
            used.append(s.gemm_tile_launches())
            s.close()
    finally:
        gpu_lib.bfmf_set_gemm_tile(-1)
    assert np.array_equal(out[0], out[1])
    assert sum(used[1].values()) == used[1]["64x64"] > 0
    # the autotuned run may split a phase into one launch per shape
    assert sum(used[0].values()) >= sum(used[1].values())


@pytest.mark.parametrize("precision,n_min", [("c128", 60), ("c64", 60), ("c64", 120)])
def test_graph_replayed_sweeps_equal_eager_sweeps(gpu_lib, precision, n_min):
    """GMRES with the preconditioner of its iterations replayed from a captured HIP
    graph gives the same iterates, bit for bit, as launching every sweep from the
    host: restarts every 3 iterations put eager applications, host synchronisations
    and the Krylov updates between the replays, and every replay feeds the result."""
    dims = (16, 16, 16)
    rp, ci, v, _ = helmholtz_7pt(dims, 0.05)
    b = rng_for("test", "rhs", (16,)).standard_normal((rp.shape[0] - 1, 4)) + 0j
    prec = gpu_lib.BFMF_C128 if precision == "c128" else gpu_lib.BFMF_C64_MIXED
    s = gpu_lib.Solver(0).analyze(rp, ci, v, dims=dims, leaf_max=64, sep_leaf=32)
    s.factor(tol=1e-2, n_min=n_min, batched=True, precision=prec, timing=True)
    out = {}
    for graphs in (False, True, True):
        gpu_lib.bfmf_reset_kernel_stats(s.h)
        X, info = s.solve(b, restart=3, rtol=1e-11, true_rtol=1e-8, max_iter=100, graphs=graphs)
        replays = s.kernel_stats()["preconditioner_graph"]["launches"]
        assert info["status"] == 0 and info["iters"] > 3, info
        assert (replays > 0) == graphs, replays
        if graphs in out:
            assert np.array_equal(X, out[graphs][0])  # a second call reuses or rebuilds the graph
        out[graphs] = (X, info["iters"])
    assert np.array_equal(out[True][0], out[False][0]) and out[True][1] == out[False][1]
    s.close()


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_direct_mode_and_tolerance_trend(gpu_lib, precision):
    """The compressed factorization used directly (no GMRES, max_iter < 0) at tol 1e-6, the
    direct mode of the paper's tolerance study: the solution matches the FP64 oracle to
    100 tol (complex128; 1e-3 with complex64 butterflies), and tightening tol from 1e-3 to
    1e-6 reduces the direct solve's error at least tenfold."""
    p = make_problem("helmholtz24")
    x_or = oracle_solution(p)
    prec = gpu_lib.BFMF_C128 if precision == "c128" else gpu_lib.BFMF_C64_MIXED
    err = {}
    for tol in (1e-3, 1e-6):
        s = gpu_lib.Solver(0).analyze(p.rowptr, p.colind, p.values, dims=p.dims)
        s.factor(tol=tol, n_min=256, batched=True, precision=prec)
        X, info = s.solve(p.rhs, max_iter=-1)
        assert info["iters"] == 0
        err[tol] = np.linalg.norm(X - x_or) / np.linalg.norm(x_or)
        res = mf.rel_residual(p.rowptr, p.colind, p.values, X, p.rhs).max()
        assert abs(res - info["relres"]) <= 1e-3 * res + 1e-14, (res, info)
        s.close()
    bound = 1e-4 if precision == "c128" else 1e-3
    assert err[1e-6] <= bound and err[1e-6] * 10 <= err[1e-3], err


def test_repeated_factor_and_solve_allocate_nothing(gpu_lib):
    """After a handle's first factorization and solve, factoring and solving again with the
    same sizes and options makes no device allocation (the scratch stack keeps its chunks and
    reorders them instead of freeing; a free would synchronize the device), and gives the same
    solution bit for bit."""
    dims = (20, 20, 20)
    rp, ci, v, _ = helmholtz_7pt(dims, 0.05)
    b = rng_for("test", "rhs", (20, 2)).standard_normal((rp.shape[0] - 1, 2)) + 0j
    s = gpu_lib.Solver(0).analyze(rp, ci, v, dims=dims, leaf_max=64, sep_leaf=32)
    try:
        for it in range(3):
            s.factor(tol=1e-3, n_min=100, batched=True, precision=gpu_lib.BFMF_C64_MIXED)
            X, info = s.solve(b, true_rtol=1e-3)
            assert info["status"] == 0
            if it == 0:
                count, X0 = gpu_lib.bfmf_device_allocation_count(), X
                assert count > 0
            else:
                assert gpu_lib.bfmf_device_allocation_count() == count, it
                assert np.array_equal(X, X0), it
    finally:
        s.close()
