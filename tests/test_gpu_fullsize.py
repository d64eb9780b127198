"""Parity at the full sizes of the measured workloads, in the launch
configuration the benchmark times: batched form, complex64 butterflies with
FP64 pivot blocks and GMRES, tol 1e-3, fronts with #I^s >= 1024 compressed,
64 samples per block, separators bisected down to the workload's leaf size.

The oracle cannot factor these grids whole, so the checks are
  * sampled outputs it computes one by one: dense fronts (leaves, and parents
    of leaves) assembled and factored by the oracle (Alg. 1: the leaves from
    A alone, the parents from A and the oracle's own leaf contribution
    blocks); at the leaves the GPU's factor panels [L U; F21'], F12' and
    pivots equal the oracle's, at the parents (whose children's Schur
    products ran on FP32 MFMA in the complex64 form) the GPU's factors
    reproduce the oracle's assembled front to 1e-5;
  * properties that hold at any size: every column's true FP64 residual at
    most 1e-3 after GMRES (Sec. 6 stopping rule) within a bounded number of
    iterations (a poor HOD-BF inverse would show as many more), every front
    with #I^s >= n_min compressed, compressed factors smaller than exact ones;
  * the error against the uncompressed factorization of the same grid on the
    GPU (complex128, no front compressed), which stands in for the oracle's
    solution at these sizes: the exact GPU path equals the oracle's
    multifrontal LU on every grid the oracle factors (the dense-front tests),
    and the compressed solution must be within 10 eps of it.
"""
import numpy as np
import pytest

from workloads import make_problem
from oracle import nd
from oracle import multifrontal as mf
from oracle.symbolic import symbolic

pytestmark = pytest.mark.gpu

N_MIN = 1024


def _analyze(gpu_lib, p):
    s = gpu_lib.Solver(0)
    sl = p.opts.get("sep_leaf", 64)
    if p.kind == "grid":
        s.analyze(p.rowptr, p.colind, p.values, dims=p.dims, sep_leaf=sl)
        od = nd.nd_grid(p.dims, leaf_max=512, sep_leaf=sl)
    else:
        s.analyze(p.rowptr, p.colind, p.values, coords=p.coords, cells=p.cells, sep_leaf=sl)
        od = nd.nd_yee(p.cells, p.coords, leaf_max=512, sep_leaf=sl)
    return s, od


def _sampled_fronts(od):
    leaves = [f for f in range(od.nfronts) if od.leaf[f]]
    parents = [f for f in range(od.nfronts)
               if not od.leaf[f] and od.children[f] and all(od.leaf[c] for c in od.children[f])]
    pick = lambda xs: sorted({xs[0], xs[len(xs) // 2], xs[-1]})
    return pick(leaves) + pick(parents)


@pytest.mark.parametrize("name", ["helmholtz100", "helmholtz128grf", "maxwell64", "acoustic64"])
def test_full_size_workload(gpu_lib, name):
    p = make_problem(name)
    print(f"\n[fullsize] {name}: N={p.n} nrhs={p.rhs.shape[1]}", flush=True)
    s, od = _analyze(gpu_lib, p)
    try:
        s.factor(tol=1e-3, n_min=N_MIN, precision=gpu_lib.BFMF_C64_MIXED, batched=True)
        st = s.stats()
        ns = od.send - od.sbeg
        assert st["compressed_fronts"] == int(np.sum(ns >= N_MIN))
        assert st["factor_bytes"] < st["dense_factor_bytes"]
        X, info = s.solve(p.rhs, true_rtol=1e-3)
        res = mf.rel_residual(p.rowptr, p.colind, p.values, X, p.rhs)
        print(f"[fullsize] {name}: iters {info['iters']} relres max {res.max():.2e} "
              f"compressed {st['compressed_fronts']} max rank {st['max_rank']}", flush=True)
        assert info["status"] == 0 and res.max() <= 1e-3, (res.max(), info)
        assert info["iters"] <= 15, info

        sym = symbolic(p.rowptr, p.colind, od)
        for f in _sampled_fronts(od):
            nsf = int(ns[f])
            cbs = {}
            for c in od.children[f]:  # leaves: assembled from A alone
                Fc = mf.assemble_front(p.rowptr, p.colind, p.values, od, sym, c, {})
                cbs[c] = mf.partial_lu(Fc, int(ns[c]))[4]
            want = mf.assemble_front(p.rowptr, p.colind, p.values, od, sym, f, cbs)
            lu, opiv, F12, F21, _ = mf.partial_lu(want.copy(), nsf)
            Ff = s.front(f, 1)
            piv = s.front(f, 2)
            scale = max(1.0, np.abs(want).max())
            assert not np.any(Ff[nsf:, nsf:]), "contribution block is not kept without keep_fronts"
            if od.leaf[f]:  # assembled from A alone, factored in FP64: the oracle's factors
                assert np.array_equal(piv, opiv), f"front {f}: pivots differ"
                for got, ref in ((Ff[:nsf, :nsf], lu), (Ff[nsf:, :nsf], F21), (Ff[:nsf, nsf:], F12)):
                    assert np.abs(got - ref).max(initial=0.0) <= 1e-11 * scale, f"front {f}"
                continue
            # a parent of leaves: its children's Schur products ran on FP32 MFMA (complex64 form), so
            # the GPU front is the oracle's to about 1e-7; its factors reproduce the oracle's front
            L = np.tril(Ff[:nsf, :nsf], -1) + np.eye(nsf)
            U = np.triu(Ff[:nsf, :nsf])
            order = mf.swaps_to_perm(piv)
            F11 = want[:nsf, :nsf]
            assert np.linalg.norm(L @ U - F11[order]) <= 1e-5 * np.linalg.norm(F11), f"front {f}"
            assert np.linalg.norm(Ff[nsf:, :nsf] @ U - want[nsf:, :nsf]) <= 1e-5 * np.linalg.norm(F11), f"front {f}"
            assert np.linalg.norm(L @ Ff[:nsf, nsf:] - want[:nsf, nsf:][order]) <= 1e-5 * np.linalg.norm(F11), \
                f"front {f}"
        s.close()
        # proxy for the oracle's solution: the uncompressed factorization on the GPU
        s, _ = _analyze(gpu_lib, p)
        s.factor(tol=1e-3, n_min=0, precision=gpu_lib.BFMF_C128, batched=True)
        Xe, info_e = s.solve(p.rhs, true_rtol=1e-10, rtol=1e-12, atol=0.0)
        err = np.linalg.norm(X - Xe) / np.linalg.norm(Xe)
        print(f"[fullsize] {name}: error against the exact GPU solve {err:.2e} "
              f"(exact: {info_e['iters']} iterations, relres {info_e['relres']:.1e})", flush=True)
        assert info_e["status"] == 0 and info_e["iters"] <= 2, info_e
        assert err <= 1e-2, err
    finally:
        s.close()
