"""Serving: resident factorizations answer a stream of point-source requests.

A request's result must be the same, bit for bit, when it is solved alone and
when it is batched with others (GMRES keeps every column's Krylov data apart
and every kernel's arithmetic on a column is independent of the other
columns), with the request's own iteration count and residual reported, and
must match the FP64 oracle to 10 tol with a true residual at most 1e-3.
"""
import numpy as np
import pytest

from workloads import helmholtz_7pt, request_stream, rng_for
from oracle import nd
from oracle import multifrontal as mf

pytestmark = pytest.mark.gpu

GRIDS = [((14, 14, 14), 0.05), ((18, 18, 18), 0.05)]


def _models(gpu_lib, precision):
    out = []
    for dims, delta in GRIDS:
        rp, ci, v, _ = helmholtz_7pt(dims, delta)
        s = gpu_lib.Solver(0).analyze(rp, ci, v, dims=dims)
        s.factor(tol=1e-3, n_min=128, batched=True, precision=precision)
        out.append((s, rp, ci, v, dims))
    return out


def _requests(n_req, sizes):
    stream = request_stream(100.0, 10.0, sizes, 6, rng_for("test", "arrivals", (n_req,)))
    return [(m, rows) for _, m, rows in stream[:n_req]]


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_alone_equals_mix_and_oracle(gpu_lib, precision):
    prec = gpu_lib.BFMF_C128 if precision == "c128" else gpu_lib.BFMF_C64_MIXED
    models = _models(gpu_lib, prec)
    sizes = [m[0].n for m in models]
    srv = gpu_lib.Server(0, max_batch_rhs=16, result_bytes=256 << 20)
    ids = [srv.attach(m[0]) for m in models]
    reqs = _requests(14, sizes)

    alone, alone_info = [], []
    for m, rows in reqs:
        t = srv.submit_points(ids[m], rows)
        X = np.zeros((sizes[m], len(rows)), dtype=np.complex128, order="F")
        info = srv.wait(t, out=X)
        assert info["status"] == 0 and info["batch_requests"] == 1, info
        alone.append(X)
        alone_info.append(info)

    tickets = [srv.submit_points(ids[m], rows) for m, rows in reqs]
    mixed, infos = [], []
    for (m, rows), t in zip(reqs, tickets):
        X = np.zeros((sizes[m], len(rows)), dtype=np.complex128, order="F")
        infos.append(srv.wait(t, out=X))
        mixed.append(X)
    srv.close()
    assert all(i["status"] == 0 for i in infos)
    assert max(i["batch_requests"] for i in infos) > 1  # requests were batched together
    for i in infos:
        assert i["t_submit"] <= i["t_start"] <= i["t_done"] and i["batch_rhs"] <= 16

    facs = []
    for s, rp, ci, v, dims in models:
        od = nd.nd_grid(dims, leaf_max=512, sep_leaf=64)
        facs.append((mf.factor(rp, ci, v, od), rp, ci, v))
    for (m, rows), Xa, Xm, ia, im in zip(reqs, alone, mixed, alone_info, infos):
        # alone and in the mix: the same columns bit for bit, the request's own iterations and residual
        assert np.array_equal(Xm, Xa), np.abs(Xm - Xa).max()
        assert im["iters"] == ia["iters"] and im["relres"] == ia["relres"], (ia, im)
        fac, rp, ci, v = facs[m]
        B = np.zeros((sizes[m], len(rows)), dtype=np.complex128)
        B[rows, np.arange(len(rows))] = 1.0
        x_or = mf.solve(fac, B)
        err = np.linalg.norm(Xm - x_or) / np.linalg.norm(x_or)
        res = mf.rel_residual(rp, ci, v, Xm, B).max()
        assert err <= 1e-2 and res <= 1e-3, (m, err, res)
    for s, *_ in models:
        s.close()


def test_admission_by_hbm_budget(gpu_lib):
    models = _models(gpu_lib, gpu_lib.BFMF_C128)
    srv = gpu_lib.Server(0, max_batch_rhs=8, result_bytes=64 << 20, hbm_budget=(64 << 20) + 4096)
    with pytest.raises(gpu_lib.BfmfError) as e:
        srv.attach(models[0][0])
    assert e.value.status == gpu_lib.BFMF_E_NOMEM
    srv.close()
    srv = gpu_lib.Server(0, max_batch_rhs=8, result_bytes=64 << 20)
    m = srv.attach(models[0][0])
    with pytest.raises(gpu_lib.BfmfError):
        srv.submit_points(m, np.arange(9))  # wider than a batch
    with pytest.raises(gpu_lib.BfmfError):
        srv.submit_points(m, [models[0][0].n])  # row out of range
    t = srv.submit_points(m, [0, 5])
    assert srv.wait(t)["status"] == 0  # result discarded
    srv.close()
    for s, *_ in models:
        s.close()
