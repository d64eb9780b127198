"""Contribution blocks in HOD-BF form (Alg. 5, last step) and extraction from them (Alg. 3).

With compress_cb a compressed front whose parent is compressed keeps its
contribution block C = (C_nu1 (+) C_nu2)(Iu, Iu) - S as an HOD-BF built by
entry evaluation (each entry: list routing to the children plus extract_BF
of S), and the parent's entry evaluation reads it through extract_HODBF.
Checked against the oracle (FP64, CPU, exact fronts):
  C of each such front  vs  F22 - F21 inv(F11) F12 of the oracle's front
      (bound C eps kappa(F11), as for S; the HOD-BF adds its own eps);
  the parent's entries through the HOD-BF blocks (bfmf_extract_front) vs the
      oracle's assembled parent front (same bound with the children's kappa);
  the parent's F11 HOD-BF vs the oracle's F11;
  the solution within 10 eps of the oracle, GMRES iterations bounded;
and the level workspace shrinks by the blocks no longer held dense.
"""
import numpy as np
import pytest

from workloads import make_problem, helmholtz_7pt, rng_for
from oracle import nd
from oracle import multifrontal as mf

pytestmark = pytest.mark.gpu

TOL = 1e-3
C_CB = 10.0  # ||C_gpu - C|| <= C_CB eps kappa(F11) ||C||


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _comp(od, n_min):
    ns = od.send - od.sbeg
    return [f for f in range(od.nfronts) if len(od.children[f]) > 0 and ns[f] >= n_min]


@pytest.fixture(scope="module")
def c1():
    p = make_problem("helmholtz24")
    od = nd.nd_grid(p.dims, leaf_max=512, sep_leaf=64)
    fac = mf.factor(p.rowptr, p.colind, p.values, od, keep_fronts=True)
    x_or = mf.solve_refined(p.rowptr, p.colind, p.values, fac, p.rhs, steps=1)
    return p, od, fac, x_or


def _oracle_cb(fac, f):
    F = fac.fronts[f]
    ns = int(fac.od.send[f] - fac.od.sbeg[f])
    F11, F12, F21, F22 = F[:ns, :ns], F[:ns, ns:], F[ns:, :ns], F[ns:, ns:]
    return F22 - F21 @ np.linalg.solve(F11, F12), np.linalg.cond(F11)


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_cb_hodbf_24(gpu_lib, c1, precision):
    p, od, fac, x_or = c1
    prec = gpu_lib.BFMF_C128 if precision == "c128" else gpu_lib.BFMF_C64_MIXED
    comp = set(_comp(od, 256))
    cbf = [f for f in comp if od.parent[f] >= 0 and od.parent[f] in comp]
    assert len(cbf) == 2  # the two level-1 separators, children of the compressed root
    res = {}
    for cb in (0, 1):
        s = gpu_lib.Solver(0).analyze(p.rowptr, p.colind, p.values, dims=p.dims)
        s.factor(tol=TOL, n_min=256, batched=True, precision=prec, keep_fronts=True, compress_cb=cb)
        st = s.stats()
        assert st["compressed_fronts"] == 3 and st["cb_compressed"] == (2 if cb else 0), st
        X, info = s.solve(p.rhs, true_rtol=1e-3)
        err = np.linalg.norm(X - x_or) / np.linalg.norm(x_or)
        print(f"{precision} compress_cb {cb}: error {err:.2e}, iterations {info['iters']}, workspace "
              f"{st['workspace_bytes'] / 1e6:.1f} MB, HOD-BF blocks {st['cb_bytes'] / 1e6:.2f} MB for "
              f"{st['cb_dense_bytes'] / 1e6:.2f} MB dense", flush=True)
        assert info["status"] == 0 and err <= 10 * TOL and info["iters"] <= 8, (cb, err, info)
        res[cb] = (st, err)
        if cb:
            kap = {}
            for f in cbf:
                C, kappa = _oracle_cb(fac, f)
                kap[f] = kappa
                nu = C.shape[0]
                got = s.front_block(f, 5, np.eye(nu, dtype=np.complex128))
                e = _rel(got, C)
                print(f"  front {f}: nu {nu}, C error {e:.3g} (kappa {kappa:.3g})", flush=True)
                assert e <= C_CB * TOL * kappa, (f, e, kappa)
            root = [f for f in comp if od.parent[f] < 0][0]
            F = fac.fronts[root]
            n, ns = F.shape[0], int(od.send[root] - od.sbeg[root])
            kmax = max(kap.values())
            rng = rng_for("test", "rhs", (24, 11))
            reqs = [(np.arange(ns), np.arange(ns)), (np.array([ns // 2]), np.array([ns // 3])),
                    (np.array([ns - 1]), np.array([0, ns - 1]))]
            for _ in range(3):
                reqs.append((rng.integers(0, n, 41), rng.integers(0, n, 29)))
            for rows, cols in reqs:
                got = gpu_lib.bfmf_extract_front(s.h, root, rows, cols)
                want = F[np.ix_(rows, cols)]
                e = np.linalg.norm(got - want) / np.linalg.norm(F[:ns, :ns]) * np.sqrt(F[:ns, :ns].size / want.size)
                assert e <= C_CB * TOL * kmax, (rows[:3], cols[:3], e)
            F11 = F[:ns, :ns]
            e11 = _rel(s.front_block(root, 0, np.eye(ns, dtype=np.complex128)), F11)
            print(f"  root F11 from HOD-BF children blocks: error {e11:.3g}", flush=True)
            assert e11 <= C_CB * TOL * kmax
        s.close()
    assert res[1][0]["workspace_bytes"] < res[0][0]["workspace_bytes"]


def test_cb_hodbf_nested_16(gpu_lib):
    """16^3 with compressed fronts on several levels, so that HOD-BF contribution blocks are built
    from children that are themselves in HOD-BF form."""
    dims = (16, 16, 16)
    rp, ci, v, _ = helmholtz_7pt(dims, 0.05)
    rng = rng_for("test", "rhs", (16,))
    b = rng.standard_normal((rp.shape[0] - 1, 2)) + 1j * rng.standard_normal((rp.shape[0] - 1, 2))
    od = nd.nd_grid(dims, leaf_max=64, sep_leaf=16)
    fac = mf.factor(rp, ci, v, od, keep_fronts=True)
    x_or = mf.solve(fac, b)
    comp = set(_comp(od, 60))
    cbf = [f for f in comp if od.parent[f] >= 0 and od.parent[f] in comp]
    nested = [f for f in cbf if any(c in cbf for c in od.children[f])]
    assert len(nested) >= 1
    for prec in ("c128", "c64"):
        s = gpu_lib.Solver(0).analyze(rp, ci, v, dims=dims, leaf_max=64, sep_leaf=16)
        s.factor(tol=TOL, n_min=60, batched=True, compress_cb=True, keep_fronts=True,
                 precision=gpu_lib.BFMF_C128 if prec == "c128" else gpu_lib.BFMF_C64_MIXED)
        st = s.stats()
        assert st["cb_compressed"] == len(cbf), (st, len(cbf))
        X, info = s.solve(b, true_rtol=1e-3)
        err = np.linalg.norm(X - x_or) / np.linalg.norm(x_or)
        print(f"{prec}: {len(cbf)} HOD-BF blocks ({len(nested)} built from HOD-BF children), error {err:.2e}, "
              f"iterations {info['iters']}", flush=True)
        assert info["status"] == 0 and err <= 10 * TOL and info["iters"] <= 10, (err, info)
        for f in nested:
            C, kappa = _oracle_cb(fac, f)
            F = fac.fronts[f]
            ns = int(od.send[f] - od.sbeg[f])
            S = F[ns:, :ns] @ np.linalg.solve(F[:ns, :ns], F[:ns, ns:])
            e = _rel(s.front_block(f, 5, np.eye(C.shape[0], dtype=np.complex128)), C)
            es = _rel(s.front_block(f, 4, np.eye(C.shape[0], dtype=np.complex128)), S)
            # the children's blocks carry their own error into F11, amplified by kappa in S and C
            print(f"  front {f} (children in HOD-BF form): C error {e:.3g}, S error {es:.3g} "
                  f"(relative to |S|), kappa {kappa:.3g}", flush=True)
            assert e <= 3 * C_CB * TOL * kappa, (f, e, kappa)
        s.close()


def test_compress_cb_option_checked(gpu_lib):
    p = make_problem("helmholtz24", n=12, config_id="test")
    s = gpu_lib.Solver(0).analyze(p.rowptr, p.colind, p.values, dims=p.dims, leaf_max=64, sep_leaf=16)
    o = gpu_lib.bfmf_default_factor_opts()
    o.tol, o.n_min, o.compress_cb = TOL, 64, 2
    with pytest.raises(gpu_lib.BfmfError) as e:
        gpu_lib.bfmf_factor(s.h, o)
    assert e.value.status == gpu_lib.BFMF_E_INVAL
    s.factor(tol=TOL, n_min=64, compress_cb=True)
    with pytest.raises(gpu_lib.BfmfError) as e:  # the root's block is not kept (it has no parent)
        s.front_block(len(s.symbolic()["parent"]) - 1, 5, np.eye(4))
    assert e.value.status == gpu_lib.BFMF_E_INVAL
    s.close()
