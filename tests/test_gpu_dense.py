"""GPU parity of the dense multifrontal path through the C ABI.

* Extend-add (kernel a): every assembled front equals the oracle's assembly of
  the same A entries and the same child contribution blocks, bit for bit
  (FP64, same addition order).
* Partial LU (kernel d): the factored front matches the oracle's LAPACK
  partial factorization of the same assembled front (pivots equal, values
  to 1e-11 relative), also on a pattern with random values where most fronts
  interchange rows, and for a 1056-row front whose first panel runs in the
  global-memory panel kernel.
* Sweeps (kernel e) and GMRES: x matches the oracle's solve to 1e-10; with
  the exact factorization GMRES stops after one iteration.
"""
import numpy as np
import pytest

from workloads import helmholtz_7pt, make_problem, rng_for
from oracle import nd
from oracle.symbolic import symbolic
from oracle import multifrontal as mf

pytestmark = pytest.mark.gpu


def maxabs(a):
    return float(np.abs(a).max()) if a.size else 0.0


def _setup(lib, dims, leaf, sl=16, batched=False, delta=0.05):
    rp, ci, v, _ = helmholtz_7pt(dims, delta)
    s = lib.Solver(0).analyze(rp, ci, v, dims=dims, leaf_max=leaf, sep_leaf=sl)
    s.factor(n_min=0, batched=batched, keep_fronts=True)
    od = nd.nd_grid(dims, leaf_max=leaf, sep_leaf=sl)
    sym = symbolic(rp, ci, od)
    return s, (rp, ci, v), od, sym


@pytest.mark.parametrize("dims,leaf,batched", [((8, 8, 8), 64, False), ((9, 7, 6), 40, True),
                                               ((24, 24, 24), 512, True)])
def test_extend_add_bit_exact_and_partial_lu(gpu_lib, dims, leaf, batched):
    s, (rp, ci, v), od, sym = _setup(gpu_lib, dims, leaf, batched=batched)
    gpu_cb = {}
    for f in range(od.nfronts):
        ns = int(od.send[f] - od.sbeg[f])
        Fa = s.front(f, 0)
        Ff = s.front(f, 1)
        piv = s.front(f, 2)
        # oracle assembly of the same A entries and the GPU's child blocks
        want = mf.assemble_front(rp, ci, v, od, sym, f, gpu_cb)
        assert np.array_equal(Fa, want), f"front {f}: assembly differs"
        lu, opiv, F12, F21, C = mf.partial_lu(want.copy(), ns)
        assert np.array_equal(piv, opiv), f"front {f}: pivots differ"
        scale = max(1.0, np.abs(want).max())
        assert maxabs(Ff[:ns, :ns] - lu) <= 1e-11 * scale
        assert maxabs(Ff[:ns, ns:] - F12) <= 1e-11 * scale
        assert maxabs(Ff[ns:, :ns] - F21) <= 1e-11 * scale
        assert maxabs(Ff[ns:, ns:] - C) <= 1e-11 * scale
        gpu_cb[f] = Ff[ns:, ns:]
    s.close()


@pytest.mark.parametrize("dims,leaf,batched", [((8, 8, 8), 64, False), ((9, 7, 6), 40, True)])
def test_row_interchanges_match_oracle(gpu_lib, dims, leaf, batched):
    """The 7-point pattern with random complex values has no dominant diagonal, so most fronts
    interchange rows (the Helmholtz fronts above never do): pivots equal the oracle's LAPACK partial
    factorization of the same assembled front, the factored blocks match it, and the preconditioner
    applies the interchanges like the oracle's solve."""
    rp, ci, v, _ = helmholtz_7pt(dims, 0.05)
    rng = rng_for("test", "coef", dims)
    v = rng.standard_normal(v.shape[0]) + 1j * rng.standard_normal(v.shape[0])
    s = gpu_lib.Solver(0).analyze(rp, ci, v, dims=dims, leaf_max=leaf, sep_leaf=16)
    s.factor(n_min=0, batched=batched, keep_fronts=True)
    od = nd.nd_grid(dims, leaf_max=leaf, sep_leaf=16)
    sym = symbolic(rp, ci, od)
    gpu_cb, moved = {}, 0
    for f in range(od.nfronts):
        ns = int(od.send[f] - od.sbeg[f])
        Fa, Ff, piv = s.front(f, 0), s.front(f, 1), s.front(f, 2)
        want = mf.assemble_front(rp, ci, v, od, sym, f, gpu_cb)
        assert np.array_equal(Fa, want), f"front {f}: assembly differs"
        lu, opiv, F12, F21, C = mf.partial_lu(want.copy(), ns)
        assert np.array_equal(piv, opiv), f"front {f}: pivots differ"
        moved += int(np.any(np.asarray(opiv) != np.arange(ns)))
        scale = max(1.0, np.abs(want).max())
        assert maxabs(Ff[:ns, :ns] - lu) <= 1e-10 * scale
        assert maxabs(Ff[:ns, ns:] - F12) <= 1e-10 * scale
        assert maxabs(Ff[ns:, :ns] - F21) <= 1e-10 * scale
        assert maxabs(Ff[ns:, ns:] - C) <= 1e-10 * scale
        gpu_cb[f] = Ff[ns:, ns:]
    assert moved >= od.nfronts // 2, (moved, od.nfronts)
    fac = mf.factor(rp, ci, v, od)
    B = rng.standard_normal((od.n, 2)) + 1j * rng.standard_normal((od.n, 2))
    X = s.precondition(B)
    Xo = mf.solve(fac, B)
    assert np.linalg.norm(X - Xo) <= 1e-9 * np.linalg.norm(Xo)
    s.close()


def test_front_taller_than_the_register_panel_with_interchanges(gpu_lib):
    """A 33 x 32 x 33 grid has a 1056-node root separator: its first panel is factored by the
    global-memory panel kernel (more than 1024 rows left), the later ones in registers. With random
    values every front interchanges rows; pivots equal the oracle's and the factored blocks match it,
    and one GMRES iteration with the exact factorization solves the system."""
    dims = (33, 32, 33)
    rp, ci, v, _ = helmholtz_7pt(dims, 0.05)
    rng = rng_for("test", "coef", dims)
    v = rng.standard_normal(v.shape[0]) + 1j * rng.standard_normal(v.shape[0])
    s = gpu_lib.Solver(0).analyze(rp, ci, v, dims=dims, leaf_max=512, sep_leaf=64)
    s.factor(n_min=0, batched=True, keep_fronts=True)
    od = nd.nd_grid(dims, leaf_max=512, sep_leaf=64)
    sym = symbolic(rp, ci, od)
    assert max(int(od.send[f] - od.sbeg[f]) for f in range(od.nfronts)) > 1024
    gpu_cb = {}
    for f in range(od.nfronts):
        ns = int(od.send[f] - od.sbeg[f])
        Fa, Ff, piv = s.front(f, 0), s.front(f, 1), s.front(f, 2)
        want = mf.assemble_front(rp, ci, v, od, sym, f, gpu_cb)
        assert np.array_equal(Fa, want), f"front {f}: assembly differs"
        lu, opiv, F12, F21, C = mf.partial_lu(want.copy(), ns)
        assert np.array_equal(piv, opiv), f"front {f}: pivots differ"
        scale = max(1.0, np.abs(want).max())
        assert maxabs(Ff[:ns, :ns] - lu) <= 1e-9 * scale, f
        assert maxabs(Ff[:ns, ns:] - F12) <= 1e-9 * scale, f
        assert maxabs(Ff[ns:, :ns] - F21) <= 1e-9 * scale, f
        assert maxabs(Ff[ns:, ns:] - C) <= 1e-9 * scale, f
        gpu_cb[f] = Ff[ns:, ns:]
    B = rng.standard_normal((od.n, 2)) + 1j * rng.standard_normal((od.n, 2))
    X, info = s.solve(B)
    assert info["status"] == 0 and info["iters"] <= 1
    assert np.all(mf.rel_residual(rp, ci, v, X, B) <= 1e-10)
    s.close()


@pytest.mark.parametrize("dims,leaf,nrhs,batched", [((8, 8, 8), 64, 1, False), ((10, 9, 8), 64, 3, True),
                                                    ((12, 12, 12), 100, 24, True), ((12, 12, 12), 100, 70, True),
                                                    ((2, 2, 2), 512, 2, False)])
def test_preconditioner_matches_oracle_solve(gpu_lib, dims, leaf, nrhs, batched):
    rp, ci, v, _ = helmholtz_7pt(dims, 0.05)
    od = nd.nd_grid(dims, leaf_max=leaf, sep_leaf=16)
    fac = mf.factor(rp, ci, v, od)
    rng = rng_for("test", "rhs", (nrhs,))
    B = rng.standard_normal((od.n, nrhs)) + 1j * rng.standard_normal((od.n, nrhs))
    s = gpu_lib.Solver(0).analyze(rp, ci, v, dims=dims, leaf_max=leaf, sep_leaf=16)
    s.factor(n_min=0, batched=batched)
    X = s.precondition(B)
    Xo = mf.solve(fac, B)
    assert np.linalg.norm(X - Xo) <= 1e-10 * np.linalg.norm(Xo)
    Xg, info = s.solve(B)
    assert info["status"] == 0 and info["iters"] <= 1
    assert np.all(mf.rel_residual(rp, ci, v, Xg, B) <= 1e-12)
    s.close()


def test_sweep_columns_independent_of_the_batch_width(gpu_lib):
    # 24 right-hand sides take the two-column-block streaming sweep product, 8 the one-block form;
    # both add the products of an entry in the same order, so the shared columns agree
    dims = (12, 12, 12)
    rp, ci, v, _ = helmholtz_7pt(dims, 0.05)
    rng = rng_for("test", "rhs", (24,))
    B = rng.standard_normal((1728, 24)) + 1j * rng.standard_normal((1728, 24))
    s = gpu_lib.Solver(0).analyze(rp, ci, v, dims=dims, leaf_max=100, sep_leaf=16)
    s.factor(n_min=0, batched=True)
    X24 = s.precondition(B)
    X8 = s.precondition(np.asfortranarray(B[:, :8]))
    s.close()
    assert np.linalg.norm(X24[:, :8] - X8) <= 1e-13 * np.linalg.norm(X8)


def test_batched_equals_plain_bitwise(gpu_lib):
    dims = (10, 10, 10)
    rp, ci, v, _ = helmholtz_7pt(dims, 0.05)
    B = rng_for("test", "rhs").standard_normal((1000, 2)) + 0j
    out = []
    for batched in (False, True):
        s = gpu_lib.Solver(0).analyze(rp, ci, v, dims=dims, leaf_max=64, sep_leaf=16)
        s.factor(n_min=0, batched=batched)
        out.append(s.precondition(B))
        s.close()
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("n_min", [0, 60])
def test_level_workspace_reuse(gpu_lib, n_min):
    """Fronts share two level workspaces (alternating with the level's parity) unless
    keep_fronts gives each its own slot: the factors and the preconditioner are the same
    bit for bit, dense and with nested compressed fronts."""
    dims = (16, 16, 16)
    rp, ci, v, _ = helmholtz_7pt(dims, 0.05)
    B = rng_for("test", "rhs").standard_normal((4096, 3)) + 0j
    out, fronts = [], []
    for keep in (True, False):
        s = gpu_lib.Solver(0).analyze(rp, ci, v, dims=dims, leaf_max=64, sep_leaf=32)
        s.factor(tol=1e-3, n_min=n_min, batched=True, keep_fronts=keep)
        out.append(s.precondition(B))
        sym = s.symbolic()
        ns = sym["send"] - sym["sbeg"]
        leaf = np.diff(sym["child_ptr"]) == 0
        dense = [f for f in range(len(ns)) if n_min == 0 or leaf[f] or ns[f] < n_min]
        fr = []
        for f in dense[:: max(1, len(dense) // 12)]:
            F = s.front(f, 1)
            k = int(ns[f])
            fr.append((F[:, :k].copy(), F[:k, k:].copy()))
        fronts.append(fr)
        s.close()
    assert np.array_equal(out[0], out[1])
    for (a0, b0), (a1, b1) in zip(*fronts):
        assert np.array_equal(a0, a1) and np.array_equal(b0, b1)


def test_helmholtz24_end_to_end(gpu_lib):
    p = make_problem("helmholtz24")
    od = nd.nd_grid(p.dims, leaf_max=512, sep_leaf=64)
    fac = mf.factor(p.rowptr, p.colind, p.values, od)
    Xo = mf.solve_refined(p.rowptr, p.colind, p.values, fac, p.rhs, steps=1)
    s = gpu_lib.Solver(0).analyze(p.rowptr, p.colind, p.values, dims=p.dims)
    s.factor(n_min=0, batched=True)
    X, info = s.solve(p.rhs, true_rtol=1e-3)
    assert info["status"] == 0
    assert np.linalg.norm(X - Xo) <= 1e-10 * np.linalg.norm(Xo)
    assert info["relres"] <= 1e-12
    st = s.stats()
    assert st["nfronts"] == 63 and st["factor_seconds"] > 0
    s.close()


def test_singular_matrix_reports_front(gpu_lib):
    dims = (4, 4, 4)
    rp, ci, v, _ = helmholtz_7pt(dims, 0.05)
    z = np.zeros_like(v)
    s = gpu_lib.Solver(0).analyze(rp, ci, z, dims=dims, leaf_max=8)
    with pytest.raises(gpu_lib.BfmfError) as e:
        s.factor(n_min=0)
    assert e.value.status == gpu_lib.BFMF_E_SINGULAR
    assert s.stats()["singular_front"] >= 0
    # solve is refused after a failed factorization
    with pytest.raises(gpu_lib.BfmfError) as e:
        s.solve(np.ones(64))
    assert e.value.status == gpu_lib.BFMF_E_STATE
    # new values bring the handle back
    gpu_lib.bfmf_set_values(s.h, v)
    s.factor(n_min=0)
    X, info = s.solve(np.ones(64))
    assert info["status"] == 0
    s.close()
