"""The 27-point visco-acoustic operator with absorbing layers (the stand-in for
the paper's main workload, Sec. 6 visco-acoustic experiments) and the method
on it, on the CPU.

Pins of the generator against what the mathematics fixes: the stencil's
Laplacian part is exact for quadratics and bilinears and annihilates
constants (a wrong weight, sign or offset breaks one of these), the mass
weights sum to one, rows outside the absorbing layers are real-coefficient
rows of the unstretched operator, and the pattern is 27 points in the
interior.  Then the oracle's multifrontal LU (Alg. 1) against a sparse direct
solve of the same matrix, and the C++ analysis against the oracle's ordering
and symbolic factorization (a single grid plane still separates a 27-point
stencil).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from workloads import acoustic_27pt, make_problem, rng_for
from workloads.acoustic import pml_profile
from oracle import nd
from oracle import multifrontal as mf
from oracle.symbolic import symbolic


def _mat(rp, ci, v):
    return sp.csr_matrix((v, ci, rp), shape=(rp.shape[0] - 1, rp.shape[0] - 1))


def _grid(n):
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    inner = ((x > 0) & (x < n - 1) & (y > 0) & (y < n - 1) & (z > 0) & (z < n - 1)).ravel()
    return x, y, z, inner


def test_laplacian_part_exact_for_quadratics():
    """omega = 0, no layers: h^2 times minus the discrete Laplacian, row by row
    in the interior, equals minus the exact Laplacian of every polynomial of
    degree <= 2 (grid units)."""
    n = 9
    A = _mat(*acoustic_27pt((n, n, n), pml=0, omega=0.0)[:3])
    x, y, z, inner = _grid(n)
    cases = [(np.ones_like(x), 0.0), (x, 0.0), (x * x, -2.0), (y * y + 3 * z * z, -8.0),
             (x * y, 0.0), (y * z - x * z, 0.0), (x * x - y * y, 0.0)]
    for p, want in cases:
        r = A @ p.ravel().astype(np.complex128)
        assert np.abs(r[inner] - want).max() < 1e-11


def test_mass_term_and_bulk_modulus():
    """No layers: A 1 = -(omega h / kappa)^2 in the interior, kappa = v (1 - i/(2q))."""
    n = 8
    for q in (1e4, 20.0):
        rp, ci, v, meta = acoustic_27pt((n, n, n), q=q, pml=0)
        x, y, z, inner = _grid(n)
        r = _mat(rp, ci, v) @ np.ones(n ** 3, dtype=np.complex128)
        want = -(meta["omega"] * meta["h"] / (1.0 - 0.5j / q)) ** 2
        assert np.abs(r[inner] - want).max() < 1e-12


def test_pattern_and_absorbing_layers():
    n, pml = 14, 4
    rp, ci, v, meta = acoustic_27pt((n, n, n), pml=pml)
    nnz = np.diff(rp)
    x, y, z, inner = _grid(n)
    assert np.all(nnz[inner] == 27) and nnz.min() == 8  # corners of the box keep 8
    A = _mat(rp, ci, v)
    assert (A != 0).nnz == A.nnz and abs(A - A.T).nnz > 0  # no explicit zeros; non-symmetric values
    P = (A != 0).astype(np.int8)
    assert (P != P.T).nnz == 0  # symmetric pattern
    # stretching factors: 1 outside the layer, quadratic growth to 1 + i g at the outer face
    xi = pml_profile(n, pml, 2.0)
    assert np.all(xi[pml:n - pml] == 1.0) and xi[0] == 1.0 + 2.0j and xi[-1] == 1.0 + 2.0j
    assert np.isclose(xi[pml // 2], 1.0 + 2.0j * (1 - (pml // 2) / pml) ** 2)
    # rows of nodes outside every layer equal the rows of the operator without layers
    A0 = _mat(*acoustic_27pt((n, n, n), pml=0, omega=meta["omega"])[:3])
    core = ((x >= pml) & (x < n - pml) & (y >= pml) & (y < n - pml) & (z >= pml) & (z < n - pml)).ravel()
    D = (A - A0).tocsr()
    assert abs(D[np.flatnonzero(core)]).max() == 0.0
    # inside the layers the Laplacian couplings are complex
    layer_row = np.flatnonzero(~core)[0]
    assert np.abs(A[layer_row].toarray().imag).max() > 0.1


@pytest.mark.parametrize("dims,pml", [((10, 10, 10), 3), ((9, 11, 10), 2)])
def test_oracle_multifrontal_solves_acoustic(dims, pml):
    """Alg. 1 on the 27-point operator: the oracle's exact multifrontal solve
    equals a sparse direct solve (SuperLU) to rounding."""
    rng = rng_for("test", "coef", dims)
    c = 1.0 + rng.random(dims[::-1])
    rp, ci, v, _ = acoustic_27pt(dims, c=c, pml=pml)
    n = rp.shape[0] - 1
    B = rng_for("test", "rhs", dims).standard_normal((n, 2)) + 0j
    od = nd.nd_grid(dims, leaf_max=64, sep_leaf=32)
    X = mf.solve(mf.factor(rp, ci, v, od), B)
    Xs = spla.spsolve(_mat(rp, ci, v).tocsc(), B)
    assert np.linalg.norm(X - Xs) <= 1e-10 * np.linalg.norm(Xs)


def test_named_config_builds():
    p = make_problem("acoustic64", n=20, nrhs=3)
    assert p.n == 8000 and p.rhs.shape == (8000, 3) and p.kind == "grid"
    assert p.opts["op"] == "acoustic27" and p.meta["pml"] == 8


bfmf = pytest.importorskip("paper_2007_00202_amd.bfmf")


@pytest.mark.parametrize("n,sl", [(18, 32), (64, 128)])
def test_cpp_analysis_matches_oracle_on_acoustic(n, sl):
    """Ordering, tree, I^u and extend-add maps of the C++ analysis equal the
    oracle's on the 27-point pattern (the full 64^3 workload included)."""
    p = make_problem("acoustic64", n=n, nrhs=1)
    h = bfmf.bfmf_create(-1)
    try:
        bfmf.bfmf_analyze(h, p.rowptr, p.colind, p.values, dims=p.dims, sep_leaf=sl)
        od = nd.nd_grid(p.dims, leaf_max=512, sep_leaf=sl)
        sym = symbolic(p.rowptr, p.colind, od)
        s = bfmf.bfmf_get_symbolic(h)
        assert np.array_equal(s["perm"], od.perm)
        assert np.array_equal(s["parent"], od.parent)
        iu_ptr = s["iu_ptr"]
        assert np.array_equal(np.diff(iu_ptr), [len(sym.Iu[f]) for f in range(od.nfronts)])
        want_iu = np.concatenate([np.asarray(sym.Iu[f], np.int64) for f in range(od.nfronts)])
        want_map = np.concatenate([np.asarray(sym.maps[f], np.int64) for f in range(od.nfronts)])
        assert np.array_equal(s["iu"][:iu_ptr[-1]], want_iu)
        assert np.array_equal(s["map"][:iu_ptr[-1]], want_map)
    finally:
        bfmf.bfmf_destroy(h)
