"""Pins of the oracle's generators, multifrontal factorization, solve and GMRES.

* Generators: sine modes are exact eigenvectors of the constant-coefficient
  7-point stencil; discrete gradients are in the kernel of the Yee curl-curl.
* Multifrontal LU (Alg. 1): brute-force dense solves on grids of at most 8^3,
  manufactured solutions, and the identity C_tau = -A(U,T) A(T,T)^-1 A(T,U)
  for the contribution block of the subtree T of tau with update set U.
* Partial LU: P L U reproduces F11 (LAPACK getrf on the same block); on the
  7-point pattern with random values (rows interchanged in most fronts) factor
  and solve still give the dense solution.
* GMRES: an exact preconditioner converges in one iteration; the residual
  estimate never increases inside a cycle; the unpreconditioned solve reaches
  the dense solution; each history entry is the least-squares minimum of
  ||M^-1 (b - A x)|| over the Krylov space (brute force); k distinct
  eigenvalues give convergence at exactly step k.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from workloads import helmholtz_7pt, make_problem, rng_for
from workloads.maxwell import yee_curlcurl, block_permittivity
from oracle import nd, gmres
from oracle.symbolic import symbolic
from oracle import multifrontal as mf


def dense(rowptr, colind, values):
    return mf.csr_matrix(rowptr, colind, values).toarray()


@pytest.mark.parametrize("q", [(1, 1, 1), (2, 3, 1), (5, 4, 6)])
def test_sine_modes_are_eigenvectors(q):
    dims = (7, 6, 8)
    delta = 0.05
    rowptr, colind, values, meta = helmholtz_7pt(dims, delta)
    h, w = meta["h"], meta["omega"]
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    # interior node i sits at (i+1) h on an axis with n_axis interior nodes; the
    # Dirichlet sine mode on that axis uses the axis' own spacing 1/(n_axis+1)
    v = (np.sin(np.pi * q[0] * (x + 1) / (nx + 1)) * np.sin(np.pi * q[1] * (y + 1) / (ny + 1))
         * np.sin(np.pi * q[2] * (z + 1) / (nz + 1))).ravel()
    lam = sum(2 - 2 * np.cos(np.pi * qq / (nn + 1)) for qq, nn in zip(q, dims)) - (w * h) ** 2 * (1 + 1j * delta)
    A = mf.csr_matrix(rowptr, colind, values)
    assert np.linalg.norm(A @ v - lam * v) <= 1e-13 * np.linalg.norm(v) * abs(lam + 6)
    # 8 points per wavelength at c = 1: (omega h)^2 = (pi / 4)^2
    assert abs((w * h) ** 2 - (np.pi / 4) ** 2) < 1e-14


def test_yee_gradients_in_kernel_of_curlcurl():
    n = 5
    delta = 0.03
    eps = block_permittivity(n, 2, rng_for("test", "coef"))
    rowptr, colind, values, meta = yee_curlcurl(n, delta, eps_cells=eps)
    coords = meta["coords"]
    A = mf.csr_matrix(rowptr, colind, values)
    # node potential, zero on the boundary (PEC), gradient on interior edges
    rng = np.random.default_rng(0)
    phi = np.zeros((n + 1, n + 1, n + 1))
    phi[1:n, 1:n, 1:n] = rng.standard_normal((n - 1, n - 1, n - 1))
    g = np.empty(coords.shape[0])
    for e, (x, y, zz) in enumerate(coords):
        d = [x % 2, y % 2, zz % 2].index(1)
        lo = [x // 2, y // 2, zz // 2]
        hi = list(lo); hi[d] += 1
        g[e] = phi[hi[0], hi[1], hi[2]] - phi[lo[0], lo[1], lo[2]]
    mass = (meta["omega"] * meta["h"]) ** 2 * (1 + 1j * delta) * meta["eps_edge"]
    assert np.linalg.norm(A @ g + mass * g) <= 1e-12 * np.linalg.norm(g)
    # 13 couplings per deep-interior edge
    assert np.max(np.diff(rowptr)) == 13


@pytest.mark.parametrize("dims,leaf", [((4, 4, 4), 8), ((6, 6, 6), 27), ((8, 8, 8), 64), ((8, 7, 5), 30)])
def test_multifrontal_matches_dense_solve(dims, leaf):
    rowptr, colind, values, _ = helmholtz_7pt(dims, 0.05)
    od = nd.nd_grid(dims, leaf_max=leaf, sep_leaf=8)
    fac = mf.factor(rowptr, colind, values, od)
    rng = rng_for("test", "manufactured", dims)
    xs = rng.standard_normal((od.n, 3)) + 1j * rng.standard_normal((od.n, 3))
    Ad = dense(rowptr, colind, values)
    B = Ad @ xs
    X = mf.solve(fac, B)
    Xd = np.linalg.solve(Ad, B)
    assert np.linalg.norm(X - Xd) <= 1e-10 * np.linalg.norm(Xd)
    assert np.linalg.norm(X - xs) <= 1e-10 * np.linalg.norm(xs)
    assert np.all(mf.rel_residual(rowptr, colind, values, X, B) <= 1e-12)


@pytest.mark.parametrize("dims,leaf", [((4, 4, 4), 8), ((6, 5, 4), 30)])
def test_multifrontal_with_row_interchanges_matches_dense_solve(dims, leaf):
    """The 7-point pattern with random complex values has no dominant diagonal, so the partial LU of the
    fronts interchanges rows (pivoting restricted to F11, Alg. 1); factor and solve must still give the
    dense solution, which fails if an interchange is dropped or applied on the wrong side."""
    rowptr, colind, values, _ = helmholtz_7pt(dims, 0.05)
    rng = rng_for("test", "coef", dims)
    values = rng.standard_normal(values.shape[0]) + 1j * rng.standard_normal(values.shape[0])
    od = nd.nd_grid(dims, leaf_max=leaf, sep_leaf=8)
    fac = mf.factor(rowptr, colind, values, od)
    moved = sum(int(np.any(np.asarray(p) != np.arange(len(p)))) for p in fac.piv)
    assert moved >= od.nfronts // 2, (moved, od.nfronts)
    xs = rng.standard_normal((od.n, 2)) + 1j * rng.standard_normal((od.n, 2))
    Ad = dense(rowptr, colind, values)
    B = Ad @ xs
    X = mf.solve(fac, B)
    Xd = np.linalg.solve(Ad, B)
    assert np.linalg.norm(X - Xd) <= 1e-8 * np.linalg.norm(Xd)
    assert np.all(mf.rel_residual(rowptr, colind, values, X, B) <= 1e-10)


def test_contribution_blocks_are_subtree_schur_complements():
    dims = (6, 6, 6)
    rowptr, colind, values, _ = helmholtz_7pt(dims, 0.05)
    od = nd.nd_grid(dims, leaf_max=27, sep_leaf=8)
    sym = symbolic(rowptr, colind, od)
    fac = mf.factor(rowptr, colind, values, od, sym, keep_fronts=True)
    Ad = dense(rowptr, colind, values)
    Anew = Ad[np.ix_(od.perm, od.perm)]
    first = np.array(od.sbeg)
    for f in range(od.nfronts):
        for c in od.children[f]:
            first[f] = min(first[f], first[c])
    for f in range(od.nfronts - 1):
        T = np.arange(first[f], od.send[f])
        U = sym.Iu[f]
        S = -Anew[np.ix_(U, T)] @ np.linalg.solve(Anew[np.ix_(T, T)], Anew[np.ix_(T, U)])
        assert np.linalg.norm(fac.cbs[f] - S) <= 1e-11 * max(1.0, np.linalg.norm(S)), f


def test_assembled_front_entries():
    """F_tau holds A entries (not A(Iu,Iu)) plus the children blocks at the mapped positions."""
    dims = (5, 5, 5)
    rowptr, colind, values, _ = helmholtz_7pt(dims, 0.05)
    od = nd.nd_grid(dims, leaf_max=16, sep_leaf=8)
    sym = symbolic(rowptr, colind, od)
    fac = mf.factor(rowptr, colind, values, od, sym, keep_fronts=True)
    Anew = dense(rowptr, colind, values)[np.ix_(od.perm, od.perm)]
    for f in range(od.nfronts):
        idx = np.concatenate([np.arange(od.sbeg[f], od.send[f]), sym.Iu[f]])
        ns = od.send[f] - od.sbeg[f]
        want = Anew[np.ix_(idx, idx)].copy()
        want[ns:, ns:] = 0
        for c in od.children[f]:
            m = sym.maps[c]
            want[np.ix_(m, m)] += fac.cbs[c]
        assert np.array_equal(fac.fronts[f], want)


def test_partial_lu_reproduces_f11():
    rng = np.random.default_rng(3)
    ns, nu = 40, 25
    F = rng.standard_normal((ns + nu, ns + nu)) + 1j * rng.standard_normal((ns + nu, ns + nu))
    lu, piv, F12, F21, C = mf.partial_lu(F.copy(), ns)
    L = np.tril(lu, -1) + np.eye(ns)
    U = np.triu(lu)
    P = np.eye(ns)[mf.swaps_to_perm(piv)]
    assert np.linalg.norm(P @ F[:ns, :ns] - L @ U) <= 1e-13 * np.linalg.norm(F)
    # pivot choice: first row maximising |Re| + |Im| of the first column
    col = F[:ns, 0]
    assert piv[0] == np.argmax(np.abs(col.real) + np.abs(col.imag))
    # full-front identity: [L 0; F21' I] [U F12'; 0 C] = [P F11 P F12; F21 F22]
    top = np.hstack([P @ F[:ns, :ns], P @ F[:ns, ns:]])
    bot = F[ns:, :]
    Lf = np.block([[L, np.zeros((ns, nu))], [F21, np.eye(nu)]])
    Uf = np.block([[U, F12], [np.zeros((nu, ns)), C]])
    assert np.linalg.norm(Lf @ Uf - np.vstack([top, bot])) <= 1e-12 * np.linalg.norm(F)


def test_refinement_and_24_cubed_workload():
    p = make_problem("helmholtz24")
    od = nd.nd_grid(p.dims, leaf_max=512, sep_leaf=64)
    fac = mf.factor(p.rowptr, p.colind, p.values, od)
    X = mf.solve_refined(p.rowptr, p.colind, p.values, fac, p.rhs, steps=1)
    assert mf.rel_residual(p.rowptr, p.colind, p.values, X, p.rhs)[0] <= 1e-13


def test_gmres_exact_preconditioner_one_iteration():
    dims = (6, 6, 6)
    rowptr, colind, values, _ = helmholtz_7pt(dims, 0.05)
    od = nd.nd_grid(dims, leaf_max=27)
    fac = mf.factor(rowptr, colind, values, od)
    A = mf.csr_matrix(rowptr, colind, values)
    b = np.random.default_rng(1).standard_normal(od.n) + 0j
    x, it, hist = gmres.gmres(lambda v: A @ v, lambda v: mf.solve(fac, v), b)
    assert it == 1
    assert np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b)


def test_gmres_unpreconditioned_properties():
    # diagonally dominant complex system: GMRES(30) converges to the dense solution
    rng = np.random.default_rng(2)
    n = 60
    Ad = np.eye(n) * 4 + 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, it, hist = gmres.gmres(lambda v: Ad @ v, lambda v: v, b, restart=30, rtol=1e-12, atol=0)
    assert np.linalg.norm(x - np.linalg.solve(Ad, b)) <= 1e-10 * np.linalg.norm(x)
    # within the first cycle the residual estimate is non-increasing and matches the true residual
    first = hist[: min(len(hist), 31)]
    assert np.all(np.diff(first) <= 1e-12 * first[0])
    # restarted run with a small restart length still converges
    x5, it5, _ = gmres.gmres(lambda v: Ad @ v, lambda v: v, b, restart=5, rtol=1e-10, atol=0, max_iter=500)
    assert np.linalg.norm(Ad @ x5 - b) <= 1e-9 * np.linalg.norm(b)


def _krylov_min_residual(Mi_A, Mi_b, j):
    """min over x in K_j(Mi_A, Mi_b) of ||Mi_b - Mi_A x||, by brute force: an orthonormal basis of the
    Krylov space from a QR of the power basis, then least squares."""
    K = np.empty((Mi_b.shape[0], j), dtype=np.complex128)
    v = Mi_b.copy()
    for c in range(j):
        K[:, c] = v / np.linalg.norm(v)
        v = Mi_A @ K[:, c]
    Q, _ = np.linalg.qr(K)
    y = np.linalg.lstsq(Mi_A @ Q, Mi_b, rcond=None)[0]
    return np.linalg.norm(Mi_b - Mi_A @ Q @ y)


@pytest.mark.parametrize("precond", [False, True])
def test_gmres_history_is_the_krylov_minimum_residual(precond):
    """GMRES (Sec. 6: left preconditioning, zero initial guess) minimises ||M^-1 (b - A x)|| over the
    Krylov space K_j(M^-1 A, M^-1 b): every entry of the first cycle's history equals that minimum,
    computed here by least squares over an explicit basis. Complex, non-normal A and M."""
    rng = np.random.default_rng(5)
    n = 40
    A = np.eye(n) * (2 + 1j) + 0.6 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    M = np.eye(n) + (0.2 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
                     if precond else 0)
    Mi = np.linalg.inv(M)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, it, hist = gmres.gmres(lambda v: A @ v, lambda v: Mi @ v, b, restart=30, rtol=1e-13, atol=0, max_iter=12)
    assert it == 12 and len(hist) == 13
    assert abs(hist[0] - np.linalg.norm(Mi @ b)) <= 1e-13 * hist[0]
    for j in range(1, 13):
        ref = _krylov_min_residual(Mi @ A, Mi @ b, j)
        assert abs(hist[j] - ref) <= 1e-10 * hist[0], (j, hist[j], ref)
    # the returned iterate attains the last value of the history
    assert abs(np.linalg.norm(Mi @ (b - A @ x)) - hist[-1]) <= 1e-10 * hist[0]


@pytest.mark.parametrize("k", [1, 3, 7])
def test_gmres_converges_in_as_many_steps_as_distinct_eigenvalues(k):
    """A diagonalisable A with k distinct eigenvalues has a minimal polynomial of degree k, so GMRES
    reaches the exact solution at step k and, for a generic b, not before."""
    rng = np.random.default_rng(10 + k)
    n = 24
    lam = rng.standard_normal(k) + 1j * rng.standard_normal(k) + 3
    S = np.eye(n) + 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    A = S @ np.diag(lam[np.arange(n) % k]) @ np.linalg.inv(S)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, it, hist = gmres.gmres(lambda v: A @ v, lambda v: v, b, restart=30, rtol=1e-10, atol=0)
    assert it == k
    assert np.linalg.norm(A @ x - b) <= 1e-9 * np.linalg.norm(b)
    if k > 1:
        assert hist[k - 1] > 1e-4 * hist[0]
