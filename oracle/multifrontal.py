"""Uncompressed multifrontal LU and solve in FP64 complex (oracle).

Follows the paper's Alg. 1 (Sec. 2) front by front, in postorder:
  assemble  F = [A(Is,Is) A(Is,Iu); A(Iu,Is) 0]  (+) C_nu1 (+) C_nu2
  P L U = F11  (partial pivoting restricted to the rows of F11; the pivot is
               the first row maximising |Re| + |Im|, LAPACK getrf convention)
  F12 <- L^-1 P^T F12,  F21 <- F21 U^-1,  C = F22 - F21 F12
and the solve x = P^T bwd(fwd(P b)) (forward: leaves to root, backward:
root to leaves), plus one step of iterative refinement as used for the
exact solver in the paper's experiments (Sec. 6).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .symbolic import symbolic


class Factors:
    pass


def _front_positions(od, sym, f):
    b, e = int(od.sbeg[f]), int(od.send[f])
    return b, e, sym.Iu[f]


def assemble_front(rowptr, colind, values, od, sym, f, cbs):
    """Dense front F_tau: A entries first, then children in child order.

    ``cbs`` maps child front id -> contribution block C (complex128).
    Entry order per position: ((0 + a) + c1) + c2.
    """
    b, e, Iu = _front_positions(od, sym, f)
    ns = e - b
    n = ns + Iu.shape[0]
    F = np.zeros((n, n), dtype=np.complex128)
    # front-local position of every global (new) index touched by this front
    local = {j: j - b for j in range(b, e)}
    local.update({int(j): ns + k for k, j in enumerate(Iu)})

    def entries(rows_new):
        """(new row, new col, value) of the CSR rows of the given new indices."""
        old = od.perm[rows_new]
        cnt = rowptr[old + 1] - rowptr[old]
        r = np.repeat(rows_new, cnt)
        t = np.concatenate([np.arange(rowptr[o], rowptr[o + 1]) for o in old]) if old.size else np.zeros(0, np.int64)
        return r, od.iperm[colind[t]], values[t]

    # A entries owned by this front: min(i, j) in I^s.  Rows in I^s: columns
    # in I^s u I^u (columns below b were assembled in a descendant front).
    r, c, v = entries(np.arange(b, e))
    keep = c >= b
    for i, j, a in zip(r[keep], c[keep], v[keep]):
        F[local[int(i)], local[int(j)]] = a
    # rows in I^u, columns in I^s
    r, c, v = entries(Iu)
    keep = (c >= b) & (c < e)
    for i, j, a in zip(r[keep], c[keep], v[keep]):
        F[local[int(i)], local[int(j)]] = a
    for c in od.children[f]:
        m = sym.maps[c]
        F[np.ix_(m, m)] += cbs[c]
    return F


def swaps_to_perm(piv):
    """Row order produced by applying the interchanges k <-> piv[k], k = 0, 1, ..."""
    order = np.arange(len(piv))
    for k, p in enumerate(piv):
        order[k], order[p] = order[p], order[k]
    return order


def partial_lu(F, ns):
    """Partial factorization of a dense front with pivots restricted to F11.

    Returns (lu, piv, F12', F21', C) where lu holds L (unit lower) and U.
    """
    F11 = F[:ns, :ns]
    F12 = F[:ns, ns:].copy()
    F21 = F[ns:, :ns]
    F22 = F[ns:, ns:]
    if ns > 0:
        lu, piv = sla.lu_factor(F11, check_finite=True)
        if np.any(np.diag(lu) == 0):
            raise ZeroDivisionError("exact zero pivot")
        F12 = F12[swaps_to_perm(piv), :]
        F12 = sla.solve_triangular(lu, F12, lower=True, unit_diagonal=True)
        F21 = sla.solve_triangular(lu, F21.T, trans="T", lower=False).T if F21.shape[0] else F21.copy()
        # X U = F21  <=>  U^T X^T = F21^T
        C = F22 - F21 @ F12
    else:
        lu, piv, C = F11.copy(), np.zeros(0, np.int32), F22.copy()
    return lu, piv, F12, F21, C


def factor(rowptr, colind, values, od, sym=None, keep_fronts=False):
    """Multifrontal factorization following Alg. 1."""
    if sym is None:
        sym = symbolic(rowptr, colind, od)
    fac = Factors()
    fac.od, fac.sym = od, sym
    fac.lu, fac.piv, fac.F12, fac.F21 = [], [], [], []
    fac.fronts = [] if keep_fronts else None
    fac.cbs = {} if keep_fronts else None
    cbs = {}
    for f in range(od.nfronts):
        F = assemble_front(rowptr, colind, values, od, sym, f, cbs)
        for c in od.children[f]:
            if not keep_fronts:
                del cbs[c]
        if keep_fronts:
            fac.fronts.append(F.copy())
        ns = int(od.send[f] - od.sbeg[f])
        lu, piv, F12, F21, C = partial_lu(F, ns)
        fac.lu.append(lu); fac.piv.append(piv); fac.F12.append(F12); fac.F21.append(F21)
        cbs[f] = C
        if keep_fronts:
            fac.cbs[f] = C
    return fac


def solve(fac, B):
    """x = P^T bwd(fwd(P b)) for a block of right-hand sides B (N x nrhs)."""
    od, sym = fac.od, fac.sym
    B = np.asarray(B, dtype=np.complex128)
    vec = B.ndim == 1
    if vec:
        B = B[:, None]
    y = B[od.perm, :].copy()
    for f in range(od.nfronts):  # forward, leaves to root
        b, e = int(od.sbeg[f]), int(od.send[f])
        z = y[b:e, :][swaps_to_perm(fac.piv[f]), :]
        if e > b:
            z = sla.solve_triangular(fac.lu[f], z, lower=True, unit_diagonal=True)
        y[b:e, :] = z
        Iu = sym.Iu[f]
        if Iu.shape[0]:
            y[Iu, :] -= fac.F21[f] @ z
    x = np.zeros_like(y)
    for f in range(od.nfronts - 1, -1, -1):  # backward, root to leaves
        b, e = int(od.sbeg[f]), int(od.send[f])
        rhs = y[b:e, :].copy()
        Iu = sym.Iu[f]
        if Iu.shape[0]:
            rhs -= fac.F12[f] @ x[Iu, :]
        if e > b:
            x[b:e, :] = sla.solve_triangular(fac.lu[f], rhs, lower=False)
    out = np.empty_like(x)
    out[od.perm, :] = x
    return out[:, 0] if vec else out


def csr_matrix(rowptr, colind, values):
    n = rowptr.shape[0] - 1
    return sp.csr_matrix((values, colind, rowptr), shape=(n, n))


def solve_refined(rowptr, colind, values, fac, B, steps=1):
    """Solve followed by ``steps`` rounds of iterative refinement."""
    A = csr_matrix(rowptr, colind, values)
    X = solve(fac, B)
    for _ in range(steps):
        R = B - A @ X
        X = X + solve(fac, R)
    return X


def rel_residual(rowptr, colind, values, X, B):
    """Per-column ||B - A X||_2 / ||B||_2."""
    A = csr_matrix(rowptr, colind, values)
    B = np.asarray(B)
    X = np.asarray(X)
    if B.ndim == 1:
        B = B[:, None]; X = X[:, None]
    R = B - A @ X
    return np.linalg.norm(R, axis=0) / np.linalg.norm(B, axis=0)
