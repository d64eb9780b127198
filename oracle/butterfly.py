"""Interpolative decomposition and butterfly algorithms (oracle, FP64 complex).

Paper Sec. 3.
  id_row          row ID by truncated column-pivoted QR of A^T: A ~= U A(J,:),
                  rank = #{k : |R_kk| > tol |R_00|}  (Sec. 3, ID paragraph)
  Trees           complete binary trees over contiguous index ranges; level l
                  has 2^l nodes (the partitioning trees T_O and T_S of Sec. 3.1)
  Butterfly       K ~= (U^L R^{L-1} .. R^{lc}) B^{lc} (W^{lc} .. W^1 V^0), lc = floor(L/2)
                  (Eq. of the hybrid butterfly, Sec. 3.1)
  bf_entry_eval   construction from entry extraction with proxy columns/rows
                  (Alg. 2): outer-to-inner from both sides, B extracted last
  bf_random_matvec construction from products with K and K^H (Sec. 3.3; the
                  algorithm is only cited by the paper -- reading: sketches with
                  random vectors supported on one column (row) node stand in for
                  the proxy columns (rows) of Alg. 2; the centre blocks come from
                  a least-squares fit of the sketch at the centre level)
  extract_bf      entries of submatrices from the factors (Alg. 3)
  bf_dense        the matrix the factors represent (the product written out)

bf_random_matvec follows a reading of an algorithm the paper only cites; it is
pinned by exactness on generic exact-rank matrices (every ID keeps exactly
min(r, rows, columns) of its block, the product equals K to rounding, L = 0..3
on ragged sizes) and by tolerance on oscillatory kernels.
"""
import numpy as np
import scipy.linalg as sla


# ------------------------------------------------------------------ ID
def id_row(M, tol, maxrank=None):
    """Row ID: M ~= U M[J, :], U[J, :] = I.  Returns (J, U)."""
    p, q = M.shape
    if p == 0 or q == 0:
        return np.zeros(0, dtype=np.int64), np.zeros((p, 0), dtype=M.dtype)
    Q, R, P = sla.qr(M.T, mode="economic", pivoting=True)
    d = np.abs(np.diag(R))
    if d.size == 0 or d[0] == 0:
        return np.zeros(0, dtype=np.int64), np.zeros((p, 0), dtype=M.dtype)
    k = int(np.sum(d > tol * d[0]))
    if maxrank is not None:
        k = min(k, maxrank)
    J = P[:k]
    T = sla.solve_triangular(R[:k, :k], R[:k, k:])  # R11^-1 R12
    U = np.zeros((p, k), dtype=np.result_type(M.dtype, np.complex128))
    U[P[:k], :] = np.eye(k)
    U[P[k:], :] = T.T
    return J.astype(np.int64), U


def id_col(M, tol, maxrank=None):
    """Column ID: M ~= M[:, J] V^T.  Returns (J, Vt) with Vt = V^T (k x q)."""
    J, U = id_row(M.T, tol, maxrank)
    return J, U.T


# ------------------------------------------------------------------ trees
class Tree:
    """Complete binary tree of depth L over [0, n): bounds[l] has 2^l + 1 entries.

    Built from a bisection of [0, n) given as preorder nodes (beg, end, left,
    right); a node without children is split in halves (first half ceil) when
    the tree must be deeper, which may create empty nodes.
    """

    def __init__(self, n, L, nodes=None):
        self.n, self.L = n, L
        self.bounds = []
        cur = [(0, n, 0 if nodes else -1)]
        for l in range(L + 1):
            self.bounds.append(np.array([c[0] for c in cur] + [cur[-1][1]], dtype=np.int64))
            if l == L:
                break
            nxt = []
            for b, e, idx in cur:
                if nodes is not None and idx >= 0 and nodes[idx][2] >= 0:
                    li, ri = nodes[idx][2], nodes[idx][3]
                    mid = nodes[li][1]
                    nxt += [(b, mid, li), (mid, e, ri)]
                else:
                    mid = b + (e - b + 1) // 2
                    nxt += [(b, mid, -1), (mid, e, -1)]
            cur = nxt

    def node(self, l, i):
        return int(self.bounds[l][i]), int(self.bounds[l][i + 1])


def tree_depth(nodes):
    """Depth of a preorder node list (a single node has depth 0)."""
    def d(i):
        if nodes[i][2] < 0:
            return 0
        return 1 + max(d(nodes[i][2]), d(nodes[i][3]))
    return d(0) if nodes else 0


def balanced_depth(n, leaf):
    L = 0
    while (n + (1 << L) - 1) >> L > leaf:
        L += 1
    return L


# ------------------------------------------------------------------ format
class Butterfly:
    """Factors of an L-level butterfly over row tree to and column tree ts.

    U[t]        |O_t| x r        (t at level L, nu = root)
    R[l][t][v]  (r_t1 + r_t2) x r (t at level l in [lc, L), v at level L - l)
    B[t][v]     r x r'           (level lc)
    W[l][t][v]  r' x (r'_v1 + r'_v2) (t at level l in [1, lc], v at level L - l)
    Vt[v]       r' x |S_v|       (t = root, v at level L)
    """

    def __init__(self, to, ts):
        assert to.L == ts.L
        self.to, self.ts = to, ts
        self.L = to.L
        self.lc = self.L // 2
        self.m, self.n = to.n, ts.n
        self.U, self.R, self.B, self.W, self.Vt = {}, {}, {}, {}, {}

    def ranks(self):
        r = [u.shape[1] for u in self.U.values()] + [b.shape[0] for b in self.B.values()]
        r += [b.shape[1] for b in self.B.values()]
        return max(r) if r else 0


def bf_dense(bf):
    """The matrix the factors represent, K = E^{lc} B F^{lc} block by block."""
    K = np.zeros((bf.m, bf.n), dtype=np.complex128)
    L, lc = bf.L, bf.lc
    for t in range(2 ** lc):
        for v in range(2 ** (L - lc)):
            E = _row_basis(bf, lc, t, v)
            F = _col_basis(bf, lc, t, v)
            r0, r1 = bf.to.node(lc, t)
            c0, c1 = bf.ts.node(L - lc, v)
            K[r0:r1, c0:c1] = E @ bf.B[(t, v)] @ F
    return K


def _row_basis(bf, l, t, v):
    """Expanded row basis of block (t at l, v at L-l): |O_t| x r."""
    if l == bf.L:
        return bf.U[t]
    pv = v // 2
    E1 = _row_basis(bf, l + 1, 2 * t, pv)
    E2 = _row_basis(bf, l + 1, 2 * t + 1, pv)
    R = bf.R[(l, t, v)]
    k1 = E1.shape[1]
    return np.vstack([E1 @ R[:k1], E2 @ R[k1:]])


def _col_basis(bf, l, t, v):
    """Expanded column basis of block (t at l, v at L-l): r' x |S_v|."""
    if l == 0:
        return bf.Vt[v]
    pt = t // 2
    F1 = _col_basis(bf, l - 1, pt, 2 * v)
    F2 = _col_basis(bf, l - 1, pt, 2 * v + 1)
    W = bf.W[(l, t, v)]
    k1 = F1.shape[0]
    return np.hstack([W[:, :k1] @ F1, W[:, k1:] @ F2])


def bf_apply(bf, X, adjoint=False):
    """K X (or K^H X) from the dense decompression (the definition)."""
    K = bf_dense(bf)
    return (K.conj().T if adjoint else K) @ X


# ------------------------------------------------------------ Alg. 2
def bf_entry_eval(extract, to, ts, tol, proxy_cols, proxy_rows):
    """Butterfly construction by entry evaluation (Alg. 2).

    extract(list of (rows, cols)) -> list of dense blocks K(rows, cols)
    proxy_cols(t_level, t, v_level, v, rows) -> column indices in S_v
    proxy_rows(t_level, t, v_level, v, cols) -> row indices in O_t
    Indices are positions in [0, m) / [0, n).
    """
    bf = Butterfly(to, ts)
    L, lc = bf.L, bf.lc
    Obar, Sbar = {}, {}
    # left to middle
    for l in range(L, lc - 1, -1):
        lst, keys = [], []
        for t in range(2 ** l):
            for v in range(2 ** (L - l)):
                if l == L:
                    r0, r1 = to.node(L, t)
                    rows = np.arange(r0, r1)
                else:
                    pv = v // 2
                    rows = np.concatenate([Obar[(l + 1, 2 * t, pv)], Obar[(l + 1, 2 * t + 1, pv)]])
                cols = proxy_cols(l, t, L - l, v, rows)
                lst.append((rows, cols))
                keys.append((t, v))
        blocks = extract(lst)
        for (t, v), (rows, cols), K in zip(keys, lst, blocks):
            J, U = id_row(K, tol)
            Obar[(l, t, v)] = rows[J]
            if l == L:
                bf.U[t] = U
            else:
                bf.R[(l, t, v)] = U
    # right to middle
    for l in range(0, lc + 1):
        lst, keys = [], []
        for t in range(2 ** l):
            for v in range(2 ** (L - l)):
                if l == 0:
                    c0, c1 = ts.node(L, v)
                    cols = np.arange(c0, c1)
                else:
                    pt = t // 2
                    cols = np.concatenate([Sbar[(l - 1, pt, 2 * v)], Sbar[(l - 1, pt, 2 * v + 1)]])
                rows = proxy_rows(l, t, L - l, v, cols)
                lst.append((rows, cols))
                keys.append((t, v))
        blocks = extract(lst)
        for (t, v), (rows, cols), K in zip(keys, lst, blocks):
            J, Vt = id_col(K, tol)
            Sbar[(l, t, v)] = cols[J]
            if l == 0:
                bf.Vt[v] = Vt
            else:
                bf.W[(l, t, v)] = Vt
    # centre: skeleton matrices
    lst, keys = [], []
    for t in range(2 ** lc):
        for v in range(2 ** (L - lc)):
            lst.append((Obar[(lc, t, v)], Sbar[(lc, t, v)]))
            keys.append((t, v))
    for (t, v), K in zip(keys, extract(lst)):
        bf.B[(t, v)] = K
    bf.Obar, bf.Sbar = Obar, Sbar
    return bf


def uniform_proxies(rng, alpha):
    """Proxy sampler: alpha * |given| uniform samples (without replacement) in the node."""
    def cols(tl, t, vl, v, rows, tree):
        b, e = tree.node(vl, v)
        k = min(e - b, max(1, int(alpha * max(len(rows), 1))))
        return np.sort(rng.choice(np.arange(b, e), size=k, replace=False)) if e > b else np.zeros(0, np.int64)
    return cols


def dense_extractor(K):
    return lambda lst: [K[np.ix_(r, c)] for r, c in lst]


# ------------------------------------------------------------ Alg. 3
def extract_bf(bf, lst):
    """Submatrices K(X, Y) of a butterfly from its factors (Alg. 3).

    For every (X, Y): the row chains E^l of the blocks touching X are built
    from U and R (left to middle), the column chains F^l of the blocks touching
    Y from V and W (right to middle), and K(X, Y) = E^{lc} B F^{lc} summed over
    the centre blocks (t, v) the request touches.
    """
    L, lc = bf.L, bf.lc
    out = []
    for X, Y in lst:
        X = np.asarray(X); Y = np.asarray(Y)
        res = np.zeros((len(X), len(Y)), dtype=np.complex128)
        # rows of X in each level-l node, columns of Y in each level-(L-l) node
        E = {}
        for l in range(L, lc - 1, -1):
            for t in range(2 ** l):
                b, e = bf.to.node(l, t)
                xi = np.where((X >= b) & (X < e))[0]
                if xi.size == 0:
                    continue
                for v in range(2 ** (L - l)):
                    vb, ve = bf.ts.node(L - l, v)
                    if not np.any((Y >= vb) & (Y < ve)):
                        continue
                    if l == L:
                        E[(l, t, v)] = (xi, bf.U[t][X[xi] - b])
                    else:
                        pv = v // 2
                        parts = [E.get((l + 1, 2 * t, pv)), E.get((l + 1, 2 * t + 1, pv))]
                        R = bf.R[(l, t, v)]
                        k1 = _rank_left(bf, l + 1, 2 * t, pv)
                        rows, vals = [], []
                        if parts[0] is not None:
                            rows.append(parts[0][0]); vals.append(parts[0][1] @ R[:k1])
                        if parts[1] is not None:
                            rows.append(parts[1][0]); vals.append(parts[1][1] @ R[k1:])
                        E[(l, t, v)] = (np.concatenate(rows), np.vstack(vals))
        F = {}
        for l in range(0, lc + 1):
            for v in range(2 ** (L - l)):
                b, e = bf.ts.node(L - l, v)
                yi = np.where((Y >= b) & (Y < e))[0]
                if yi.size == 0:
                    continue
                for t in range(2 ** l):
                    tb, te = bf.to.node(l, t)
                    if not np.any((X >= tb) & (X < te)):
                        continue
                    if l == 0:
                        F[(l, t, v)] = (yi, bf.Vt[v][:, Y[yi] - b])
                    else:
                        pt = t // 2
                        parts = [F.get((l - 1, pt, 2 * v)), F.get((l - 1, pt, 2 * v + 1))]
                        Wm = bf.W[(l, t, v)]
                        k1 = _rank_right(bf, l - 1, pt, 2 * v)
                        cols, vals = [], []
                        if parts[0] is not None:
                            cols.append(parts[0][0]); vals.append(Wm[:, :k1] @ parts[0][1])
                        if parts[1] is not None:
                            cols.append(parts[1][0]); vals.append(Wm[:, k1:] @ parts[1][1])
                        F[(l, t, v)] = (np.concatenate(cols), np.hstack(vals))
        for (l, t, v), (xi, Ev) in E.items():
            if l != lc or (lc, t, v) not in F:
                continue
            yi, Fv = F[(lc, t, v)]
            res[np.ix_(xi, yi)] = Ev @ bf.B[(t, v)] @ Fv
        out.append(res)
    return out


def _rank_left(bf, l, t, v):
    if l == bf.L:
        return bf.U[t].shape[1]
    return bf.R[(l, t, v)].shape[1]


def _rank_right(bf, l, t, v):
    if l == 0:
        return bf.Vt[v].shape[0]
    return bf.W[(l, t, v)].shape[0]


# ------------------------------------------------------------ Sec. 3.3
def bf_random_matvec(matvec, rmatvec, to, ts, tol, samples, rng, max_samples=1024):
    """Randomized construction with adaptive sampling: whenever an ID rank
    comes within 8 of the number of samples the construction is repeated with
    twice the samples (a reading: the paper leaves the sample count open)."""
    while True:
        bf = _bf_random_matvec_once(matvec, rmatvec, to, ts, tol, samples, rng)
        if bf.max_id_rank < samples - 8 or samples >= max_samples:
            bf.samples = samples
            return bf
        samples *= 2


def _bf_random_matvec_once(matvec, rmatvec, to, ts, tol, samples, rng):
    """Butterfly from products with K (matvec) and K^H (rmatvec).

    Left side, level l: for every column node v at level L - l, a block of
    `samples` complex Gaussian vectors supported on S_v; the sketch K Omega_v
    restricted to the candidate rows (O_t at l = L, else the children's
    skeleton rows) replaces the proxy columns of Alg. 2 in the row ID.  The
    right side mirrors it with K^H.  The centre blocks solve
    B_{t,v} (V^T_{t,v} Omega_v) = (K Omega_v)(Obar_{t,v}, :) in least squares.
    """
    bf = Butterfly(to, ts)
    L, lc = bf.L, bf.lc
    m, n = to.n, ts.n

    def gauss(shape):
        return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)

    Obar, Sbar, Om, Ysk = {}, {}, {}, {}
    for l in range(L, lc - 1, -1):
        for v in range(2 ** (L - l)):
            b, e = ts.node(L - l, v)
            O = np.zeros((n, samples), dtype=np.complex128)
            O[b:e] = gauss((e - b, samples))
            Om[(l, v)] = O
            Ysk[(l, v)] = matvec(O)
    Psi, Zsk = {}, {}
    for l in range(0, lc + 1):
        for t in range(2 ** l):
            b, e = to.node(l, t)
            P = np.zeros((m, samples), dtype=np.complex128)
            P[b:e] = gauss((e - b, samples))
            Psi[(l, t)] = P
            Zsk[(l, t)] = rmatvec(P)
    for l in range(L, lc - 1, -1):
        for t in range(2 ** l):
            for v in range(2 ** (L - l)):
                if l == L:
                    r0, r1 = to.node(L, t)
                    rows = np.arange(r0, r1)
                else:
                    rows = np.concatenate([Obar[(l + 1, 2 * t, v // 2)], Obar[(l + 1, 2 * t + 1, v // 2)]])
                J, U = id_row(Ysk[(l, v)][rows], tol)
                Obar[(l, t, v)] = rows[J]
                if l == L:
                    bf.U[t] = U
                else:
                    bf.R[(l, t, v)] = U
    for l in range(0, lc + 1):
        for t in range(2 ** l):
            for v in range(2 ** (L - l)):
                if l == 0:
                    c0, c1 = ts.node(L, v)
                    cols = np.arange(c0, c1)
                else:
                    cols = np.concatenate([Sbar[(l - 1, t // 2, 2 * v)], Sbar[(l - 1, t // 2, 2 * v + 1)]])
                # column ID of K(O_t, cols) <=> row ID of K^H(cols, O_t), sketched by Psi_t
                J, Uc = id_row(Zsk[(l, t)][cols], tol)
                Sbar[(l, t, v)] = cols[J]
                Vt = Uc.conj().T  # K(:, cols) ~= K(:, cols[J]) Vt
                if l == 0:
                    bf.Vt[v] = Vt
                else:
                    bf.W[(l, t, v)] = Vt
    bf.max_id_rank = max([len(o) for o in Obar.values()] + [len(s_) for s_ in Sbar.values()] + [0])
    for t in range(2 ** lc):
        for v in range(2 ** (L - lc)):
            b, e = ts.node(L - lc, v)
            F = _col_basis(bf, lc, t, v)            # r' x |S_v|
            G = F @ Om[(lc, v)][b:e]                # r' x samples
            Yt = Ysk[(lc, v)][Obar[(lc, t, v)]]     # r x samples
            bf.B[(t, v)] = np.linalg.lstsq(G.T, Yt.T, rcond=None)[0].T
    bf.Obar, bf.Sbar = Obar, Sbar
    return bf
