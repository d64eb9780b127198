"""Pins of the oracle's ID and butterfly algorithms (paper Sec. 3).

* ID: exact-rank matrices are reproduced to rounding with U(J,:) = I; for a
  matrix with decaying singular values the error follows the tolerance.
* Trees: the partition shapes of the 4-level example (Fig. 'complementary
  rank': 1x16, 2x8, 4x4, 8x2, 16x1 blocks).
* bf_entry_eval (Alg. 2) and bf_random_matvec: closed-form oscillatory
  kernels -- a Fourier-type kernel exp(2 pi i n x y) and the 3D Helmholtz
  Green's function between two parallel planes -- are compressed with
  ||K - K~||_F <= 10 eps ||K||_F; an exactly rank-3 matrix is reproduced.
* bf_random_matvec on a generic rank-r matrix: exact to rounding for L = 0..3
  on ragged sizes, each ID keeping exactly min(r, rows, columns) of its block.
* extract_bf (Alg. 3): entries equal the decompressed matrix, including the
  1x1 and 1x2 requests of the 2-level example (Fig. 'extract').
"""
import numpy as np
import pytest

from oracle import butterfly as bfo


def fourier_kernel(n, band):
    x = np.arange(n) / n
    return np.exp(2j * np.pi * band * np.outer(x, x))


def green_planes(k, wave, gap=0.15, return_points=False):
    """exp(i kappa r) / r between two parallel k x k point planes, bisection order."""
    h = 1.0 / k
    pts = []
    def rec(x0, x1, y0, y1):
        if (x1 - x0) * (y1 - y0) == 1:
            pts.append((x0, y0))
            return
        if x1 - x0 >= y1 - y0:
            m = x0 + (x1 - x0 + 1) // 2
            rec(x0, m, y0, y1); rec(m, x1, y0, y1)
        else:
            m = y0 + (y1 - y0 + 1) // 2
            rec(x0, x1, y0, m); rec(x0, x1, m, y1)
    rec(0, k, 0, k)
    P = np.array(pts, dtype=float) * h
    X = np.column_stack([P, np.zeros(len(P))])
    Y = np.column_stack([P, np.full(len(P), gap)])
    r = np.linalg.norm(X[:, None, :] - Y[None, :, :], axis=2)
    kappa = 2 * np.pi * wave
    K = np.exp(1j * kappa * r) / r
    return (K, X, Y) if return_points else K


def samplers(to, ts, rng, alpha=4, X=None, Y=None, knn=0):
    """alpha |given| uniform proxies, plus the knn nearest points of every given
    index inside the node when coordinates X (rows) / Y (columns) are known."""
    def pick(b, e, given, P, Q):
        k = min(e - b, max(8, alpha * len(given)))
        sel = set(rng.choice(np.arange(b, e), size=k, replace=False).tolist())
        if knn and P is not None and e > b:
            d = np.linalg.norm(P[given][:, None, :] - Q[b:e][None, :, :], axis=2)
            for row in np.argsort(d, axis=1)[:, :knn]:
                sel.update((b + row).tolist())
        return np.array(sorted(sel), dtype=np.int64)

    def pc(tl, t, vl, v, rows):
        b, e = ts.node(vl, v)
        return pick(b, e, rows, X, Y)

    def pr(tl, t, vl, v, cols):
        b, e = to.node(tl, t)
        return pick(b, e, cols, Y, X)
    return pc, pr


def test_id_exact_rank_and_tolerance():
    rng = np.random.default_rng(0)
    A = (rng.standard_normal((40, 3)) + 1j * rng.standard_normal((40, 3))) @ rng.standard_normal((3, 30))
    J, U = bfo.id_row(A, 1e-12)
    assert len(J) == 3
    assert np.allclose(U[J], np.eye(3))
    assert np.linalg.norm(A - U @ A[J]) <= 1e-12 * np.linalg.norm(A)
    # geometric singular values 2^-k: error of the order of the tolerance
    Q1, _ = np.linalg.qr(rng.standard_normal((60, 60)) + 1j * rng.standard_normal((60, 60)))
    Q2, _ = np.linalg.qr(rng.standard_normal((60, 60)))
    M = Q1 @ np.diag(2.0 ** -np.arange(60)) @ Q2
    for tol in (1e-3, 1e-6):
        J, U = bfo.id_row(M, tol)
        err = np.linalg.norm(M - U @ M[J], 2)
        assert err <= 100 * tol and len(J) <= int(np.log2(1 / tol)) + 6
    J2, Vt = bfo.id_col(A, 1e-12)
    assert np.linalg.norm(A - A[:, J2] @ Vt) <= 1e-12 * np.linalg.norm(A)


def test_tree_partitions_of_the_4_level_example():
    t = bfo.Tree(16, 4)
    for l in range(5):
        sizes = np.diff(t.bounds[l])
        assert len(sizes) == 2 ** l and np.all(sizes == 16 // 2 ** l)
    # blocks at level l: 2^l row nodes x 2^(L-l) column nodes -> 1x16, 2x8, 4x4, 8x2, 16x1
    assert [(2 ** l, 2 ** (4 - l)) for l in range(5)] == [(1, 16), (2, 8), (4, 4), (8, 2), (16, 1)]
    # bisection nodes are honoured; leaves without children are split ceil/floor
    nodes = [[0, 11, 1, 2], [0, 6, -1, -1], [6, 11, -1, -1]]
    t2 = bfo.Tree(11, 2, nodes)
    assert list(t2.bounds[1]) == [0, 6, 11] and list(t2.bounds[2]) == [0, 3, 6, 9, 11]


@pytest.mark.parametrize("tol", [1e-3, 1e-6])
@pytest.mark.parametrize("kind", ["fourier", "green"])
def test_entry_eval_compresses_oscillatory_kernels(tol, kind):
    rng = np.random.default_rng(7)
    L = 4
    if kind == "fourier":
        K = fourier_kernel(256, 16)
        to, ts = bfo.Tree(K.shape[0], L), bfo.Tree(K.shape[1], L)
        pc, pr = samplers(to, ts, rng)
    else:
        # close-by planes: uniform proxies plus nearest neighbours (Sec. 3.2)
        K, X, Y = green_planes(16, 4, return_points=True)
        to, ts = bfo.Tree(K.shape[0], L), bfo.Tree(K.shape[1], L)
        pc, pr = samplers(to, ts, rng, X=X, Y=Y, knn=8)
    bf = bfo.bf_entry_eval(bfo.dense_extractor(K), to, ts, tol, pc, pr)
    Kt = bfo.bf_dense(bf)
    err = np.linalg.norm(K - Kt) / np.linalg.norm(K)
    assert err <= 10 * tol, err
    if kind == "fourier" or tol >= 1e-3:
        assert bf.ranks() < 64  # genuinely compressed at the 64 x 64 centre blocks
    x = rng.standard_normal((K.shape[1], 2)) + 0j
    assert np.allclose(bfo.bf_apply(bf, x), Kt @ x)


def test_nearest_neighbour_proxies_beat_uniform_for_close_planes():
    """Uniform proxies lose accuracy for close-by interactions (Sec. 3.2)."""
    K, X, Y = green_planes(16, 4, return_points=True)
    to, ts = bfo.Tree(256, 4), bfo.Tree(256, 4)
    errs = []
    for knn in (0, 8):
        pc, pr = samplers(to, ts, np.random.default_rng(7), X=X, Y=Y, knn=knn)
        bf = bfo.bf_entry_eval(bfo.dense_extractor(K), to, ts, 1e-3, pc, pr)
        errs.append(np.linalg.norm(K - bfo.bf_dense(bf)) / np.linalg.norm(K))
    assert errs[1] < errs[0] and errs[1] <= 1e-2


def test_entry_eval_reproduces_exact_low_rank():
    rng = np.random.default_rng(1)
    K = (rng.standard_normal((96, 3)) + 1j * rng.standard_normal((96, 3))) @ rng.standard_normal((3, 80))
    for L in (0, 1, 2, 3):
        to, ts = bfo.Tree(96, L), bfo.Tree(80, L)
        pc, pr = samplers(to, ts, rng)
        bf = bfo.bf_entry_eval(bfo.dense_extractor(K), to, ts, 1e-12, pc, pr)
        assert np.linalg.norm(bfo.bf_dense(bf) - K) <= 1e-10 * np.linalg.norm(K)


def test_extract_matches_decompression():
    rng = np.random.default_rng(3)
    K = fourier_kernel(64, 6)
    to, ts = bfo.Tree(64, 2), bfo.Tree(64, 2)
    pc, pr = samplers(to, ts, rng)
    bf = bfo.bf_entry_eval(bfo.dense_extractor(K), to, ts, 1e-8, pc, pr)
    D = bfo.bf_dense(bf)
    # the two requests of the 2-level example: a 1x1 and a 1x2 submatrix
    lst = [(np.array([5]), np.array([40])), (np.array([50]), np.array([3, 30]))]
    lst += [(np.sort(rng.choice(64, 7, replace=False)), np.sort(rng.choice(64, 9, replace=False))) for _ in range(5)]
    for (X, Y), blk in zip(lst, bfo.extract_bf(bf, lst)):
        assert np.allclose(blk, D[np.ix_(X, Y)], atol=1e-13 * np.abs(D).max())


@pytest.mark.parametrize("kind", ["fourier", "green"])
def test_random_matvec_construction(kind):
    rng = np.random.default_rng(11)
    K = fourier_kernel(256, 16) if kind == "fourier" else green_planes(16, 4)
    tol = 1e-4
    to, ts = bfo.Tree(K.shape[0], 4), bfo.Tree(K.shape[1], 4)
    bf = bfo.bf_random_matvec(lambda X: K @ X, lambda X: K.conj().T @ X, to, ts, tol, 48, rng)
    err = np.linalg.norm(K - bfo.bf_dense(bf)) / np.linalg.norm(K)
    assert err <= 10 * tol, err


@pytest.mark.parametrize("L", [0, 1, 2, 3])
@pytest.mark.parametrize("r", [1, 5, 11])
def test_random_matvec_is_exact_on_exact_rank(L, r):
    """A generic rank-r matrix K = X Y^H: every block K(rows, S_v) has rank min(r, |rows|, |S_v|), and a
    Gaussian sketch with at least that many columns keeps every row dependency (the range-finder argument
    of randomized low-rank approximation), so the construction is exact up to rounding and each ID keeps
    exactly that many rows (columns).  At L = 0 this is the two-sided randomized ID of the whole matrix.
    Ragged sizes (97 x 83) give unequal siblings at every level."""
    rng = np.random.default_rng(100 * L + r)
    m, n = 97, 83
    X = rng.standard_normal((m, r)) + 1j * rng.standard_normal((m, r))
    Y = rng.standard_normal((n, r)) + 1j * rng.standard_normal((n, r))
    K = X @ Y.conj().T
    to, ts = bfo.Tree(m, L), bfo.Tree(n, L)
    bf = bfo.bf_random_matvec(lambda V: K @ V, lambda V: K.conj().T @ V, to, ts, 1e-12, 24, rng)
    assert bf.samples == 24
    assert np.linalg.norm(bfo.bf_dense(bf) - K) <= 1e-10 * np.linalg.norm(K)
    for (l, t, v), rows in bf.Obar.items():
        if l == L:
            cand = to.node(L, t)[1] - to.node(L, t)[0]
        else:
            cand = len(bf.Obar[(l + 1, 2 * t, v // 2)]) + len(bf.Obar[(l + 1, 2 * t + 1, v // 2)])
        b, e = ts.node(L - l, v)
        assert len(rows) == min(r, cand, e - b), (l, t, v)
    for (l, t, v), cols in bf.Sbar.items():
        if l == 0:
            cand = ts.node(L, v)[1] - ts.node(L, v)[0]
        else:
            cand = len(bf.Sbar[(l - 1, t // 2, 2 * v)]) + len(bf.Sbar[(l - 1, t // 2, 2 * v + 1)])
        b, e = to.node(l, t)
        assert len(cols) == min(r, cand, e - b), (l, t, v)
