"""GPU parity of the butterfly kernels on caller-given dense matrices.

* Construction (kernel c): entry evaluation (Alg. 2) and randomized products
  (Sec. 3.3) of a Fourier-type kernel and of the Helmholtz Green's function
  between two separated planes reproduce the matrix within 10 * tol in the
  Frobenius norm; an exactly rank-3 matrix is reproduced to rounding for
  every level count L = 0..4 (ragged sizes, empty tree nodes).
* Apply (kernel b): K X and K^H X from the factors equal the decompressed
  matrix times X (decompression = the product applied to the identity), and
  the adjoint product is the conjugate transpose of the forward one.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def fourier_kernel(n, band):
    x = np.arange(n) / n
    return np.exp(2j * np.pi * band * np.outer(x, x))


def green_planes(k, wave, gap):
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
    return np.exp(2j * np.pi * wave * r) / r


def decompress(lib, b, shape):
    return lib.bfmf_bf_apply(b, shape, np.eye(shape[1], dtype=np.complex128))


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("kind,tol", [("fourier", 1e-3), ("fourier", 1e-6), ("green", 1e-4)])
def test_construction_and_apply(gpu_lib, method, kind, tol):
    K = fourier_kernel(256, 16) if kind == "fourier" else green_planes(16, 4, 0.5)
    b, shape = gpu_lib.bfmf_bf_compress_dense(K, 4, tol, method=method, samples=48, seed=5)
    try:
        D = decompress(gpu_lib, b, shape)
        err = np.linalg.norm(K - D) / np.linalg.norm(K)
        assert err <= 10 * tol, err
        info = gpu_lib.bfmf_bf_info(b)
        assert info["L"] == 4 and info["max_rank"] < 64
        rng = np.random.default_rng(1)
        X = rng.standard_normal((256, 5)) + 1j * rng.standard_normal((256, 5))
        Y = gpu_lib.bfmf_bf_apply(b, shape, X)
        assert np.linalg.norm(Y - D @ X) <= 1e-12 * np.linalg.norm(D @ X)
        Yh = gpu_lib.bfmf_bf_apply(b, shape, X, adjoint=True)
        assert np.linalg.norm(Yh - D.conj().T @ X) <= 1e-12 * np.linalg.norm(Yh)
    finally:
        gpu_lib.bfmf_bf_destroy(b)


@pytest.mark.parametrize("method", [0, 1])
def test_exact_low_rank_all_levels(gpu_lib, method):
    rng = np.random.default_rng(2)
    K = (rng.standard_normal((97, 3)) + 1j * rng.standard_normal((97, 3))) @ rng.standard_normal((3, 83))
    for L in range(5):
        b, shape = gpu_lib.bfmf_bf_compress_dense(K, L, 1e-12, method=method, samples=16, seed=L)
        try:
            D = decompress(gpu_lib, b, shape)
            assert np.linalg.norm(D - K) <= 1e-9 * np.linalg.norm(K), L
        finally:
            gpu_lib.bfmf_bf_destroy(b)


def test_rectangular_and_many_rhs(gpu_lib):
    K = fourier_kernel(300, 8)[:, :200]
    b, shape = gpu_lib.bfmf_bf_compress_dense(K, 3, 1e-8, method=0, seed=3)
    try:
        D = decompress(gpu_lib, b, shape)
        assert np.linalg.norm(D - K) <= 1e-6 * np.linalg.norm(K)
        X = np.random.default_rng(4).standard_normal((200, 130)) + 0j
        Y = gpu_lib.bfmf_bf_apply(b, shape, X)
        assert np.linalg.norm(Y - D @ X) <= 1e-12 * np.linalg.norm(Y)
    finally:
        gpu_lib.bfmf_bf_destroy(b)


def test_every_gemm_tile_shape_gives_the_same_result(gpu_lib):
    """The grouped GEMM behind every butterfly product runs in one of eight tile
    shapes (autotuned per launch, phases split by task height); each adds the products of an entry in the
    same order, so forcing any shape reproduces the autotuned result bit for
    bit: for applies of K and K^H with 1, 16 and 130 right-hand sides, and for
    a construction by randomized products."""
    K = green_planes(16, 3.0, 0.25)
    rng = np.random.default_rng(7)
    X = {nr: rng.standard_normal((K.shape[1], nr)) + 1j * rng.standard_normal((K.shape[1], nr))
         for nr in (1, 16, 130)}
    ref, ref_d = None, None
    try:
        for cfg in [-1, 0, 1, 2, 3, 4, 5, 6, 7]:
            gpu_lib.bfmf_set_gemm_tile(cfg)
            b, shape = gpu_lib.bfmf_bf_compress_dense(K, 3, 1e-6, method=1, seed=5)
            try:
                got = {nr: (gpu_lib.bfmf_bf_apply(b, shape, x), gpu_lib.bfmf_bf_apply(b, shape, x, adjoint=True))
                       for nr, x in X.items()}
                D = decompress(gpu_lib, b, shape)
            finally:
                gpu_lib.bfmf_bf_destroy(b)
            if ref is None:
                ref, ref_d = got, D
                assert np.linalg.norm(D - K) <= 1e-4 * np.linalg.norm(K)
                continue
            assert np.array_equal(D, ref_d), cfg
            for nr in X:
                assert np.array_equal(got[nr][0], ref[nr][0]) and np.array_equal(got[nr][1], ref[nr][1]), (cfg, nr)
    finally:
        gpu_lib.bfmf_set_gemm_tile(-1)
    with pytest.raises(gpu_lib.BfmfError):
        gpu_lib.bfmf_set_gemm_tile(8)


@pytest.mark.parametrize("method", [0, 1])
def test_interpolative_decomposition_over_1296_columns(gpu_lib, method):
    """The Gram ID kernel takes blocks of up to 2048 columns: a 1296 x 1296
    Green's-function block compressed with L = 0 (one ID over all 1296
    columns, tol 1e-3) by entry evaluation and by random products."""
    K = green_planes(36, 2, 0.5)
    assert K.shape == (1296, 1296)
    b, shape = gpu_lib.bfmf_bf_compress_dense(K, 0, 1e-3, method=method, samples=48, seed=11)
    try:
        D = decompress(gpu_lib, b, shape)
        err = np.linalg.norm(K - D) / np.linalg.norm(K)
        assert err <= 1e-2, err
        assert gpu_lib.bfmf_bf_info(b)["max_rank"] < 400
    finally:
        gpu_lib.bfmf_bf_destroy(b)


@pytest.mark.parametrize("m,n,r,tol", [(1300, 1100, 800, 1e-8), (2200, 1300, 1200, 1e-3)])
def test_wide_id_block_whose_column_chunks_have_full_rank(gpu_lib, m, n, r, tol):
    """Entry evaluation with L = 0 gives one ID over all m rows (with all n
    columns as proxies) and one over all n columns (all m rows as proxies).
    Blocks wider than one ID kernel takes are split into column chunks; when
    every chunk has full rank (rank r above the chunk width) the chunks'
    skeletons are as wide as the block and the whole block goes to one
    Householder ID instead (up to 8192 columns): at tol 1e-8 from the
    Householder limit of 1024 columns (both IDs), at tol 1e-3 from the Gram
    limit of 2048 (the 2200-column row ID).  K has exact rank r, so the
    butterfly has rank r and reproduces K to rounding.  Its factors have
    orthonormal columns and rows, so a chunk of K's rows or columns keeps
    singular values far above tol relative to its largest (a Gaussian
    factor's condition number would truncate the chunks below full rank)."""
    rng = np.random.default_rng(m + r)
    U = np.linalg.qr(rng.standard_normal((m, r)) + 1j * rng.standard_normal((m, r)))[0]
    V = np.linalg.qr(rng.standard_normal((n, r)) + 1j * rng.standard_normal((n, r)))[0].conj().T
    K = U @ V
    b, shape = gpu_lib.bfmf_bf_compress_dense(K, 0, tol, method=0, seed=13)
    try:
        assert gpu_lib.bfmf_bf_info(b)["max_rank"] == r
        D = decompress(gpu_lib, b, shape)
        err = np.linalg.norm(K - D) / np.linalg.norm(K)
        assert err <= 1e-6, err
    finally:
        gpu_lib.bfmf_bf_destroy(b)


def test_proxies_capped_at_the_householder_row_limit(gpu_lib):
    """Below tol 1e-4 the ID blocks go to the Householder kernel, which takes
    at most 2048 rows; entry evaluation on a 2600 x 700 matrix would draw
    min(2600, 4 * 700) = 2600 proxy rows for the column ID, so the sampler
    stops at 2048.  K has exact rank 300, which 2048 random rows still span,
    so the butterfly reproduces K to rounding."""
    rng = np.random.default_rng(17)
    m, n, r = 2600, 700, 300
    U = np.linalg.qr(rng.standard_normal((m, r)) + 1j * rng.standard_normal((m, r)))[0]
    V = np.linalg.qr(rng.standard_normal((n, r)) + 1j * rng.standard_normal((n, r)))[0].conj().T
    K = U @ V
    b, shape = gpu_lib.bfmf_bf_compress_dense(K, 0, 1e-8, method=0, seed=19)
    try:
        assert gpu_lib.bfmf_bf_info(b)["max_rank"] == r
        D = decompress(gpu_lib, b, shape)
        err = np.linalg.norm(K - D) / np.linalg.norm(K)
        assert err <= 1e-6, err
    finally:
        gpu_lib.bfmf_bf_destroy(b)
