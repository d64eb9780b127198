"""Entry extraction from butterflies (extract_BF, Alg. 3).

CPU: the oracle's extract_bf, which multiplies only the factor blocks a
request touches, equals the submatrices of the full decompression (the
factored form of Sec. 3 multiplied out) on random factors, including blocks
of rank zero, empty tree nodes and repeated indices.
GPU: the library's extraction of the same factors (imported through the C
ABI, expanded to the centre level and read one dot product per entry)
equals the oracle's extract_bf element by element.
"""
import numpy as np
import pytest

from oracle.butterfly import Tree, Butterfly, bf_dense, extract_bf
from workloads import random_butterfly, rng_for


def oracle_bf(m, n, L, blocks):
    bf = Butterfly(Tree(m, L), Tree(n, L))
    bf.U, bf.R, bf.B, bf.W, bf.Vt = blocks["U"], blocks["R"], blocks["B"], blocks["W"], blocks["V"]
    return bf


def requests(m, n, rng, count, max_len):
    out = []
    for _ in range(count):
        r = rng.integers(0, m, size=int(rng.integers(1, max_len + 1)))
        c = rng.integers(0, n, size=int(rng.integers(1, max_len + 1)))
        out.append((r, c))
    return out


# the two requests of the paper's extraction figure on a 2-level butterfly: one entry, and one
# row against two columns that lie in different centre column nodes
def figure_requests(m, n):
    return [(np.array([m // 8]), np.array([n - 1 - n // 8])),
            (np.array([max(m - 2, 0)]), np.array([min(1, n - 1), min(n // 2 + 1, n - 1)]))]


CASES = [  # m, n, L, rmin, rmax, zero_frac
    (1, 1, 0, 1, 1, 0.0),
    (7, 5, 0, 1, 4, 0.0),
    (16, 16, 1, 1, 3, 0.0),
    (40, 33, 2, 1, 5, 0.0),
    (64, 64, 2, 0, 4, 0.3),
    (50, 70, 3, 1, 6, 0.1),
    (130, 97, 4, 1, 5, 0.2),
    (6, 20, 3, 1, 2, 0.0),  # empty row-tree nodes
]


@pytest.mark.parametrize("m,n,L,rmin,rmax,zf", CASES)
def test_oracle_extract_equals_decompression(m, n, L, rmin, rmax, zf):
    rl, rr, flat, blocks = random_butterfly(m, n, L, rmin, rmax, seed=L, zero_frac=zf)
    bf = oracle_bf(m, n, L, blocks)
    K = bf_dense(bf)
    rng = rng_for("test", "factors", (m, n, L, 1000))
    lst = requests(m, n, rng, 12, 9) + figure_requests(m, n)
    for (r, c), got in zip(lst, extract_bf(bf, lst)):
        np.testing.assert_allclose(got, K[np.ix_(r, c)], rtol=0, atol=1e-13 * max(1.0, np.abs(K).max()))


def test_import_count_checked():
    bfmf = pytest.importorskip("paper_2007_00202_amd.bfmf")
    rl, rr, flat, _ = random_butterfly(40, 33, 2, 1, 5, seed=2)
    with pytest.raises(bfmf.BfmfError) as e:
        bfmf.bfmf_bf_import(40, 33, 2, rl, rr, flat[:-1], device=-1)
    assert e.value.status == bfmf.BFMF_E_INVAL
    bad = rl.copy()
    bad[0, 0] = -1
    with pytest.raises(bfmf.BfmfError) as e:
        bfmf.bfmf_bf_import(40, 33, 2, bad, rr, flat, device=-1)
    assert e.value.status == bfmf.BFMF_E_INVAL


@pytest.mark.gpu
@pytest.mark.parametrize("m,n,L,rmin,rmax,zf", CASES + [(1000, 900, 6, 8, 24, 0.05)])
def test_gpu_extract_equals_oracle(gpu_lib, m, n, L, rmin, rmax, zf):
    rl, rr, flat, blocks = random_butterfly(m, n, L, rmin, rmax, seed=L, zero_frac=zf)
    bf = oracle_bf(m, n, L, blocks)
    rng = rng_for("test", "factors", (m, n, L, 2000))
    lst = requests(m, n, rng, 40, 70) + figure_requests(m, n)
    want = extract_bf(bf, lst)
    print(f"m {m} n {n} L {L}: {len(lst)} requests", flush=True)
    b, shape = gpu_lib.bfmf_bf_import(m, n, L, rl, rr, flat)
    try:
        got = gpu_lib.bfmf_bf_extract(b, lst)
        got2 = gpu_lib.bfmf_bf_extract(b, lst[::-1])  # the centre form is built once and reused
    finally:
        gpu_lib.bfmf_bf_destroy(b)
    scale = max(1.0, max(np.abs(w).max() for w in want))
    for w, g, g2 in zip(want, got, got2[::-1]):
        assert g.shape == w.shape
        np.testing.assert_allclose(g, w, rtol=0, atol=1e-13 * scale)
        assert np.array_equal(g, g2)
