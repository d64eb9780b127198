"""GPU list routing (Sec. 5) against the oracle's assembled fronts, element by element.

The compressed fronts never form F = [A(Is,Is) A(Is,Iu); A(Iu,Is) 0] (+) C_nu1
(+) C_nu2: entry evaluation requests entries F(rows, cols), and each request
is split into its A part and its child parts through the inverse extend-add
maps.  bfmf_extract_front runs that extraction for arbitrary index lists.  For
a front whose children are dense the entries must equal the oracle's
assembled front (Alg. 1 assembly) to rounding of the children's Schur
products (1e-12 in complex128; 1e-5 in complex64, whose Schur products run on
FP32 MFMA); for a dense front they must equal the GPU's own assembled front
bit for bit (the same additions in the same order).  The requests include
whole blocks, the 1 x 1 and 1 x 2 requests of the extraction figure,
repeated indices and rows or columns of I^u alone (where A contributes
nothing)."""
import numpy as np
import pytest

from workloads import make_problem, rng_for
from oracle import nd
from oracle import multifrontal as mf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c1_fronts():
    p = make_problem("helmholtz24")
    od = nd.nd_grid(p.dims, leaf_max=512, sep_leaf=64)
    fac = mf.factor(p.rowptr, p.colind, p.values, od, keep_fronts=True)
    return p, od, fac


def _requests(n, ns, rng):
    all_ = np.arange(n)
    out = [(all_, all_),                                     # the whole front
           (np.arange(ns), np.arange(ns, n)),                 # F12
           (np.arange(ns, n), np.arange(ns)),                 # F21
           (np.arange(ns, n), np.arange(ns, n)),              # C_nu1 (+) C_nu2 on I^u x I^u only
           (np.array([n // 2]), np.array([ns // 3])),         # 1 x 1
           (np.array([ns - 1]), np.array([0, n - 1]))]        # 1 x 2
    for _ in range(4):  # scattered lists, with repeats
        out.append((rng.integers(0, n, 37), rng.integers(0, n, 23)))
    return out


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_list_routing_equals_the_assembled_front(gpu_lib, c1_fronts, precision):
    p, od, fac = c1_fronts
    prec = gpu_lib.BFMF_C128 if precision == "c128" else gpu_lib.BFMF_C64_MIXED
    tol = 1e-12 if precision == "c128" else 1e-5
    s = gpu_lib.Solver(0).analyze(p.rowptr, p.colind, p.values, dims=p.dims)
    try:
        s.factor(tol=1e-3, n_min=256, batched=True, precision=prec, keep_fronts=True)
        ns_all = od.send - od.sbeg
        comp = lambda f: len(od.children[f]) > 0 and ns_all[f] >= 256
        # compressed fronts whose children are dense, and dense separator fronts
        fronts = [f for f in range(od.nfronts) if comp(f) and not any(comp(c) for c in od.children[f])]
        dense = [f for f in range(od.nfronts) if od.children[f] and not comp(f)][:4]
        assert len(fronts) == 2 and len(dense) == 4
        rng = rng_for("test", "rhs", (24, 7))
        for f in fronts + dense:
            F = fac.fronts[f]
            n, ns = F.shape[0], int(ns_all[f])
            scale = np.abs(F).max()
            Fg = s.front(f, 0) if f in dense else None  # the GPU's assembled front (dense fronts)
            for rows, cols in _requests(n, ns, rng):
                got = gpu_lib.bfmf_extract_front(s.h, f, rows, cols)
                want = F[np.ix_(rows, cols)]
                assert np.abs(got - want).max() <= tol * scale, (f, rows[:4], cols[:4])
                if Fg is not None:
                    assert np.array_equal(got, Fg[np.ix_(rows, cols)]), (f, rows[:4], cols[:4])
        with pytest.raises(gpu_lib.BfmfError):
            gpu_lib.bfmf_extract_front(s.h, fronts[0], np.array([0]), np.array([10 ** 6]))
    finally:
        s.close()
