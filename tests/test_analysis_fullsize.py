"""The C++ analysis at the full sizes of the measured workloads, on the CPU.

Ordering, assembly tree, update sets I^u, extend-add maps and separator
bisection trees (Alg. 1 and Alg. 5, steps before the numeric loop; Sec. 2 and
Sec. 5.1) must equal the oracle's bit for bit on the 100^3 and 128^3
Helmholtz grids, the 64^3-cell Yee grid and the three serving grids.
"""
import numpy as np
import pytest

from workloads import make_problem
from workloads.configs import serving_grids
from oracle import nd
from oracle.symbolic import symbolic

bfmf = pytest.importorskip("paper_2007_00202_amd.bfmf")

pytestmark = pytest.mark.slow


def _check(p, sl=None):
    h = bfmf.bfmf_create(-1)
    sl = sl or p.opts.get("sep_leaf", 64)
    try:
        if p.kind == "grid":
            bfmf.bfmf_analyze(h, p.rowptr, p.colind, p.values, dims=p.dims, sep_leaf=sl)
            od = nd.nd_grid(p.dims, leaf_max=512, sep_leaf=sl)
        else:
            bfmf.bfmf_analyze(h, p.rowptr, p.colind, p.values, kind=bfmf.BFMF_ORD_YEE, dims=(p.cells, 0, 0),
                              coords=p.coords, sep_leaf=sl)
            od = nd.nd_yee(p.cells, p.coords, leaf_max=512, sep_leaf=sl)
        sym = symbolic(p.rowptr, p.colind, od)
        s = bfmf.bfmf_get_symbolic(h)
        assert np.array_equal(s["perm"], od.perm)
        assert np.array_equal(s["sbeg"], od.sbeg) and np.array_equal(s["send"], od.send)
        assert np.array_equal(s["parent"], od.parent)
        kids = [list(s["child_list"][s["child_ptr"][f]:s["child_ptr"][f + 1]]) for f in range(od.nfronts)]
        assert kids == [list(c) for c in od.children]
        iu_ptr = s["iu_ptr"]
        want_iu = np.concatenate([np.asarray(sym.Iu[f], np.int64) for f in range(od.nfronts)])
        want_map = np.concatenate([np.asarray(sym.maps[f], np.int64) for f in range(od.nfronts)])
        assert np.array_equal(np.diff(iu_ptr), [len(sym.Iu[f]) for f in range(od.nfronts)])
        assert np.array_equal(s["iu"][:iu_ptr[-1]], want_iu)
        assert np.array_equal(s["map"][:iu_ptr[-1]], want_map)
        for f in range(od.nfronts):
            nodes = s["sep_nodes"][s["sep_ptr"][f]:s["sep_ptr"][f + 1]]
            assert nodes.tolist() == [list(t) for t in od.septree[f]], f
        return od
    finally:
        bfmf.bfmf_destroy(h)


@pytest.mark.parametrize("name,root_ns,nfronts", [("helmholtz100", 100 * 100, 4095),
                                                  ("helmholtz128grf", 128 * 128, 8191),
                                                  ("maxwell64", None, 4095)])
def test_full_size_analysis_matches_oracle(name, root_ns, nfronts):
    p = make_problem(name)
    od = _check(p)
    assert od.nfronts == nfronts
    if root_ns is not None:
        assert od.send[-1] - od.sbeg[-1] == root_ns


@pytest.mark.parametrize("g", serving_grids())
def test_serving_grids_analysis_matches_oracle(g):
    _check(make_problem("helmholtz100", n=g, nrhs=1, config_id="serving"), sl=64)


def test_full_size_analysis_default_leaf():
    """The 100^3 grid with the default separator leaf size (64) as well."""
    _check(make_problem("helmholtz100"), sl=64)
