"""Separator variant of the Sec. 6 remark on high frequencies: the top levels
of the nested dissection cut across one axis, so their separators are
parallel planes and the F12/F21 blocks of those fronts couple
well-separated planes.

Pins that follow from the geometry rather than from the oracle's code: the
separators at depth < parallel_levels are whole planes perpendicular to the
grid's longest axis at the box midpoints; a depth-1 front's update set I^u is
exactly the root plane (its subtree is a slab bounded by that plane alone,
7-point stencil); a depth-2 slab between two planes has both planes as I^u;
parallel_levels = 0 reproduces the default ordering.  Then the C++ analysis
against the oracle with the variant on, and its error paths.
"""
import numpy as np
import pytest

from workloads import helmholtz_7pt
from oracle import nd
from oracle.symbolic import symbolic


def _xyz(g, dims):
    nx, ny, _ = dims
    return g % nx, (g // nx) % ny, g // (nx * ny)


def _depth(od):
    d = np.zeros(od.nfronts, np.int32)
    for f in range(od.nfronts - 1, -1, -1):
        d[f] = 0 if od.parent[f] < 0 else d[od.parent[f]] + 1
    return d


def _plane_nodes(dims, x):
    nx, ny, nz = dims
    y, z = np.meshgrid(np.arange(ny), np.arange(nz), indexing="ij")
    return np.sort((x + nx * (y + ny * z)).ravel())


@pytest.mark.parametrize("dims", [(16, 12, 10), (10, 17, 9)])
def test_top_separators_are_parallel_planes(dims):
    a = int(np.argmax(dims))
    od = nd.nd_grid(dims, leaf_max=64, sep_leaf=16, parallel_levels=3)
    dep = _depth(od)
    perm = np.asarray(od.perm)
    plane = int(np.prod(dims)) // dims[a]
    cuts = set()
    for f in np.flatnonzero(dep < 3):
        g = perm[od.sbeg[f]:od.send[f]]
        c = _xyz(g, dims)[a]
        assert len(g) == plane and np.all(c == c[0]), f  # a whole plane across axis a
        cuts.add(int(c[0]))
    n = dims[a]
    h = n // 2
    q1, q2 = h // 2, h + 1 + (n - h - 1) // 2
    assert {h, q1, q2} <= cuts
    # default rule below: some deeper separator is not perpendicular to axis a
    assert any(len(set(_xyz(perm[od.sbeg[f]:od.send[f]], dims)[a])) > 1 for f in np.flatnonzero(dep >= 3)
               if not od.leaf[f])


def test_update_sets_of_parallel_fronts_are_the_bounding_planes():
    dims = (16, 8, 6)  # x longest
    rp, ci, v, _ = helmholtz_7pt(dims, 0.05)
    od = nd.nd_grid(dims, leaf_max=32, sep_leaf=8, parallel_levels=3)
    sym = symbolic(rp, ci, od)
    dep = _depth(od)
    perm = np.asarray(od.perm)
    xs_of = lambda f: sorted(set(_xyz(perm[np.asarray(sym.Iu[f], np.int64)], dims)[0].tolist()))
    for f in np.flatnonzero(dep == 1):  # slab [0,8) or [9,16): bounded by x = 8 alone
        assert np.array_equal(np.sort(perm[np.asarray(sym.Iu[f], np.int64)]), _plane_nodes(dims, 8))
    got = sorted(xs_of(f) for f in np.flatnonzero(dep == 2))
    # slabs [0,4) | [5,8) | [9,12) | [13,16): one or two bounding planes each
    assert got == [[4], [4, 8], [8, 12], [12]]


def test_zero_parallel_levels_is_the_default_ordering():
    dims = (12, 9, 10)
    a = nd.nd_grid(dims, leaf_max=40, sep_leaf=8)
    b = nd.nd_grid(dims, leaf_max=40, sep_leaf=8, parallel_levels=0)
    assert np.array_equal(a.perm, b.perm) and np.array_equal(a.parent, b.parent)
    c = nd.nd_grid(dims, leaf_max=40, sep_leaf=8, parallel_levels=2)
    assert not np.array_equal(a.perm, c.perm)


bfmf = pytest.importorskip("paper_2007_00202_amd.bfmf")


@pytest.mark.parametrize("dims,leaf,sl,pl", [((16, 12, 10), 64, 16, 2), ((10, 17, 9), 40, 8, 3),
                                             ((12, 12, 12), 27, 8, 20), ((100, 100, 100), 512, 128, 2)])
def test_cpp_analysis_matches_oracle_with_parallel_separators(dims, leaf, sl, pl):
    rp, ci, v, _ = helmholtz_7pt(dims, 0.05)
    h = bfmf.bfmf_create(-1)
    try:
        bfmf.bfmf_analyze(h, rp, ci, v, dims=dims, leaf_max=leaf, sep_leaf=sl, parallel_levels=pl)
        od = nd.nd_grid(dims, leaf_max=leaf, sep_leaf=sl, parallel_levels=pl)
        sym = symbolic(rp, ci, od)
        s = bfmf.bfmf_get_symbolic(h)
        assert np.array_equal(s["perm"], od.perm)
        assert np.array_equal(s["sbeg"], od.sbeg) and np.array_equal(s["send"], od.send)
        assert np.array_equal(s["parent"], od.parent)
        iu_ptr = s["iu_ptr"]
        assert np.array_equal(np.diff(iu_ptr), [len(sym.Iu[f]) for f in range(od.nfronts)])
        want_iu = np.concatenate([np.asarray(sym.Iu[f], np.int64) for f in range(od.nfronts)])
        want_map = np.concatenate([np.asarray(sym.maps[f], np.int64) for f in range(od.nfronts)])
        assert np.array_equal(s["iu"][:iu_ptr[-1]], want_iu)
        assert np.array_equal(s["map"][:iu_ptr[-1]], want_map)
        for f in range(od.nfronts):
            nodes = s["sep_nodes"][s["sep_ptr"][f]:s["sep_ptr"][f + 1]]
            assert nodes.tolist() == [list(t) for t in od.septree[f]], f
    finally:
        bfmf.bfmf_destroy(h)


def test_parallel_levels_error_paths():
    from workloads.maxwell import yee_curlcurl
    rp, ci, v, _ = helmholtz_7pt((6, 6, 6), 0.05)
    h = bfmf.bfmf_create(-1)
    try:
        with pytest.raises(bfmf.BfmfError) as e:
            bfmf.bfmf_analyze(h, rp, ci, v, dims=(6, 6, 6), parallel_levels=-1)
        assert e.value.status == bfmf.BFMF_E_INVAL
        rp2, ci2, v2, meta = yee_curlcurl(4, 0.03)
        with pytest.raises(bfmf.BfmfError) as e:
            bfmf.bfmf_analyze(h, rp2, ci2, v2, kind=bfmf.BFMF_ORD_YEE, dims=(4, 0, 0), coords=meta["coords"],
                              parallel_levels=1)
        assert e.value.status == bfmf.BFMF_E_INVAL
        bfmf.bfmf_analyze(h, rp, ci, v, dims=(6, 6, 6), leaf_max=27, sep_leaf=8, parallel_levels=1)
    finally:
        bfmf.bfmf_destroy(h)
