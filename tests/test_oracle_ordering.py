"""Pins of the oracle's nested dissection, separator bisection and symbolic phase.

Checked against the paper's worked 11^2 example (Sec. 5, Fig.
'separator_ordering'), the closed-form root separator size of a k^3 grid
(Sec. 6, Poisson paragraph: the top separator of a k^3 grid is k x k), the
separator property, and a brute-force characterisation of I^u: the update set
of a front is the set of vertices outside its subtree adjacent to it; a box of
exactly leaf_max nodes is a leaf and one node fewer in the bound splits it.
"""
import json
import os

import numpy as np
import pytest

from workloads import helmholtz_7pt
from workloads.maxwell import yee_curlcurl
from oracle import nd
from oracle.symbolic import symbolic

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _xyz(idx, dims):
    nx, ny, _ = dims
    return idx % nx, (idx // nx) % ny, idx // (nx * ny)


def test_fig_11x11_separators_and_bisection():
    g = json.load(open(os.path.join(GOLD, "fig_separator_ordering_11x11.json")))
    dims = tuple(g["grid"])
    od = nd.nd_grid(dims, leaf_max=10, sep_leaf=3)
    root = od.nfronts - 1
    pts = od.perm[od.sbeg[root]:od.send[root]]
    x, y, _ = _xyz(pts, dims)
    assert len(pts) == g["root_separator"]["nodes"]
    assert np.all(x == g["root_separator"]["plane"])
    # level-1 separators: the children of the root
    kids = od.children[root]
    assert len(kids) == 2
    for k, spec in zip(kids, g["level1_separators"]):
        p = od.perm[od.sbeg[k]:od.send[k]]
        x, y, _ = _xyz(p, dims)
        assert np.all(y == spec["plane"]) and len(p) == spec["nodes"]
        assert x.min() == spec["x_range"][0] and x.max() == spec["x_range"][1] - 1
    lvl2 = []
    for k in kids:
        for kk in od.children[k]:
            p = od.perm[od.sbeg[kk]:od.send[kk]]
            x, y, _ = _xyz(p, dims)
            assert np.all(x == x[0])
            lvl2.append((int(x[0]), int(y.min()), int(y.max()) + 1, len(p)))
    want = sorted((s["plane"], s["y_range"][0], s["y_range"][1], s["nodes"]) for s in g["level2_separators"])
    assert sorted(lvl2) == want
    # recursive bisection of the root separator (y intervals, preorder)
    ys = _xyz(od.perm[od.sbeg[root]:od.send[root]], dims)[1]
    ivals = [[int(ys[b]), int(ys[e - 1])] for b, e, _, _ in od.septree[root][1:]]
    assert ivals == g["root_bisection_intervals_y"]
    # left row separator: 5 -> 3 | 2
    t = od.septree[kids[0]]
    assert [t[t[0][2]][1] - t[t[0][2]][0], t[t[0][3]][1] - t[t[0][3]][0]] == g["left_row_bisection_sizes"]


@pytest.mark.parametrize("k", [8, 24, 31, 40])
def test_root_separator_is_k_squared(k):
    od = nd.nd_grid((k, k, k), leaf_max=min(512, k ** 3 // 8))
    root = od.nfronts - 1
    assert od.send[root] - od.sbeg[root] == k * k


def _check_structure(rowptr, colind, od):
    n = od.n
    # bijection
    assert np.array_equal(np.sort(od.perm), np.arange(n))
    # postorder: children precede parents, separator ranges tile [0, n)
    assert od.sbeg[0] == 0 and od.send[-1] == n
    assert np.all(od.sbeg[1:] == od.send[:-1])
    for f in range(od.nfronts):
        for c in od.children[f]:
            assert c < f and od.parent[c] == f
    assert np.sum(od.parent < 0) == 1
    # subtree of each front is a contiguous range ending at send[f]
    first = np.array(od.sbeg)
    for f in range(od.nfronts):
        for c in od.children[f]:
            first[f] = min(first[f], first[c])
    # separator property: no A edge between the two children subtrees
    iperm = od.iperm
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    ri, ci = iperm[rows], iperm[colind]
    for f in range(od.nfronts):
        ks = od.children[f]
        if len(ks) == 2:
            a0, a1 = first[ks[0]], od.send[ks[0]]
            b0, b1 = first[ks[1]], od.send[ks[1]]
            cross = ((ri >= a0) & (ri < a1) & (ci >= b0) & (ci < b1))
            assert not np.any(cross)
    return first


def _check_iu_brute(rowptr, colind, od, sym, first):
    n = od.n
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    ri, ci = od.iperm[rows], od.iperm[colind]
    for f in range(od.nfronts):
        lo, hi = first[f], od.send[f]
        inside = (ri >= lo) & (ri < hi)
        boundary = np.unique(ci[inside & ((ci < lo) | (ci >= hi))])
        # postorder: vertices outside the subtree and adjacent to it are ancestors
        assert np.all(boundary >= hi)
        assert np.array_equal(sym.Iu[f], boundary), f
        p = od.parent[f]
        if p >= 0:
            allowed = np.concatenate([np.arange(od.sbeg[p], od.send[p]), sym.Iu[p]])
            assert np.all(np.isin(sym.Iu[f], allowed))
    assert sym.Iu[od.nfronts - 1].shape[0] == 0


@pytest.mark.parametrize("dims,leaf", [((6, 6, 6), 27), ((8, 8, 8), 64), ((7, 5, 9), 20), ((24, 24, 24), 512)])
def test_grid_structure_and_update_sets(dims, leaf):
    rowptr, colind, values, _ = helmholtz_7pt(dims, 0.05)
    od = nd.nd_grid(dims, leaf_max=leaf, sep_leaf=16)
    first = _check_structure(rowptr, colind, od)
    sym = symbolic(rowptr, colind, od)
    _check_iu_brute(rowptr, colind, od, sym, first)
    # maps: child update sets land inside the parent front, strictly increasing
    for f in range(od.nfronts):
        p = od.parent[f]
        if p < 0:
            continue
        m = sym.maps[f]
        assert np.all(np.diff(m) > 0)
        ns = od.send[p] - od.sbeg[p]
        full = np.concatenate([np.arange(od.sbeg[p], od.send[p]), sym.Iu[p]])
        assert np.array_equal(full[m], sym.Iu[f])
    # inverse maps: parent-local position -> child-local index, -1 where the child has no entry
    for f in range(od.nfronts):
        for k, c in enumerate(od.children[f]):
            inv = sym.invmaps[f][k]
            assert inv.shape[0] == (od.send[f] - od.sbeg[f]) + sym.Iu[f].shape[0]
            assert np.array_equal(inv[sym.maps[c]], np.arange(sym.maps[c].shape[0]))
            assert np.count_nonzero(inv >= 0) == sym.maps[c].shape[0] and np.all(inv >= -1)


def test_24_cubed_tree_matches_stated_shape():
    dims = (24, 24, 24)
    od = nd.nd_grid(dims, leaf_max=512)
    assert od.nfronts == 63
    assert int(np.sum(od.leaf)) == 32
    sep_sizes = sorted((int(od.send[f] - od.sbeg[f]) for f in range(od.nfronts) if not od.leaf[f]), reverse=True)
    # compressing separators of at least 256 nodes selects exactly the top three fronts
    assert sep_sizes[:3] == [576, 288, 264] and sep_sizes[3] < 256


def test_separator_bisection_tree_is_consistent():
    od = nd.nd_grid((20, 20, 20), leaf_max=512, sep_leaf=64)
    for f in range(od.nfronts):
        if od.leaf[f]:
            continue  # leaf boxes are never bisected
        t = od.septree[f]
        ns = od.send[f] - od.sbeg[f]
        assert t[0][0] == 0 and t[0][1] == ns
        for b, e, l, r in t:
            if l >= 0:
                assert t[l][0] == b and t[l][1] == t[r][0] and t[r][1] == e
                # first half holds ceil(ext / 2) planes: never smaller than the second
                assert t[l][1] - t[l][0] >= t[r][1] - t[r][0]
            else:
                assert e - b <= 64


def test_balanced_tree():
    t = nd.balanced_tree(11, 3)
    leaves = [(b, e) for b, e, l, r in t if l < 0]
    assert leaves == [(0, 3), (3, 6), (6, 9), (9, 11)]


def test_yee_structure_and_update_sets():
    n = 6
    rowptr, colind, values, meta = yee_curlcurl(n, 0.03)
    od = nd.nd_yee(n, meta["coords"], leaf_max=40, sep_leaf=16)
    first = _check_structure(rowptr, colind, od)
    sym = symbolic(rowptr, colind, od)
    _check_iu_brute(rowptr, colind, od, sym, first)
    # the root separator is the set of edges in the middle node plane x = n/2
    root = od.nfronts - 1
    c = meta["coords"][od.perm[od.sbeg[root]:od.send[root]]]
    assert np.all(c[:, 0] == 2 * (n // 2))
    assert c.shape[0] == 2 * n * (n - 1)  # y- and z-edges of one interior node plane


@pytest.mark.parametrize("dims,leaf_max", [((8, 8, 8), 512), ((4, 4, 4), 64), ((5, 4, 3), 60), ((7, 1, 1), 7)])
def test_box_of_exactly_leaf_max_nodes_is_a_leaf(dims, leaf_max):
    """A box with at most leaf_max nodes is a leaf: exactly leaf_max nodes gives one front holding the
    whole grid in natural order; one node fewer in the bound splits it at the middle plane of the
    longest axis, and the root separator is that plane."""
    n = dims[0] * dims[1] * dims[2]
    od = nd.nd_grid(dims, leaf_max=leaf_max)
    assert od.nfronts == 1 and od.leaf[0]
    assert np.array_equal(np.asarray(od.perm), np.arange(n))
    od2 = nd.nd_grid(dims, leaf_max=leaf_max - 1)
    assert od2.nfronts > 1
    a = int(np.argmax(dims))
    root = od2.nfronts - 1
    assert od2.send[root] - od2.sbeg[root] == n // dims[a]


def test_yee_separator_bisection_order_by_hand():
    """The P-hat bisection of a Yee separator, derived by hand from the reading of the separator
    bisection (longest in-plane extent of the region in doubled coordinates, ties to the lower axis,
    ceil(count / 2) coordinate positions first, natural order z, y, x inside a leaf) for 4^3 cells,
    separator leaves of at most 8 edges.  The root separator is the node plane x = 2 (doubled 4): its
    y-edges (y odd, z even) and z-edges (y even, z odd) with doubled y, z in [1, 7], 24 edges.
      split y at [1, 4] | [5, 7]: 14 | 10 edges
        [1, 4]: split z at [1, 4] | [5, 7]: 8 | 6
        [5, 7]: split z at [1, 4] | [5, 7]: 6 | 4"""
    from workloads.maxwell import yee_curlcurl
    _, _, _, meta = yee_curlcurl(4, 0.03)
    coords = np.asarray(meta["coords"])
    od = nd.nd_yee(4, coords, leaf_max=40, sep_leaf=8)
    root = od.nfronts - 1
    assert od.septree[root] == [[0, 24, 1, 4], [0, 14, 2, 3], [0, 8, -1, -1], [8, 14, -1, -1],
                                [14, 24, 5, 6], [14, 20, -1, -1], [20, 24, -1, -1]]
    sep = [tuple(int(v) for v in coords[e]) for e in od.perm[od.sbeg[root]:od.send[root]]]

    def leaf(ys_yedge, zs_yedge, ys_zedge, zs_zedge):
        """natural order (z outer, then y, then x) of the leaf's y-edges and z-edges"""
        pts = [(4, y, z) for y in ys_yedge for z in zs_yedge] + [(4, y, z) for y in ys_zedge for z in zs_zedge]
        return sorted(pts, key=lambda c: (c[2], c[1], c[0]))

    assert sep[0:8] == leaf([1, 3], [2, 4], [2, 4], [1, 3])
    assert sep[8:14] == leaf([1, 3], [6], [2, 4], [5, 7])
    assert sep[14:20] == leaf([5, 7], [2, 4], [6], [1, 3])
    assert sep[20:24] == leaf([5, 7], [6], [6], [5, 7])
