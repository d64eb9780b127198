"""Geometric nested dissection and separator bisection (oracle).

Paper, Sec. 2: the fill-reducing permutation P is a nested-dissection
ordering of the pattern of A + A^T; the experiments on regular grids use
planar separators (Sec. 6).  Sec. 5.1: inside every separator a recursive
bisection defines the HOD-BF tree of F11 and the permutation P-hat; the
indices of I^u are sorted and split by a balanced binary tree.

Readings (the paper leaves the exact rules to METIS):
  * box [lo, hi) per axis; a box with at most ``leaf_max`` nodes is a leaf;
    otherwise cut the axis of largest extent (ties: x before y before z) at
    p = lo + ext // 2; children [lo, p) and [p+1, hi); empty children dropped.
  * numbering is postorder: left subtree, right subtree, then the separator.
  * a separator is bisected along its longest in-plane extent (ties: lower
    axis) with the first half holding ceil(ext / 2) planes, recursively down
    to at most ``sep_leaf`` nodes; nodes inside a leaf box are in natural
    order (x fastest).
  * Yee edge grids: a box is a range of cells, its unknowns are the edges
    strictly inside it, a separator is the set of edges lying in the middle
    node plane p = clo + ext // 2 (cells [clo, p) and [p, chi) remain).
"""
import numpy as np


class Ordering:
    """Result of nested dissection.

    perm[new] = old index; iperm[old] = new index.
    Fronts are numbered in postorder.  For front f: I^s = [sbeg[f], send[f]),
    parent[f] (-1 for the root), children[f] (list, left first), leaf[f].
    septree[f] is the bisection tree of I^s as a list of nodes
    (beg, end, left, right) in preorder, beg/end relative to sbeg[f],
    left/right indices into the same list (-1 at a leaf).
    """

    def __init__(self, n):
        self.n = n
        self.perm = []
        self.sbeg, self.send, self.parent, self.children, self.leaf = [], [], [], [], []
        self.septree = []

    def finish(self):
        self.perm = np.asarray(self.perm, dtype=np.int64)
        assert self.perm.shape[0] == self.n
        self.iperm = np.empty(self.n, dtype=np.int64)
        self.iperm[self.perm] = np.arange(self.n)
        self.sbeg = np.asarray(self.sbeg, dtype=np.int64)
        self.send = np.asarray(self.send, dtype=np.int64)
        self.parent = np.asarray(self.parent, dtype=np.int32)
        self.leaf = np.asarray(self.leaf, dtype=bool)
        return self

    @property
    def nfronts(self):
        return len(self.sbeg)


def _natural(lo, hi, nx, ny):
    """Global indices of the nodes in box [lo, hi), x fastest."""
    out = []
    for z in range(lo[2], hi[2]):
        for y in range(lo[1], hi[1]):
            for x in range(lo[0], hi[0]):
                out.append(x + nx * (y + ny * z))
    return out


def _bisect_tree(count_fn, emit_fn, split_fn, box, sep_leaf, nodes, base):
    """Recursive bisection of a separator; appends preorder nodes."""
    me = len(nodes)
    beg = base[0]
    nodes.append([beg, None, -1, -1])
    if count_fn(box) <= sep_leaf:
        emit_fn(box)
        base[0] += count_fn(box)
        nodes[me][1] = base[0]
        return me
    b1, b2 = split_fn(box)
    l = _bisect_tree(count_fn, emit_fn, split_fn, b1, sep_leaf, nodes, base)
    r = _bisect_tree(count_fn, emit_fn, split_fn, b2, sep_leaf, nodes, base)
    nodes[me][1] = base[0]
    nodes[me][2] = l
    nodes[me][3] = r
    return me


def nd_grid(dims, leaf_max=512, sep_leaf=64, parallel_levels=0):
    """Nested dissection of an nx*ny*nz node grid (natural index x fastest).

    parallel_levels > 0 is the separator variant of the Sec. 6 remark on high
    frequencies: a box at depth < parallel_levels is cut across the longest
    axis of the whole grid (while the box's extent there is at least 3), so
    the separators of the top levels are parallel planes.
    """
    nx, ny, nz = dims
    od = Ordering(nx * ny * nz)
    fixed = int(np.argmax([nx, ny, nz]))

    def count(box):
        lo, hi = box
        return max(0, hi[0] - lo[0]) * max(0, hi[1] - lo[1]) * max(0, hi[2] - lo[2])

    def emit(box):
        od.perm.extend(_natural(box[0], box[1], nx, ny))

    def split_sep(box):
        lo, hi = box
        ext = [hi[d] - lo[d] for d in range(3)]
        a = int(np.argmax(ext))  # first maximum: lower axis wins ties
        first = (ext[a] + 1) // 2
        hi1 = list(hi); hi1[a] = lo[a] + first
        lo2 = list(lo); lo2[a] = lo[a] + first
        return (list(lo), hi1), (lo2, list(hi))

    def rec(lo, hi, depth):
        vol = count((lo, hi))
        if vol == 0:
            return None
        if vol <= leaf_max:
            f = len(od.sbeg)
            beg = len(od.perm)
            emit((lo, hi))
            od.sbeg.append(beg); od.send.append(len(od.perm))
            od.parent.append(-1); od.children.append([]); od.leaf.append(True)
            od.septree.append([[0, len(od.perm) - beg, -1, -1]])
            return f
        ext = [hi[d] - lo[d] for d in range(3)]
        a = int(np.argmax(ext))
        if depth < parallel_levels and ext[fixed] >= 3:
            a = fixed
        p = lo[a] + ext[a] // 2
        hl = list(hi); hl[a] = p
        lr = list(lo); lr[a] = p + 1
        kids = [c for c in (rec(list(lo), hl, depth + 1), rec(lr, list(hi), depth + 1)) if c is not None]
        slo = list(lo); slo[a] = p
        shi = list(hi); shi[a] = p + 1
        beg = len(od.perm)
        nodes = []
        _bisect_tree(count, emit, split_sep, (slo, shi), sep_leaf, nodes, [0])
        f = len(od.sbeg)
        od.sbeg.append(beg); od.send.append(len(od.perm))
        od.parent.append(-1); od.children.append(kids); od.leaf.append(False)
        od.septree.append(nodes)
        for c in kids:
            od.parent[c] = f
        return f

    rec([0, 0, 0], [nx, ny, nz], 0)
    return od.finish()


def nd_yee(n, coords, leaf_max=512, sep_leaf=64):
    """Nested dissection of the interior edges of an n^3-cell Yee grid.

    coords: (N, 3) doubled edge coordinates; the edge numbering of the
    matrix is the row order of ``coords``.
    """
    coords = np.asarray(coords)
    N = coords.shape[0]
    od = Ordering(N)
    m = 2 * n + 1
    lookup = -np.ones((m, m, m), dtype=np.int64)
    lookup[coords[:, 2], coords[:, 1], coords[:, 0]] = np.arange(N)

    def inside_edges(dlo, dhi):
        """Edges with doubled coords in [dlo, dhi] per axis, natural order."""
        out = []
        for z in range(dlo[2], dhi[2] + 1):
            for y in range(dlo[1], dhi[1] + 1):
                for x in range(dlo[0], dhi[0] + 1):
                    e = lookup[z, y, x]
                    if e >= 0:
                        out.append(int(e))
        return out

    # a box of cells [clo, chi): interior edges have doubled coords in (2clo, 2chi)
    def count_cells(box):
        lo, hi = box
        return len(inside_edges([2 * lo[d] + 1 for d in range(3)], [2 * hi[d] - 1 for d in range(3)]))

    # separator region: doubled ranges [dlo, dhi] with one axis fixed
    def count_sep(box):
        return len(inside_edges(box[0], box[1]))

    def emit_sep(box):
        od.perm.extend(inside_edges(box[0], box[1]))

    def split_sep(box):
        dlo, dhi = box
        # extent measured in doubled units; the fixed axis has extent 0
        ext = [dhi[d] - dlo[d] for d in range(3)]
        a = int(np.argmax(ext))
        # split the doubled range into two halves of ceil/floor coordinate count
        cnt = ext[a] + 1
        first = (cnt + 1) // 2
        hi1 = list(dhi); hi1[a] = dlo[a] + first - 1
        lo2 = list(dlo); lo2[a] = dlo[a] + first
        return (list(dlo), hi1), (lo2, list(dhi))

    def rec(lo, hi):
        vol = count_cells((lo, hi))
        if vol == 0:
            return None
        if vol <= leaf_max:
            f = len(od.sbeg)
            beg = len(od.perm)
            od.perm.extend(inside_edges([2 * lo[d] + 1 for d in range(3)], [2 * hi[d] - 1 for d in range(3)]))
            od.sbeg.append(beg); od.send.append(len(od.perm))
            od.parent.append(-1); od.children.append([]); od.leaf.append(True)
            od.septree.append([[0, len(od.perm) - beg, -1, -1]])
            return f
        ext = [hi[d] - lo[d] for d in range(3)]
        a = int(np.argmax(ext))
        p = lo[a] + ext[a] // 2
        hl = list(hi); hl[a] = p
        lr = list(lo); lr[a] = p
        kids = [c for c in (rec(list(lo), hl), rec(lr, list(hi))) if c is not None]
        dlo = [2 * lo[d] + 1 for d in range(3)]
        dhi = [2 * hi[d] - 1 for d in range(3)]
        dlo[a] = 2 * p
        dhi[a] = 2 * p
        beg = len(od.perm)
        nodes = []
        _bisect_tree(count_sep, emit_sep, split_sep, (dlo, dhi), sep_leaf, nodes, [0])
        f = len(od.sbeg)
        od.sbeg.append(beg); od.send.append(len(od.perm))
        od.parent.append(-1); od.children.append(kids); od.leaf.append(False)
        od.septree.append(nodes)
        for c in kids:
            od.parent[c] = f
        return f

    rec([0, 0, 0], [n, n, n])
    return od.finish()


def balanced_tree(count, leaf):
    """Balanced bisection tree of ``count`` sorted indices (first half ceil).

    Returns preorder nodes (beg, end, left, right) like the separator tree.
    """
    nodes = []

    def rec(beg, end):
        me = len(nodes)
        nodes.append([beg, end, -1, -1])
        if end - beg <= leaf:
            return me
        mid = beg + (end - beg + 1) // 2
        l = rec(beg, mid)
        r = rec(mid, end)
        nodes[me][2] = l
        nodes[me][3] = r
        return me

    if count > 0:
        rec(0, count)
    return nodes
