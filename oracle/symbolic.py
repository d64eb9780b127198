"""Assembly tree, update index sets and extend-add maps (oracle).

Paper, Sec. 2: front F_tau has fully-summed rows/columns I^s_tau and update
rows/columns I^u_tau; for a child nu of tau, I^u_nu is contained in
I^s_tau u I^u_tau, and the root has an empty I^u.  Extend-add scatters the
child's contribution block C_nu into the parent front.

I^u_tau = sorted((U_children I^u_nu  u  adj_{A+A^T}(I^s_tau)) minus I^s_tau),
restricted to indices above max I^s_tau (ancestors, in postorder).

map_nu[k]   = position of I^u_nu[k] in concat(I^s_tau, I^u_tau)
invmap[c][p] = k with map_{child c}[k] = p, or -1 (parent-local -> child-local)
"""
import numpy as np
import scipy.sparse as sp


class Symbolic:
    pass


def symmetric_pattern_new(rowptr, colind, od):
    """CSR pattern of P (A + A^T) P^T in the new numbering (no values)."""
    n = rowptr.shape[0] - 1
    A = sp.csr_matrix((np.ones(colind.shape[0]), colind, rowptr), shape=(n, n))
    S = (A + A.T).tocsr()
    Pm = sp.csr_matrix((np.ones(n), (np.arange(n), od.perm)), shape=(n, n))
    Snew = (Pm @ S @ Pm.T).tocsr()
    Snew.sort_indices()
    return Snew.indptr.astype(np.int64), Snew.indices.astype(np.int64)


def symbolic(rowptr, colind, od):
    """Compute I^u, maps and inverse maps for every front of ``od``."""
    sptr, sind = symmetric_pattern_new(rowptr, colind, od)
    nf = od.nfronts
    Iu = [None] * nf
    for f in range(nf):
        b, e = int(od.sbeg[f]), int(od.send[f])
        parts = [sind[sptr[b]:sptr[e]]]
        for c in od.children[f]:
            parts.append(Iu[c])
        u = np.unique(np.concatenate(parts)) if parts else np.zeros(0, np.int64)
        Iu[f] = u[u >= e].astype(np.int64)
    maps = [None] * nf
    for f in range(nf):
        p = int(od.parent[f])
        if p < 0:
            maps[f] = np.zeros(0, dtype=np.int32)
            continue
        pb, pe = int(od.sbeg[p]), int(od.send[p])
        u = Iu[f]
        pos = np.empty(u.shape[0], dtype=np.int64)
        ins = (u >= pb) & (u < pe)
        pos[ins] = u[ins] - pb
        k = np.searchsorted(Iu[p], u[~ins])
        assert np.all(Iu[p][k] == u[~ins]), "I^u of a child not contained in its parent front"
        pos[~ins] = (pe - pb) + k
        maps[f] = pos.astype(np.int32)
    invmaps = []
    for f in range(nf):
        nfr = int(od.send[f] - od.sbeg[f]) + Iu[f].shape[0]
        inv = []
        for c in od.children[f]:
            a = -np.ones(nfr, dtype=np.int32)
            a[maps[c]] = np.arange(maps[c].shape[0], dtype=np.int32)
            inv.append(a)
        invmaps.append(inv)
    s = Symbolic()
    s.Iu = Iu
    s.maps = maps
    s.invmaps = invmaps
    s.sptr, s.sind = sptr, sind
    return s


def front_size(od, sym, f):
    return int(od.send[f] - od.sbeg[f]) + sym.Iu[f].shape[0]


def levels(od):
    """Depth of every front (root = 0)."""
    d = np.zeros(od.nfronts, dtype=np.int32)
    for f in range(od.nfronts - 1, -1, -1):
        p = od.parent[f]
        d[f] = 0 if p < 0 else d[p] + 1
    return d
