"""3D Maxwell curl-curl operator on a Yee staggered grid with PEC walls.

Unknowns are the tangential electric field on the interior edges of an
n^3 cell grid on the unit cube (spacing h = 1/n).  Edges tangential to the
boundary are zero (perfect electric conductor) and eliminated, leaving
3 n (n-1)^2 unknowns.  With C the edge-to-face incidence (circulation with
+-1 entries) the scaled operator is

    A = C^T C - (omega h)^2 (1 + i delta) diag(eps_e)

where eps_e is the mean permittivity of the four cells sharing an edge and
mu = 1.  Each edge is described by doubled integer coordinates
(2i+1, 2j, 2k) for an x-edge, (2i, 2j+1, 2k) for a y-edge and
(2i, 2j, 2k+1) for a z-edge; edges are numbered x-edges first, then y, then
z, each block in natural order of its doubled coordinates (x fastest).
"""
import numpy as np


def _edge_lists(n):
    """Doubled coordinates of interior edges, grouped by orientation."""
    out = []
    rng1 = np.arange(1, n)       # interior node planes
    rng0 = np.arange(0, n)       # cell index along the edge direction
    # x-edges: i in [0,n), j,k in [1,n)
    k, j, i = np.meshgrid(rng1, rng1, rng0, indexing="ij")
    out.append(np.stack([2 * i + 1, 2 * j, 2 * k], axis=-1).reshape(-1, 3))
    k, j, i = np.meshgrid(rng1, rng0, rng1, indexing="ij")
    out.append(np.stack([2 * i, 2 * j + 1, 2 * k], axis=-1).reshape(-1, 3))
    k, j, i = np.meshgrid(rng0, rng1, rng1, indexing="ij")
    out.append(np.stack([2 * i, 2 * j, 2 * k + 1], axis=-1).reshape(-1, 3))
    return np.concatenate(out).astype(np.int32)


def yee_curlcurl(n, delta, eps_cells=None, omega=None):
    """CSR (rowptr, colind, values, meta) of the scaled Yee curl-curl operator.

    n         : cells per axis
    delta     : damping of omega^2
    eps_cells : (n, n, n) permittivity per cell indexed [k, j, i]; None -> 1
    omega     : angular frequency; default pi / (8 h), i.e. 8 cells per
                wavelength where eps = 4
    meta['coords'] holds the doubled edge coordinates (N, 3) int32.
    """
    h = 1.0 / n
    if omega is None:
        omega = np.pi / (8.0 * h)
    if eps_cells is None:
        eps_cells = np.ones((n, n, n))
    coords = _edge_lists(n)
    N = coords.shape[0]
    m = 2 * n + 1
    lookup = -np.ones((m, m, m), dtype=np.int64)  # [z, y, x] doubled
    lookup[coords[:, 2], coords[:, 1], coords[:, 0]] = np.arange(N)

    # faces in doubled coordinates: a face has two odd coordinates
    rows_f, cols_f, vals_f = [], [], []
    face_id = 0
    for normal in range(3):
        a, b = [d for d in range(3) if d != normal]
        # face centre: odd along a and b, even along normal
        ra = np.arange(1, 2 * n, 2)
        rn = np.arange(0, 2 * n + 1, 2)
        grids = {a: ra, b: ra, normal: rn}
        gz, gy, gx = np.meshgrid(grids[2], grids[1], grids[0], indexing="ij")
        centre = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=-1)
        nf = centre.shape[0]
        fid = face_id + np.arange(nf)
        face_id += nf
        # circulation around the normal (right-handed a -> b)
        # edges: (-b side, along a) +, (+a side, along b) +, (+b side, along a) -, (-a side, along b) -
        for off_axis, sign_side, sign in ((b, -1, 1.0), (a, +1, 1.0), (b, +1, -1.0), (a, -1, -1.0)):
            e = centre.copy()
            e[:, off_axis] += sign_side
            inside = np.all((e >= 0) & (e <= 2 * n), axis=1)
            eid = -np.ones(nf, dtype=np.int64)
            ei = e[inside]
            eid[inside] = lookup[ei[:, 2], ei[:, 1], ei[:, 0]]
            keep = eid >= 0
            rows_f.append(fid[keep])
            cols_f.append(eid[keep])
            vals_f.append(np.full(int(keep.sum()), sign))
    rows_f = np.concatenate(rows_f)
    cols_f = np.concatenate(cols_f)
    vals_f = np.concatenate(vals_f)
    import scipy.sparse as sp
    C = sp.csr_matrix((vals_f, (rows_f, cols_f)), shape=(face_id, N))
    K = (C.T @ C).tocsr()

    # permittivity per edge: mean over the (up to 4) cells touching it
    eps_e = np.zeros(N)
    cnt = np.zeros(N)
    for d in range(3):
        sel = np.where(coords[:, d] % 2 == 1)[0]
        others = [q for q in range(3) if q != d]
        for s1 in (-1, 1):
            for s2 in (-1, 1):
                cc = coords[sel].copy()
                cc[:, others[0]] += s1
                cc[:, others[1]] += s2
                ok = np.all((cc > 0) & (cc < 2 * n), axis=1)
                ci = (cc[ok] - 1) // 2  # cell index (i, j, k)
                eps_e[sel[ok]] += eps_cells[ci[:, 2], ci[:, 1], ci[:, 0]]
                cnt[sel[ok]] += 1
    eps_e /= cnt
    M = sp.diags((omega * h) ** 2 * (1.0 + 1j * delta) * eps_e)
    A = (K.astype(np.complex128) - M).tocsr()
    A.sort_indices()
    meta = {"h": h, "omega": float(omega), "delta": float(delta), "cells": n,
            "coords": coords, "eps_edge": eps_e}
    return (A.indptr.astype(np.int64), A.indices.astype(np.int32),
            A.data.astype(np.complex128), meta)


def block_permittivity(n, block, rng, lo=1.0, hi=4.0):
    """Piecewise-constant permittivity on cubes of ``block`` cells, U[lo, hi]."""
    nb = (n + block - 1) // block
    vals = rng.uniform(lo, hi, size=(nb, nb, nb))
    k = np.arange(n) // block
    return vals[k[:, None, None], k[None, :, None], k[None, None, :]]
