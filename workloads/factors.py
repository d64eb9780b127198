"""Random butterfly factors (seeded), for checking entry extraction.

The factored form K = U^L R^{L-1} .. R^{lc} B^{lc} W^{lc} .. W^1 V^0 of a
butterfly is a set of dense blocks whose shapes follow from one rank per
block; this module draws the ranks and complex Gaussian blocks of those shapes
and lists them in the order the C ABI's import expects.  It performs no step
of any factorization: the same blocks are handed to the CPU oracle (as a
dictionary) and to the library (as a flat array).
"""
import numpy as np

from .seeds import rng_for


def halving_bounds(n, L):
    """Node boundaries per level of the halving tree of [0, n) (first half ceil)."""
    out = [np.array([0, n], dtype=np.int64)]
    for _ in range(L):
        b = out[-1]
        nxt = [int(b[0])]
        for i in range(len(b) - 1):
            lo, hi = int(b[i]), int(b[i + 1])
            nxt += [lo + (hi - lo + 1) // 2, hi]
        out.append(np.array(nxt, dtype=np.int64))
    return out


def random_butterfly(m, n, L, rmin, rmax, seed, zero_frac=0.0):
    """Ranks in [rmin, rmax] (a fraction zero_frac of them 0) and Gaussian blocks.

    Returns (ranks_left, ranks_right, flat, blocks): the rank arrays and flat
    complex128 array of the C ABI's import, and blocks = {"U": {t: ..},
    "R": {(l, t, v): ..}, "B": {(t, v): ..}, "W": {(l, t, v): ..},
    "V": {v: ..}} with the same matrices."""
    rng = rng_for("test", "factors", (m, n, L, seed))
    lc = L // 2
    nb = 1 << L
    to, ts = halving_bounds(m, L), halving_bounds(n, L)

    def rank():
        if zero_frac > 0 and rng.random() < zero_frac:
            return 0
        return int(rng.integers(rmin, rmax + 1))

    rl = np.array([[rank() for _ in range(nb)] for _ in range(lc, L + 1)], dtype=np.int32)
    rr = np.array([[rank() for _ in range(nb)] for _ in range(lc + 1)], dtype=np.int32)

    def RL(l, t, v):
        return int(rl[l - lc][t * (1 << (L - l)) + v])

    def RR(l, t, v):
        return int(rr[l][t * (1 << (L - l)) + v])

    def gauss(r, c):
        k = max(c, 1)
        return (rng.standard_normal((r, c)) + 1j * rng.standard_normal((r, c))) / np.sqrt(2.0 * k)

    blocks = {"U": {}, "R": {}, "B": {}, "W": {}, "V": {}}
    flat = []
    for t in range(nb):
        U = gauss(int(to[L][t + 1] - to[L][t]), RL(L, t, 0))
        blocks["U"][t] = U
        flat.append(U.ravel(order="F"))
    for l in range(L - 1, lc - 1, -1):
        vs = 1 << (L - l)
        for t in range(1 << l):
            for v in range(vs):
                rows = RL(l + 1, 2 * t, v // 2) + RL(l + 1, 2 * t + 1, v // 2)
                R = gauss(rows, RL(l, t, v))
                blocks["R"][(l, t, v)] = R
                flat.append(R.ravel(order="F"))
    vs = 1 << (L - lc)
    for t in range(1 << lc):
        for v in range(vs):
            B = gauss(RL(lc, t, v), RR(lc, t, v))
            blocks["B"][(t, v)] = B
            flat.append(B.ravel(order="F"))
    for l in range(lc, 0, -1):
        vs = 1 << (L - l)
        for t in range(1 << l):
            for v in range(vs):
                cols = RR(l - 1, t // 2, 2 * v) + RR(l - 1, t // 2, 2 * v + 1)
                W = gauss(RR(l, t, v), cols)
                blocks["W"][(l, t, v)] = W
                flat.append(W.ravel(order="F"))
    for v in range(nb):
        V = gauss(RR(0, 0, v), int(ts[L][v + 1] - ts[L][v]))
        blocks["V"][v] = V
        flat.append(V.ravel(order="F"))
    flat = np.concatenate(flat) if flat else np.zeros(0, np.complex128)
    return rl, rr, flat.astype(np.complex128), blocks
