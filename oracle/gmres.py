"""Restarted GMRES(m) with modified Gram-Schmidt (oracle).

Sec. 6 of the paper: the approximate factorization M is a left
preconditioner for GMRES(30) with modified Gram-Schmidt and zero initial
guess, stopping when ||u_i|| <= 1e-10 or ||u_i|| / ||u_0|| <= 1e-6 where
u_i = M^-1 (A x_i - b).  Columns of a right-hand-side block are solved
independently (no block Krylov).
"""
import numpy as np


def gmres(matvec, precond, b, restart=30, max_iter=300, rtol=1e-6, atol=1e-10):
    """Left-preconditioned GMRES for one column. Returns (x, iters, hist)."""
    b = np.asarray(b, dtype=np.complex128)
    n = b.shape[0]
    x = np.zeros(n, dtype=np.complex128)
    u0 = None
    hist = []
    it = 0
    while it < max_iter:
        r = precond(b - matvec(x))
        beta = np.linalg.norm(r)
        if u0 is None:
            u0 = beta
            hist.append(beta)
        if beta <= atol or (u0 > 0 and beta / u0 <= rtol):
            break
        V = np.zeros((n, restart + 1), dtype=np.complex128)
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        cs = np.zeros(restart, dtype=np.complex128)
        sn = np.zeros(restart, dtype=np.complex128)
        g = np.zeros(restart + 1, dtype=np.complex128)
        g[0] = beta
        V[:, 0] = r / beta
        j_done = 0
        for j in range(restart):
            w = precond(matvec(V[:, j]))
            for i in range(j + 1):  # modified Gram-Schmidt
                H[i, j] = np.vdot(V[:, i], w)
                w = w - H[i, j] * V[:, i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0:
                V[:, j + 1] = w / H[j + 1, j]
            for i in range(j):  # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + np.conj(cs[i]) * H[i + 1, j]
                H[i, j] = t
            a, bb = H[j, j], H[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            if den == 0:
                cs[j], sn[j] = 1.0, 0.0
            else:
                cs[j] = a / den if a != 0 else 0.0
                sn[j] = (np.conj(bb) / den) if a == 0 else (a / abs(a)) * np.conj(bb) / den
                if a != 0:
                    cs[j] = abs(a) / den
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_done = j + 1
            res = abs(g[j + 1])
            hist.append(res)
            if res <= atol or res / u0 <= rtol or it >= max_iter:
                break
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), g[:j_done]) if j_done else np.zeros(0)
        x = x + V[:, :j_done] @ y
        if hist[-1] <= atol or hist[-1] / u0 <= rtol:
            break
    return x, it, np.asarray(hist)
