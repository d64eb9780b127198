"""Right-hand sides: point sources, noisy centre source, edge dipoles.

All blocks are column-major (N, nrhs) complex128 arrays.
"""
import numpy as np


def center_source_with_noise(dims, rng, noise=1e-3):
    """Unit source at node (nx//2, ny//2, nz//2) plus noise * CN(0,1) per entry."""
    nx, ny, nz = dims
    n = nx * ny * nz
    b = np.zeros((n, 1), dtype=np.complex128)
    c = nx // 2 + nx * (ny // 2 + ny * (nz // 2))
    b[c, 0] = 1.0
    g = rng.standard_normal((n, 2))
    b[:, 0] += noise * (g[:, 0] + 1j * g[:, 1]) / np.sqrt(2.0)
    return b


def point_sources(n, nrhs, rng):
    """nrhs unit sources at uniformly random unknowns (one per column)."""
    nodes = rng.integers(0, n, size=nrhs)
    b = np.zeros((n, nrhs), dtype=np.complex128, order="F")
    b[nodes, np.arange(nrhs)] = 1.0
    return b


def random_edge_dipoles(n_edges, nrhs, rng):
    """Unit current on a uniformly random edge per column."""
    return point_sources(n_edges, nrhs, rng)


def request_stream(rate, seconds, sizes, max_rhs, rng):
    """Serving requests: Poisson arrivals at `rate` per second during `seconds`;
    each request picks a model uniformly among len(sizes) and carries 1..max_rhs
    (uniform) unit point sources at distinct uniformly random unknowns of that
    model.  Returns a list of (arrival time, model, rows)."""
    out = []
    t = rng.exponential(1.0 / rate)
    while t < seconds:
        m = int(rng.integers(0, len(sizes)))
        k = int(rng.integers(1, max_rhs + 1))
        rows = rng.choice(sizes[m], size=k, replace=False)
        out.append((float(t), m, rows))
        t += rng.exponential(1.0 / rate)
    return out
