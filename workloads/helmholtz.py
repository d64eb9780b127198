"""3D Helmholtz operator on a regular grid (7-point finite differences).

The problem is  -Laplace(u) - (omega/c)^2 (1 + i delta) u = f  on the unit cube
with homogeneous Dirichlet data.  Unknowns sit on the n_x*n_y*n_z interior
nodes x_i = (i+1) h, h = 1/(n+1) (the boundary nodes carry 0 and are
eliminated).  The matrix is scaled by h^2, so the diagonal is
6 - (omega h / c)^2 (1 + i delta) and every neighbour coupling is -1.

Nodes are numbered naturally: index = x + n_x * (y + n_y * z).
"""
import numpy as np


def omega_for_ppw(h, c_min=1.0, ppw=8.0):
    """Angular frequency giving ``ppw`` grid points per wavelength at ``c_min``."""
    return 2.0 * np.pi * c_min / (ppw * h)


def grid_spacing(dims):
    return 1.0 / (max(dims) + 1)


def helmholtz_7pt(dims, delta, c=None, ppw=8.0, omega=None):
    """CSR matrix (rowptr int64, colind int32, values complex128) of h^2 * H.

    dims   : (nx, ny, nz) interior nodes per axis
    delta  : damping, omega^2 is replaced by omega^2 (1 + i delta)
    c      : None for c = 1, else an array of shape (nz, ny, nx) of velocities
    ppw    : points per wavelength at min(c) (ignored when omega is given)
    omega  : explicit angular frequency (0 gives the Poisson operator)
    Returns (rowptr, colind, values, meta) with meta holding h and omega.
    """
    nx, ny, nz = (int(d) for d in dims)
    n = nx * ny * nz
    h = grid_spacing(dims)
    if c is None:
        cfield = np.ones((nz, ny, nx))
    else:
        cfield = np.asarray(c, dtype=np.float64).reshape(nz, ny, nx)
    cmin = float(cfield.min())
    if omega is None:
        omega = omega_for_ppw(h, cmin, ppw)
    kh2 = (omega * h / cfield) ** 2  # (omega h / c)^2 per node
    diag = (6.0 - kh2 * (1.0 + 1j * delta)).ravel()

    idx = np.arange(n, dtype=np.int64).reshape(nz, ny, nx)
    rows = [idx.ravel()]
    cols = [idx.ravel()]
    vals = [diag]
    # neighbours along each axis, both directions
    for axis in range(3):
        for step in (-1, 1):
            src = [slice(None)] * 3
            dst = [slice(None)] * 3
            # numpy axes are (z, y, x): map our axis 0=x to numpy axis 2
            ax = 2 - axis
            if step == -1:
                src[ax] = slice(1, None)
                dst[ax] = slice(None, -1)
            else:
                src[ax] = slice(None, -1)
                dst[ax] = slice(1, None)
            r = idx[tuple(src)].ravel()
            cc = idx[tuple(dst)].ravel()
            rows.append(r)
            cols.append(cc)
            vals.append(np.full(r.shape, -1.0 + 0.0j))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    meta = {"h": h, "omega": float(omega), "delta": float(delta), "dims": (nx, ny, nz),
            "coords": None}
    return rowptr, cols.astype(np.int32), vals.astype(np.complex128), meta


def grf_velocity(dims, rng, corr=0.1, std=0.5, lo=1.0, hi=2.0):
    """c(x) = clip(1 + g(x), lo, hi), g a Gaussian random field.

    g has zero mean, standard deviation ``std`` and covariance
    std^2 exp(-r^2 / (2 corr^2)); it is sampled by circulant embedding on a
    periodic grid padded to twice the size along each axis.  Returns an
    array of shape (nz, ny, nx).
    """
    nx, ny, nz = dims
    h = grid_spacing(dims)
    shp = (2 * nz, 2 * ny, 2 * nx)
    axes = []
    for m in shp:
        k = np.arange(m)
        d = np.minimum(k, m - k) * h  # periodic distance
        axes.append(d)
    dz, dy, dx = np.meshgrid(*axes, indexing="ij", sparse=True)
    cov = np.exp(-(dx ** 2 + dy ** 2 + dz ** 2) / (2.0 * corr ** 2))
    lam = np.real(np.fft.fftn(cov))
    lam = np.sqrt(np.maximum(lam, 0.0))
    w = rng.standard_normal(shp)
    g = np.real(np.fft.ifftn(lam * np.fft.fftn(w)))
    g = g[:nz, :ny, :nx] * std
    return np.clip(1.0 + g, lo, hi)
