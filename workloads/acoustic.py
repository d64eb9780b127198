"""3D visco-acoustic Helmholtz operator on a regular grid, 27-point stencil
with absorbing (PML) layers.

The paper's main workload is the visco-acoustic Helmholtz equation (Sec. 6,
the visco-acoustic experiments) with density rho, complex bulk modulus
kappa = v (1 - i / (2 q)) (v the velocity, q the quality factor), discretized
by an external 27-point staggered-grid stencil with 8 absorbing layers.  That
discretization is not available here, so this module defines a stand-in of
the same structure, derived from scratch:

* rho = 1 (as in the paper's heterogeneous-media run), so the operator is
  -(Laplace + (omega / kappa)^2) p = f.
* Laplace is the equal-weight average of three second-order discretizations
  that are each exact for quadratics: the axis stencil (6 face neighbours),
  the three rotated stencils that use the face diagonals of one coordinate
  plane plus the remaining axis (12 edge neighbours, 6 faces), and the
  body-diagonal stencil (8 corners; the sum of the four diagonal second
  differences is 4 h^2 times the Laplacian).  Scaled by h^2 the neighbour
  weights are then face 1/3 + 1/9, edge 1/18, corner 1/12.
* The mass term (omega h / kappa)^2 p is spread over the 27 points: half
  lumped at the centre and half the trilinear tensor-product average
  (centre 1/8, face 1/16, edge 1/32, corner 1/64 per point).
* Absorbing layers of `pml` nodes on every face: coordinate stretching
  d/dx_a -> (1 / xi_a) d/dx_a with xi_a = 1 + i gamma(d) / omega,
  gamma(d) = gamma0 (d / pml)^2 at depth d nodes into the layer and
  gamma0 = 3 v_max ln(1/R) / (2 L) for a nominal reflection R = 1e-3 over
  the layer width L = pml h.  A coupling along offset delta (with m nonzero
  components) is scaled by prod_a xi_a^(-2/m) at the row's node, so axis
  couplings carry 1 / xi_a^2 and diagonal ones the geometric mean of their
  axes' factors; the derivative of xi is neglected.
* The diagonal is minus the sum of the 26 scaled Laplacian weights (so the
  stretched Laplacian annihilates constants) minus the centre mass weight.

Unknowns are the n_x n_y n_z nodes (absorbing layers included) with
homogeneous Dirichlet data outside; index = x + n_x (y + n_y z).  Interior
rows have 27 nonzeros; the matrix is complex and non-symmetric inside the
absorbing layers.
"""
import numpy as np

from .helmholtz import grid_spacing, omega_for_ppw

# Laplacian weights (times h^2) by number of nonzero offset components
LAP_W = {1: 1.0 / 3.0 + 1.0 / 9.0, 2: 1.0 / 18.0, 3: 1.0 / 12.0}
# mass weights per neighbour by number of nonzero components, and the centre's
MASS_W = {1: 0.5 / 16.0, 2: 0.5 / 32.0, 3: 0.5 / 64.0}
MASS_CENTER = 0.5 + 0.5 / 8.0


def pml_profile(n, pml, gamma0_over_omega):
    """xi along one axis (length n): 1 + i gamma(d)/omega, d = depth into the layer."""
    i = np.arange(n, dtype=np.float64)
    d = np.maximum(np.maximum(pml - i, i - (n - 1 - pml)), 0.0)
    frac = d / pml if pml > 0 else np.zeros_like(d)
    return 1.0 + 1j * gamma0_over_omega * frac ** 2


def acoustic_27pt(dims, c=None, q=1e4, pml=8, ppw=8.0, omega=None, reflection=1e-3):
    """CSR matrix (rowptr int64, colind int32, values complex128) of h^2 times the operator.

    dims       : (nx, ny, nz) nodes per axis, absorbing layers included
    c          : None for v = 1, else an array of shape (nz, ny, nx) of velocities
    q          : quality factor (kappa = v (1 - i / (2 q)))
    pml        : absorbing-layer width in nodes (0: none)
    ppw        : points per wavelength at min(v) (ignored when omega is given)
    omega      : explicit angular frequency (0: the stretched Laplacian alone)
    Returns (rowptr, colind, values, meta).
    """
    nx, ny, nz = (int(d) for d in dims)
    n = nx * ny * nz
    h = grid_spacing(dims)
    v = np.ones((nz, ny, nx)) if c is None else np.asarray(c, dtype=np.float64).reshape(nz, ny, nx)
    vmin, vmax = float(v.min()), float(v.max())
    if omega is None:
        omega = omega_for_ppw(h, vmin, ppw)
    kappa = v * (1.0 - 0.5j / q)
    k2h2 = (omega * h / kappa) ** 2  # per node
    if pml > 0 and omega > 0:
        g = 3.0 * vmax * np.log(1.0 / reflection) / (2.0 * pml * h) / omega
    else:
        g = 0.0
    xi = [pml_profile(m, pml, g) for m in (nx, ny, nz)]
    # per-axis factors broadcast to (nz, ny, nx)
    xi3 = [xi[0][None, None, :], xi[1][None, :, None], xi[2][:, None, None]]

    idx = np.arange(n, dtype=np.int64).reshape(nz, ny, nx)
    rows, cols, vals = [], [], []
    diag = -MASS_CENTER * k2h2.astype(np.complex128)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                off = (dx, dy, dz)
                m = sum(1 for t in off if t != 0)
                if m == 0:
                    continue
                scale = np.ones((nz, ny, nx), dtype=np.complex128)
                for a in range(3):
                    if off[a] != 0:
                        scale = scale * xi3[a] ** (-2.0 / m)
                lap = LAP_W[m] * scale  # at every row node
                diag = diag + lap       # every neighbour enters the diagonal, inside the domain or not
                # rows whose neighbour at `off` exists; numpy axes are (z, y, x)
                src = [slice(None)] * 3
                dst = [slice(None)] * 3
                for a, t in enumerate(off):
                    ax = 2 - a
                    if t == -1:
                        src[ax], dst[ax] = slice(1, None), slice(None, -1)
                    elif t == 1:
                        src[ax], dst[ax] = slice(None, -1), slice(1, None)
                src, dst = tuple(src), tuple(dst)
                rows.append(idx[src].ravel())
                cols.append(idx[dst].ravel())
                vals.append((-lap[src] - MASS_W[m] * k2h2[src]).ravel())
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    meta = {"h": h, "omega": float(omega), "q": float(q), "pml": int(pml), "dims": (nx, ny, nz),
            "gamma0_over_omega": float(g), "coords": None}
    return rowptr, cols.astype(np.int32), vals.astype(np.complex128), meta
