"""Named workloads with their sizes, damping, precision and right-hand sides.

The paper's own experiments use a 27-point staggered stencil with PML, the
Marmousi2 model and a Nedelec finite-element mesh; none of those inputs are
available, so these synthetic problems of the same structure stand in for
them (3D cube, planar nested-dissection separators, point-source
excitations, heterogeneous velocity, indefinite curl-curl, and a 27-point
visco-acoustic stencil with absorbing layers derived here).
"""
from dataclasses import dataclass, field
import numpy as np

from .seeds import rng_for
from .helmholtz import helmholtz_7pt, grf_velocity
from .acoustic import acoustic_27pt
from .maxwell import yee_curlcurl, block_permittivity
from .rhs import center_source_with_noise, point_sources, random_edge_dipoles


@dataclass
class Problem:
    name: str
    n: int
    rowptr: np.ndarray
    colind: np.ndarray
    values: np.ndarray
    rhs: np.ndarray
    kind: str                 # "grid" or "yee"
    dims: tuple = None        # grid dims (nx, ny, nz) for kind == "grid"
    cells: int = 0            # cells per axis for kind == "yee"
    coords: np.ndarray = None # doubled edge coordinates for kind == "yee"
    meta: dict = field(default_factory=dict)
    opts: dict = field(default_factory=dict)


CONFIGS = {
    # 24^3, delta 0.05, leaves <= 512, compress separators >= 256, tol 1e-3, c128, 1 RHS
    "helmholtz24": dict(kind="grid", n=24, delta=0.05, nrhs=1, rhs="center_noise",
                        n_min=256, tol=1e-3, precision="c128", samples=64),
    # 100^3, delta 0.02, compress >= 1024, 64 probes per block, c64 bulk, 8 RHS; separators bisected
    # down to 128 nodes (the HOD-BF leaf size, a tuning parameter: 128 measured faster than 64)
    "helmholtz100": dict(kind="grid", n=100, delta=0.02, nrhs=8, rhs="points",
                         n_min=1024, tol=1e-3, precision="c64", samples=64, sep_leaf=128),
    # 128^3 GRF velocity, batched levels, 32 RHS (damping not stated: 0.02 as above)
    "helmholtz128grf": dict(kind="grid", n=128, delta=0.02, nrhs=32, rhs="points",
                            n_min=1024, tol=1e-3, precision="c64", samples=64, grf=True, sep_leaf=128),
    # 3D Poisson (omega = 0) on the same path: the separator ranks grow far more slowly than at
    # high frequency, the first comparison workload after the Helmholtz runs
    "poisson100": dict(kind="grid", n=100, delta=0.0, nrhs=8, rhs="points", omega=0.0,
                       n_min=1024, tol=1e-3, precision="c64", samples=64),
    # visco-acoustic 27-point stencil, 64^3 nodes including 8 absorbing layers per face, GRF
    # velocity in [1, 2], q = 1e4 (the paper's heterogeneous-media setting), 8 points per
    # wavelength at the slowest velocity, 8 point sources
    "acoustic64": dict(kind="grid", op="acoustic27", n=64, delta=0.0, nrhs=8, rhs="points",
                       n_min=1024, tol=1e-3, precision="c64", samples=64, grf=True, q=1e4, pml=8,
                       sep_leaf=128),
    # Yee curl-curl 64^3 cells, eps on 8^3 blocks in U[1,4], delta 0.03, 16 RHS
    "maxwell64": dict(kind="yee", n=64, delta=0.03, nrhs=16, rhs="dipoles",
                      n_min=1024, tol=1e-3, precision="c64", samples=64, sep_leaf=128),
}


def make_problem(name, n=None, nrhs=None, delta=None, grf=None, config_id=None,
                 omega=None):
    """Build a Problem by config name, optionally overriding the size.

    ``config_id`` selects the seed stream (defaults to the config's own).
    """
    cfg = dict(CONFIGS[name])
    if n is not None:
        cfg["n"] = n
    if nrhs is not None:
        cfg["nrhs"] = nrhs
    if delta is not None:
        cfg["delta"] = delta
    if grf is not None:
        cfg["grf"] = grf
    seed_cfg = name if config_id is None else config_id
    if omega is None:
        omega = cfg.get("omega")
    nn = cfg["n"]
    if cfg["kind"] == "grid":
        dims = (nn, nn, nn)
        c = None
        if cfg.get("grf"):
            c = grf_velocity(dims, rng_for(seed_cfg, "coef"))
        if cfg.get("op") == "acoustic27":
            rowptr, colind, values, meta = acoustic_27pt(dims, c=c, q=cfg["q"], pml=cfg["pml"], omega=omega)
        else:
            rowptr, colind, values, meta = helmholtz_7pt(dims, cfg["delta"], c=c, omega=omega)
        N = nn ** 3
        if cfg["rhs"] == "center_noise":
            b = center_source_with_noise(dims, rng_for(seed_cfg, "rhs"))
        else:
            b = point_sources(N, cfg["nrhs"], rng_for(seed_cfg, "rhs"))
        return Problem(name, N, rowptr, colind, values, np.asfortranarray(b), "grid",
                       dims=dims, meta=meta, opts=cfg)
    eps = block_permittivity(nn, 8, rng_for(seed_cfg, "coef"))
    rowptr, colind, values, meta = yee_curlcurl(nn, cfg["delta"], eps_cells=eps, omega=omega)
    N = rowptr.shape[0] - 1
    b = random_edge_dipoles(N, cfg["nrhs"], rng_for(seed_cfg, "rhs"))
    return Problem(name, N, rowptr, colind, values, np.asfortranarray(b), "yee",
                   cells=nn, coords=meta["coords"], meta=meta, opts=cfg)


def serving_grids():
    """The three resident factorizations of the serving workload."""
    return [48, 64, 80]
