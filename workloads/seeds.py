"""Seed derivation shared by every generator.

Every random draw comes from ``numpy.random.default_rng`` seeded with a
``SeedSequence([200700202, config_id, purpose_id])`` so that a workload is
reproducible from its config name and the purpose of the draw alone.
"""
import numpy as np

BASE_SEED = 200700202

CONFIG_IDS = {
    "helmholtz24": 1,     # 24^3 plain method, complex128
    "helmholtz100": 2,    # 100^3, complex64 bulk
    "helmholtz128grf": 3, # 128^3 heterogeneous velocity, batched levels
    "maxwell64": 4,       # Yee curl-curl on 64^3 cells
    "serving": 5,         # three resident factorizations
    "poisson100": 6,      # 3D Poisson, omega = 0
    "acoustic64": 7,      # 27-point visco-acoustic stencil with absorbing layers
    "test": 99,           # small grids used by the test-suite
}

PURPOSE_IDS = {"coef": 0, "rhs": 1, "arrivals": 2, "probe": 3, "manufactured": 4, "factors": 5}


def rng_for(config, purpose, extra=()):
    """Generator for (config, purpose[, extra ints])."""
    cid = CONFIG_IDS[config] if isinstance(config, str) else int(config)
    pid = PURPOSE_IDS[purpose] if isinstance(purpose, str) else int(purpose)
    return np.random.default_rng(np.random.SeedSequence([BASE_SEED, cid, pid, *map(int, extra)]))
