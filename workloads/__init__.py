"""Seeded synthetic inputs for the butterfly-compressed multifrontal solver.

This package only builds problem data: sparse operators in CSR form, velocity
and permittivity fields, right-hand sides and request streams.  It contains no
step of the solver itself, so both the CPU oracle and the GPU path can draw
their inputs from it without sharing any solver arithmetic.
"""
from .seeds import rng_for, CONFIG_IDS, PURPOSE_IDS
from .helmholtz import helmholtz_7pt, omega_for_ppw, grf_velocity
from .maxwell import yee_curlcurl
from .acoustic import acoustic_27pt
from .rhs import point_sources, center_source_with_noise, random_edge_dipoles, request_stream
from .configs import CONFIGS, make_problem
from .factors import random_butterfly, halving_bounds

__all__ = [
    "rng_for", "CONFIG_IDS", "PURPOSE_IDS",
    "helmholtz_7pt", "omega_for_ppw", "grf_velocity", "yee_curlcurl", "acoustic_27pt",
    "point_sources", "center_source_with_noise", "random_edge_dipoles", "request_stream",
    "CONFIGS", "make_problem", "random_butterfly", "halving_bounds",
]
