"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package only builds input data: sparse SPD matrices in CSR form, their
vertex coordinates, partition specifications and right-hand sides.  It holds
none of the solver's arithmetic (no splitting, no factorisation, no sweep), so
that the CPU oracle and the GPU library can both consume it without sharing
any solver code.
"""
from .systems import (  # noqa: F401
    CSR,
    laplace2d_dirichlet,
    lognormal_conductance_2d,
    poisson3d_dirichlet,
    grf_field,
    diffusion_tpfa,
    random_geometric_graph,
    random_rhs,
    block_diag,
    paper_example_32,
)
from .configs import make_config, CONFIG_NAMES  # noqa: F401
