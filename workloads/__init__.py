"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package builds the finite-difference diffusion matrices, right-hand sides
and targets that stand in for the paper's PDE workloads (the paper's own
problems -- deal.II elasticity, mixed Raviart-Thomas Poisson and the Florida
collection matrices of Section 6 -- are not available here).  It holds none of
the solver's arithmetic: no ordering, no factorization, no Krylov iteration.
"""
from .grids import (  # noqa: F401
    GridProblem,
    grid_problem,
    grid_coordinates,
    clique_separator,
    batched_problems,
    workload_config,
    WORKLOADS,
)
