"""Seeded synthetic problem generators.

These build the matrices and right-hand sides that both the CPU oracle and the
HIP library consume.  They hold none of the relaxation or Krylov arithmetic:
only stencil / element assembly and random draws.  Every array is CSR with
int32 row pointers and column indices (sorted, no duplicates, diagonal
present) and float64 values.
"""
from .problems import (  # noqa: F401
    CSR,
    MASTER_SEED,
    rng_streams,
    poisson2d,
    laplace1d,
    laplace3d,
    vardiff3d,
    elasticity_q1,
    convdiff2d,
    convdiff_batch,
    random_sparse,
    make_rhs,
    config_problem,
)
