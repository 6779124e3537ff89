"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package builds matrices and right-hand sides only.  It holds none of the
solver's arithmetic (no Krylov basis, no sketch, no least squares), so both
the CPU oracle and the GPU path may draw their inputs from it.
"""

from .problems import (  # noqa: F401
    CSR,
    cd2d_upwind,
    cd3d_upwind,
    cd2d_central,
    helmholtz2d,
    theta_weighted,
    edge_weighted,
    shifted_diagonal,
    column_scaled,
    log_uniform,
    randn,
    crandn,
    workload,
    describe,
    sequence_system,
    WORKLOADS,
)
