"""Seeded synthetic inputs for the elliptic depth solve.

This package is shared by the oracle, the tests and the benchmark.  It holds
only input generation (random smooth fields on the sphere, time steps, grid
sizes); none of the solver's arithmetic (no operator, no preconditioner, no
Krylov step) lives here, so neither side of a parity test can borrow the
other's numerics through it.
"""
from .fields import (  # noqa: F401
    cell_centres,
    harmonic_field,
    problem,
    batch_problems,
    jet_sequence_depth,
    zonal_flow_state,
    model_state,
    CONFIG_SEED_BASE,
)
