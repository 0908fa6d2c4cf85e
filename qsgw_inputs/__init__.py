"""Seeded synthetic inputs for RI qsGW workloads.

This package holds the input generators shared by the FP64 oracle and the
HIP path.  It performs no step of the qsGW method itself: it only draws
random numbers and shapes them into an RI tensor B^P_{mu nu}, an orthogonal
LCAO matrix C and sorted orbital energies eps.
"""
from .generator import (  # noqa: F401
    CONFIGS,
    COUPLING,
    Problem,
    batch_shapes,
    cfg1_omega_grid,
    make_config,
    make_mo_tensor,
    make_problem,
)
