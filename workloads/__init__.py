"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds only input generation: random coefficient fields, right-hand
sides, observation sets and the 7- and 27-point stencils that turn fields into the
operator handed to the solver.  It contains none of the cyclic-reduction or
hierarchical-matrix arithmetic; those live, independently, in ``oracle/`` (CPU,
test-only) and in ``paper_1701_00182_amd`` (GPU).
"""
from .fields import (  # noqa: F401
    SEEDS, grid_h, gaussian_random_field, lognormal_kappa, rhs_normal,
    divergence_free_velocity, helmholtz_speed, helmholtz_omega,
    observation_cells, observation_noise, fd_directions,
)
from .stencil import (  # noqa: F401
    SLOT_NAMES, diffusion_coef, add_upwind_convection, helmholtz_coef,
    problem, PROBLEMS, slot27, fem_q1_coef, perturbed_q1_coef, helmholtz27_wavenumber,
)
