"""Seeded synthetic inputs for CP decompositions.

This package only draws random numbers and assembles synthetic tensors
from known factors (the CP model, Section 2, plus additive Gaussian noise,
Section 6).  It holds no step of the damped Gauss-Newton method and is the
only code shared by the FP64 oracle and the GPU path.
"""
from .synth import (  # noqa: F401
    collinear_factor,
    nu_collinear_factors,
    cp_tensor,
    add_noise,
    random_init,
    Problem,
    small_problem,
    cfg1,
    cfg2,
    cfg3,
    cfg4,
)
