"""Seeded synthetic inputs for spatially-varying image subtraction.

This package produces the *inputs* of the method only: reference star
fields R, second images I that do not depend on the method, coefficient
arrays a, and the basis/spatial-term specifications of the workloads.  It
holds none of the method's arithmetic (no basis function, no spatial term,
no convolution), so the plain CPU oracle and the GPU library can both be
fed from it without sharing any code.
"""

from .configs import WORKLOADS, Workload, n_basis, n_spatial, const_basis_index
from .starfield import (star_field, coefficients, sky_sigma, SKY_LEVEL, poisson_noise,
                        uniform_image, workload_inputs, second_image, render_stars)

__all__ = [
    "WORKLOADS", "Workload", "n_basis", "n_spatial", "const_basis_index",
    "star_field", "coefficients", "sky_sigma", "SKY_LEVEL", "poisson_noise",
    "uniform_image", "workload_inputs", "second_image", "render_stars",
]
