"""Seeded synthetic inputs for the priorconditioned lagged-diffusivity solver.

This package builds problem *inputs* only: piecewise-constant phantoms, the
forward operators' definitions (blur taps, dense source/detector sensitivity
matrices), noisy data and request arrival traces. It holds none of the
solver's arithmetic (no gradients, diffusivities, multigrid or Krylov steps),
so both the FP64 oracle and the HIP path can consume what it produces.

Every draw comes from ``numpy.random.default_rng(seed)`` (PCG64); within one
problem the phantom parameters are drawn first, then the noise.
"""

from .phantoms import rectangles_2d, ellipsoids_3d, boxes_spheres_3d
from .operators import gaussian_taps, ring_geometry, dense_sensitivity, blur_data, dense_data
from .configs import (Problem, make_blur_problem, make_dense_problem, config_c1, config_c2,
                      config_c3, config_c4, config_c5_requests, c5_request, auto_levels,
                      small_dense_case, small_blur_case)

__all__ = [
    "rectangles_2d", "ellipsoids_3d", "boxes_spheres_3d", "gaussian_taps", "ring_geometry",
    "dense_sensitivity", "blur_data", "dense_data", "Problem", "make_blur_problem",
    "make_dense_problem", "config_c1", "config_c2", "config_c3", "config_c4",
    "config_c5_requests", "c5_request", "auto_levels", "small_dense_case", "small_blur_case",
]
