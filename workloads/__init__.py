"""Seeded synthetic inputs for generalized-sampling problems.

This module is shared by the tests, the oracle-side checks and the product
benchmarks.  It holds NO arithmetic of the method itself (no scaling
functions, no change-of-basis matrix, no transforms): only sampling patterns,
density-compensation weights, phantoms, coefficient vectors and noise.

The paper's own datasets (the brain phantom and its frequency files, the
Table 1 patterns) are not available; these generators stand in for them with
the same shapes and structure:

* ``grid``            -- uniform points eps*(-M/2 .. M/2-1) (the paper's grid helper).
* ``jitter_1d``       -- xi_k = (k + U(-1/4, 1/4)) * spacing.
* ``spiral_2d``       -- interleaved Archimedean spiral, constant arc-length spacing.
* ``jitter_2d``       -- jittered square grid.
* ``voronoi_weights_1d`` / ``voronoi_weights_2d`` -- Voronoi cell measures
  clipped to a bandwidth region (App. B).
* ``ellipse_phantom`` -- random ellipses times a smooth field, and its cell
  averages at scale J as a stand-in for the projection onto V_J.
"""
from .patterns import grid, jitter_1d, spiral_2d, jitter_2d
from .weights import voronoi_weights_1d, voronoi_weights_2d
from .phantom import ellipse_phantom_params, phantom_cell_averages, phantom_cell_averages_torch
from .configs import (config_c1, config_c2, config_c3, config_c4_problem, config_c5_pattern,
                      complex_noise, relative_noise)

__all__ = [
    "grid", "jitter_1d", "spiral_2d", "jitter_2d",
    "voronoi_weights_1d", "voronoi_weights_2d",
    "ellipse_phantom_params", "phantom_cell_averages", "phantom_cell_averages_torch",
    "config_c1", "config_c2", "config_c3", "config_c4_problem", "config_c5_pattern",
    "complex_noise", "relative_noise",
]
