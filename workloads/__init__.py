"""Seeded synthetic inputs for the square-wall compliance problem.

This package only draws and shapes input data: phase-density fields and
load vectors on a structured nelx x nely grid of unit-square Q4 elements.
It holds none of the solver's arithmetic (no stiffness, no multigrid, no
compliance), so both the HIP path and the CPU oracle take its output as
plain arrays.
"""

from .square_wall import (  # noqa: F401
    Problem,
    cone_filter,
    density_random_cone,
    density_binary_contrast,
    density_gaussian_sum,
    density_near_binary,
    load_top_traction,
    load_point,
    load_left_traction,
    four_load_cases,
    make_problem,
    batched_design,
    batched_designs,
    PHYSICS,
)
