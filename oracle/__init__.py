"""FP64 CPU oracle for the differentiable Gaussian rasteriser.

Test infrastructure only (tests, the smoke check and the benchmark's
CPU-baseline leg).  The product path never imports it.
"""
from .oracle import (ALPHA_MAX, ALPHA_MIN, T_MIN, Options, Projection, Result, Targets, bin_view,  # noqa: F401
                     brute_render, build, project_view, quat_to_rot, rect_boundary_margin, run)
