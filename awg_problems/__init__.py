"""Seeded synthetic inputs (sparse SPD matrices and overlapping subdomains).

This package generates inputs only and holds none of the AWG method's
arithmetic; the oracle tests and the GPU path both draw from it.
"""
from .fem import Problem, fd5_diffusion, q1_diffusion, q1_elasticity  # noqa: F401
from .configs import (Workload, fd5_32, q1_2d, elast3d, diff3d_grf, paper_x0,  # noqa: F401
                      paper_long, by_name)
