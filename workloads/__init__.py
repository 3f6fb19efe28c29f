"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

Only input generation lives here (meshes, Q1 assembly, box hierarchies, random
coefficients and right-hand sides).  None of the RSD method's arithmetic does.
"""
from .problems import (Problem, config_problem, diffusion_fe_map,  # noqa: F401
                       diffusion_problem, elasticity_problem, skew_diffusion_problem,
                       strip_problem, uneven_cuts)
