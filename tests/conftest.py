import functools
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")


@functools.lru_cache(maxsize=None)
def cached_problem(kind, *args):
    from workloads import (config_problem, diffusion_problem, elasticity_problem,
                           skew_diffusion_problem, strip_problem)
    if kind == "config":
        return config_problem(*args)
    if kind == "diffusion":
        return diffusion_problem(*args)
    if kind == "strip":
        return strip_problem(*args)
    if kind == "skew":
        return skew_diffusion_problem(*args)
    if kind == "diffusion_binary":           # one cut axis per depth (deeper trees)
        return diffusion_problem(*args, tree="binary")
    if kind == "skew_binary":
        return skew_diffusion_problem(*args, tree="binary")
    if kind == "elasticity":
        return elasticity_problem(*args)
    raise KeyError(kind)


@pytest.fixture(scope="session")
def problem_cache():
    return cached_problem
