"""Seeded synthetic workloads shared by the oracle, the tests and the benchmark (inputs only)."""
from .stencils import Problem, cd1d, cd2d, cd3d, gaussian_rhs, make_problem  # noqa: F401
from . import configs  # noqa: F401
