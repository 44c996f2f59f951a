"""Seeded synthetic workloads shared by the oracle, the tests and the benchmark.

This package holds problem *data* only: mesh sizes, species constants, velocity
kinds, boundary tags and seeded random arrays.  It contains none of the
discretisation's arithmetic, so both the CPU oracle and the GPU library can be
fed from it without sharing any code with each other.
"""
from .configs import CONFIGS, Config, get_config, n_boundary_nodes  # noqa: F401
from .seeded import adjoint_params, boundary_data, n_dof_field, random_state, random_vector  # noqa: F401
