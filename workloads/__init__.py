"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module generates problem data only: surface meshes, time grids and
random densities.  It contains none of the boundary-element or fast-multipole
arithmetic, so that the CPU oracle and the GPU path can be fed identical
inputs without sharing any computation.
"""
from .cube import cube_surface_mesh, uniform_time_nodes, densities, CONFIGS, config_problem, batch_sizes

__all__ = ["cube_surface_mesh", "uniform_time_nodes", "densities", "CONFIGS", "config_problem", "batch_sizes"]
