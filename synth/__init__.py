"""Seeded synthetic inputs (meshes, particle clouds) shared by the oracle and the GPU path."""
from . import meshes, workload  # noqa: F401
from .workload import (SINGULAR, FEATURE, SURFACE, VOLUME, FIXED, ALL_MOVING,  # noqa: F401
                       Workload, Geometry, cube_workload, sphere_workload, tetra_workload, gear_workload, cylinder_workload,
                       dyadic_lattice_workload, particle_grid, f32)
