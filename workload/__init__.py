"""Seeded synthetic workloads for the elastic ADER-DG element kernels.

This module holds no arithmetic of the numerical method: it generates meshes
(cube grids split into tetrahedra, jittered, periodic), their face
connectivity (neighbour element, neighbour face, relative orientation),
material parameters and degree-of-freedom arrays, per-element CFL time steps
and their rate-2 cluster labels (inputs of local time stepping).  It is the one module that
both the oracle (test infrastructure) and the product path consume.
"""
from .mesh import (CubeMesh, cube_mesh, random_materials, random_dofs, seed_for,
                   dt_from_mesh, graded_cube_mesh, element_time_steps, rate2_clusters, permute_elements,
                   layered_materials)

__all__ = ["CubeMesh", "cube_mesh", "random_materials", "random_dofs", "seed_for", "dt_from_mesh",
           "graded_cube_mesh", "element_time_steps", "rate2_clusters", "permute_elements", "layered_materials"]
