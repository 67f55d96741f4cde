"""Seeded synthetic workloads for the elastic ADER-DG element kernels.

This module holds no arithmetic of the numerical method: it generates meshes
(cube grids split into tetrahedra, jittered, periodic), their face
connectivity (neighbour element, neighbour face, relative orientation),
material parameters and degree-of-freedom arrays.  It is the one module that
both the oracle (test infrastructure) and the product path consume.
"""
from .mesh import (CubeMesh, cube_mesh, random_materials, random_dofs, seed_for,
                   dt_from_mesh)

__all__ = ["CubeMesh", "cube_mesh", "random_materials", "random_dofs", "seed_for", "dt_from_mesh"]
