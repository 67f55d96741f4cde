"""Shared helpers of the parity tests: input builders and the tolerance metric.

Metric (per quantity p, and per derivative order where there is one):
err_p = ||X_p - Y_p||_F / ||Y_p||_F over all elements; a result passes if
max_p err_p <= tol.  Stage results are compared as increments.
"""
from __future__ import annotations

import numpy as np

from oracle import elements as oelements
from oracle import refmat
from workload import cube_mesh, random_dofs, random_materials, seed_for, dt_from_mesh

STAR_PATTERN = np.zeros((9, 9), dtype=bool)
for p, qs in enumerate([(6, 7, 8)] * 3 + [(6, 7), (7, 8), (6, 8), (0, 3, 5), (1, 3, 4), (2, 4, 5)]):
    STAR_PATTERN[p, list(qs)] = True


def rel_err(x, y, qaxis=-2):
    """max over quantities (and leading per-slice axes in `keep`) of the
    relative Frobenius error."""
    x = np.moveaxis(np.asarray(x, dtype=np.float64), qaxis, 0)
    y = np.moveaxis(np.asarray(y, dtype=np.float64), qaxis, 0)
    worst = 0.0
    for p in range(x.shape[0]):
        den = np.linalg.norm(y[p])
        num = np.linalg.norm(x[p] - y[p])
        if den == 0.0:
            if num != 0.0:
                return float("inf")
            continue
        worst = max(worst, num / den)
    return worst


def random_stage_inputs(N, E, seed, P=9):
    """Random inputs shaped like the paper's performance reproducer: random
    DOFs, random neighbour relations (all 12 face/orientation cases), star
    matrices with the elastic sparsity pattern, dense flux solvers."""
    rng = np.random.default_rng(seed)
    B = refmat.n_basis(N)
    Q = rng.standard_normal((E, P, B))
    I = rng.standard_normal((E, P, B))
    star = rng.standard_normal((E, 3, P, P)) * STAR_PATTERN[None, None]
    Ap = rng.standard_normal((E, 4, P, P))
    Am = rng.standard_normal((E, 4, P, P))
    neigh = rng.integers(0, E, (E, 4)).astype(np.int32)
    nface = rng.integers(0, 4, (E, 4)).astype(np.int8)
    orient = rng.integers(0, 3, (E, 4)).astype(np.int8)
    return dict(Q=Q, I=I, star=star, Ap=Ap, Am=Am, neigh=neigh, nface=nface, orient=orient,
                face_rot=(nface.astype(np.uint8) | (orient.astype(np.uint8) << 2)))


def mesh_inputs(n, N, seed_index=0, relabel=False):
    """A jittered periodic cube-split mesh with random materials and N(0,1)
    DOFs (the recipe of the single-mesh workloads)."""
    seed = seed_for(seed_index)
    mesh = cube_mesh(n, seed, relabel=relabel)
    mats = random_materials(mesh.E, seed)
    Q = random_dofs(mesh.E, 9, refmat.n_basis(N), seed)
    dt = dt_from_mesh(mesh, mats)
    return mesh, mats, Q, dt


def oracle_element_data(mesh, mats):
    star = oelements.star_matrices(mesh.X, mats)
    Ap, Am = oelements.flux_matrices(mesh.X, mats, mesh.neigh)
    return star, Ap, Am


def oracle_element_data_subset(mesh, mats, ids):
    """Oracle star matrices for `ids` and their neighbours and flux solvers for
    `ids`, scattered into full-size arrays (other rows zero)."""
    E = mesh.E
    nb = mesh.neigh[ids]
    allids = np.unique(np.concatenate([ids, nb.ravel()]))
    star = np.zeros((E, 3, 9, 9))
    star[allids] = oelements.star_matrices(mesh.X[allids], mats[allids])
    ap, am = oelements.flux_matrices(mesh.X[ids], mats[ids], None, neighbour_materials=mats[nb])
    Ap = np.zeros((E, 4, 9, 9))
    Am = np.zeros((E, 4, 9, 9))
    Ap[ids] = ap
    Am[ids] = am
    return star, Ap, Am
