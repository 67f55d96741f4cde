"""Shared helpers of the parity tests: input builders and the tolerance metrics.

Two metrics, both required to pass (stage results compared as increments):
  * per quantity p (and per derivative order where there is one),
    err_p = ||X_p - Y_p||_F / ||Y_p||_F over all elements (the paper's
    Frobenius-norm comparison, Sec. 4.9); pass if max_p err_p <= tol;
  * per element e and quantity p, ||X_ep - Y_ep|| / max(||Y_ep||, rms_p)
    with rms_p = ||Y_p||_F / sqrt(E); pass if the maximum over e and p is
    <= tol.  A single wrong element (a tail workgroup, a clamped slot, one
    face/orientation case) cannot hide in the mean; the rms floor keeps
    elements whose own values nearly cancel from dominating.
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


def elem_err(x, y, qaxis=-2):
    """Maximum over elements (axis 0) and quantities of the per-element
    relative error (see the module docstring)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    E = x.shape[0]
    if E == 0:
        return 0.0
    qa = qaxis % x.ndim
    x = np.moveaxis(x, qa, 1).reshape(E, x.shape[qa], -1)
    y = np.moveaxis(y, qa, 1).reshape(E, y.shape[qa], -1)
    rms = np.sqrt(np.sum(y * y, axis=(0, 2)) / E)
    num = np.linalg.norm(x - y, axis=2)
    den = np.maximum(np.linalg.norm(y, axis=2), rms[None, :])
    bad = (den == 0.0) & (num != 0.0)
    if np.any(bad):
        return float("inf")
    with np.errstate(invalid="ignore", divide="ignore"):
        r = np.where(den > 0.0, num / np.where(den > 0.0, den, 1.0), 0.0)
    return float(r.max())


def errors(x, y, qaxis=-2):
    return rel_err(x, y, qaxis), elem_err(x, y, qaxis)


def assert_close(x, y, tol, what="", qaxis=-2):
    """Both metrics at the bar `tol`; prints the measured values."""
    f, m = errors(x, y, qaxis)
    print("  %-40s frobenius %.3e  per-element %.3e  bar %.0e" % (what, f, m, tol), flush=True)
    assert f <= tol, "%s: relative Frobenius error %.3e above %.0e" % (what, f, tol)
    assert m <= tol, "%s: per-element relative error %.3e above %.0e" % (what, m, tol)


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
