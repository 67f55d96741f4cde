"""Pins of the local-time-stepping oracle (oracle/lts.py) against facts that
do not come from it:

  * one cluster is global time stepping: the oracle's per-tick schedule
    collapses to repeated oracle.stages.step;
  * space-time polynomial solutions of degree N are reproduced exactly with
    three clusters (every receiver integrates its neighbours' exact Taylor
    pieces over its own interval, so any wrong piece, interval or order
    breaks exactness);
  * in a homogeneous periodic medium the Godunov flux is conservative, so the
    element means (the degree-0 coefficients times the element volumes) sum
    to the same total after a cycle, whatever the clusters: a smaller
    neighbour's two pieces must both enter the larger element's flux, and the
    larger neighbour's piece must be split at the right time.
"""
import math

import numpy as np
import pytest

import manufactured as mf
from oracle import elements, lts, refmat, stages
from workload import cube_mesh, dt_from_mesh, random_dofs, random_materials, seed_for


def _normalise(c, neigh):
    c = c.copy()
    while True:
        lim = np.min(c[neigh], axis=1) + 1
        new = np.minimum(c, lim)
        if np.array_equal(new, c):
            return c
        c = new


def _homogeneous(n, seed, relabel=True):
    mesh = cube_mesh(n, seed_for(seed), relabel=relabel)
    mat1 = random_materials(1, 3 + seed)[0]
    mats = np.tile(mat1, (mesh.E, 1))
    star = elements.star_matrices(mesh.X, mats)
    Ap, Am = elements.flux_matrices(mesh.X, mats, mesh.neigh)
    Jac = elements.jacobians(*elements.lame(mat1))
    return mesh, mats, star, Ap, Am, Jac


def test_one_cluster_is_global_time_stepping():
    N = 3
    mesh = cube_mesh(3, seed_for(0), relabel=True)
    mats = random_materials(mesh.E, seed_for(0))
    rm = refmat.refmats(N)
    star = elements.star_matrices(mesh.X, mats)
    Ap, Am = elements.flux_matrices(mesh.X, mats, mesh.neigh)
    dt = dt_from_mesh(mesh, mats)
    Q0 = random_dofs(mesh.E, 9, rm.B, 5)
    args = (star, Ap, Am, mesh.neigh, mesh.nface, mesh.orient)
    ref = Q0
    for _ in range(3):
        ref = stages.step(rm, dt, ref, *args)
    got = lts.run(rm, np.zeros(mesh.E, np.int32), dt, Q0, *args, n_cycles=3)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    # a single cluster of level 1 steps with 2 dt0
    got2 = lts.run(rm, np.ones(mesh.E, np.int32), dt / 2, Q0, *args, n_cycles=1)
    ref2 = stages.step(rm, dt, Q0, *args)
    assert np.max(np.abs(got2 - ref2)) <= 1e-13 * np.max(np.abs(ref2))


@pytest.mark.parametrize("N", [2, 3])
def test_patch_test_three_clusters(N):
    """Clusters by shells around the cube's centre (level 0 inside, level 2
    at the periodic seam), one cycle = 4 ticks: the state after the cycle is
    the projection of the exact space-time polynomial on every element away
    from the seam."""
    mesh, mats, star, Ap, Am, Jac = _homogeneous(6, 2)
    rm = refmat.refmats(N)
    cen = mesh.X.mean(axis=1)
    d = np.max(np.abs(cen - 0.5), axis=1)
    c = np.where(d <= 0.15, 0, np.where(d <= 0.3, 1, 2)).astype(np.int32)
    c = _normalise(c, mesh.neigh)
    ok = mf.seam_free(mesh)
    assert np.all(c[~ok] == 2), "seam elements must take one step per cycle"
    assert np.bincount(c, minlength=3).min() > 40
    dt0 = dt_from_mesh(mesh, mats) / 4
    rng = np.random.default_rng(11 + N)
    q0 = mf.random_poly(N, 9, rng, np.array([1e7] * 6 + [1.0] * 3))
    Q0 = mf.project(q0, mesh.X, N, 9)
    Q1 = lts.run(rm, c, dt0, Q0, star, Ap, Am, mesh.neigh, mesh.nface, mesh.orient, n_cycles=1)
    exact = mf.project(mf.taylor_state(q0, Jac, 4 * dt0, N), mesh.X, N, 9)
    for cl in range(3):
        sel = ok & (c == cl)
        assert sel.sum() > 20
        for p in range(9):
            inc = np.linalg.norm(exact[sel, p] - Q0[sel, p])
            assert np.linalg.norm(Q1[sel, p] - exact[sel, p]) <= 2e-11 * inc, (cl, p)


def test_cluster_means_conserved():
    N = 2
    mesh, mats, star, Ap, Am, Jac = _homogeneous(4, 4)
    rm = refmat.refmats(N)
    rng = np.random.default_rng(3)
    c = _normalise(rng.integers(0, 3, mesh.E).astype(np.int32), mesh.neigh)
    assert len(np.unique(c)) == 3
    dt0 = dt_from_mesh(mesh, mats) / 4
    Q0 = random_dofs(mesh.E, 9, rm.B, 8)
    Q1 = lts.run(rm, c, dt0, Q0, star, Ap, Am, mesh.neigh, mesh.nface, mesh.orient, n_cycles=1)
    X = mesh.X
    vol = np.abs(np.einsum("ei,ei->e", X[:, 1] - X[:, 0], np.cross(X[:, 2] - X[:, 0], X[:, 3] - X[:, 0])))
    before = np.einsum("e,ep->p", vol, Q0[:, :, 0])
    after = np.einsum("e,ep->p", vol, Q1[:, :, 0])
    scale = np.einsum("e,ep->p", vol, np.abs(Q1[:, :, 0] - Q0[:, :, 0]))
    assert np.all(scale > 0)
    assert np.all(np.abs(after - before) <= 1e-12 * scale), (after - before) / scale


def test_piece_integral_closed_form():
    """The integral of a Taylor piece over [lo, hi] against the antiderivative
    of the polynomial written out (one quantity, N = 4)."""
    D = np.arange(1.0, 6.0)[None, :, None, None] * np.ones((1, 5, 1, 1))
    lo, hi = 0.3, 1.1
    poly = np.polynomial.Polynomial([D[0, d, 0, 0] / math.factorial(d) for d in range(5)])
    ref = poly.integ()(hi) - poly.integ()(lo)
    assert abs(lts.piece_integral(D, lo, hi)[0, 0, 0] - ref) <= 1e-14 * abs(ref)
