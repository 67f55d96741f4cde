"""Pins of the oracle stage loop nests: brute-force index sums, every
association order, exact time derivatives and the exact space-time
polynomial solution (patch test), free stream, linearity."""
from math import exp
from types import SimpleNamespace

import numpy as np
import pytest

import manufactured as mf
from oracle import elements, refmat, stages
from workload import cube_mesh, dt_from_mesh, random_dofs, random_materials, seed_for


def _rand_inputs(N, E, seed, P=9):
    rng = np.random.default_rng(seed)
    rm = refmat.refmats(N)
    B = rm.B
    Q = rng.standard_normal((E, P, B))
    star = rng.standard_normal((E, 3, P, P))
    Ap = rng.standard_normal((E, 4, P, P))
    Am = rng.standard_normal((E, 4, P, P))
    neigh = rng.integers(0, E, (E, 4)).astype(np.int32)
    nface = rng.integers(0, 4, (E, 4)).astype(np.int8)
    orient = rng.integers(0, 3, (E, 4)).astype(np.int8)
    return rm, Q, star, Ap, Am, neigh, nface, orient


@pytest.mark.parametrize("N", [1, 2])
def test_brute_force_index_sums(N):
    """The C loop nests equal the fully expanded multi-index sums."""
    E = 3
    rm, Q, star, Ap, Am, neigh, nface, orient = _rand_inputs(N, E, 11 + N)
    D = stages.predictor(rm, star, Q)
    dt = 0.37
    I = stages.time_integral(N, D, dt)
    vol = stages.volume(rm, star, I)
    lf = stages.local_flux(rm, Ap, I)
    nf = stages.neighbour_flux(rm, Am, I, neigh, nface, orient)
    for e in range(E):
        Dl = [Q[e].tolist()]
        for d in range(N):
            Dl.append(stages.brute_derivative(rm.Ktilde.tolist(), star[e].tolist(), Dl[-1]))
        assert np.allclose(D[e], np.array(Dl), rtol=1e-13, atol=1e-13 * np.abs(D[e]).max())
        Ib = np.array(stages.brute_time_integral(N, np.array(Dl).tolist(), dt))
        assert np.allclose(I[e], Ib, rtol=1e-13, atol=1e-14)
        vb = np.array(stages.brute_volume(rm.Khat.tolist(), star[e].tolist(), I[e].tolist()))
        assert np.allclose(vol[e], vb, rtol=1e-12, atol=1e-13 * np.abs(vb).max())
        lb = sum(np.array(stages.brute_face(rm.Rhat[s].tolist(), None, rm.R[s].tolist(),
                                            I[e].tolist(), Ap[e, s].tolist())) for s in range(4))
        assert np.allclose(lf[e], lb, rtol=1e-12, atol=1e-13 * np.abs(lb).max())
        nb = sum(np.array(stages.brute_face(rm.Rhat[s].tolist(), rm.f[orient[e, s]].tolist(),
                                            rm.R[nface[e, s]].tolist(), I[neigh[e, s]].tolist(),
                                            Am[e, s].tolist())) for s in range(4))
        assert np.allclose(nf[e], nb, rtol=1e-12, atol=1e-13 * np.abs(nb).max())


@pytest.mark.parametrize("N", [3, 5])
def test_all_association_orders_agree(N):
    """Every binary evaluation order of each Einstein term gives the same
    result (up to rounding): the oracle's fixed order is not special."""
    E = 5
    rm, Q, star, Ap, Am, neigh, nface, orient = _rand_inputs(N, E, 20 + N)
    I = Q * 1e-3
    vol = stages.volume(rm, star, I)
    # K (I A^T) vs (K I) A^T
    alt = sum(np.einsum("epq,ekq->epk", star[:, d], np.einsum("kl,eql->ekq", rm.Khat[d], I)) for d in range(3))
    assert np.allclose(vol, alt, rtol=1e-12, atol=1e-13 * np.abs(vol).max())
    D = stages.predictor(rm, star, Q)
    alt = sum(np.einsum("epq,ekq->epk", star[:, d], np.einsum("kl,eql->ekq", rm.Ktilde[d], Q)) for d in range(3))
    assert np.allclose(D[:, 1], alt, rtol=1e-12, atol=1e-13 * np.abs(alt).max())
    nf = stages.neighbour_flux(rm, Am, I, neigh, nface, orient)
    alt = np.zeros_like(nf)
    for e in range(E):
        for s in range(4):
            j, h, nu = nface[e, s], orient[e, s], neigh[e, s]
            RhF = rm.Rhat[s] @ rm.f[h]                         # (Rhat f) first
            RI = rm.R[j].T @ I[nu].T                           # (Bf, P)
            alt[e] += (RhF @ (RI @ Am[e, s].T)).T
    assert np.allclose(nf, alt, rtol=1e-12, atol=1e-13 * np.abs(nf).max())
    lf = stages.local_flux(rm, Ap, I)
    alt = np.zeros_like(lf)
    for e in range(E):
        for s in range(4):
            big = rm.Rhat[s] @ rm.R[s].T                       # B x B first
            alt[e] += Ap[e, s] @ (big @ I[e].T).T
    assert np.allclose(lf, alt, rtol=1e-12, atol=1e-13 * np.abs(lf).max())


def test_time_integral_closed_form():
    """B = P = 1, star = lam: I is the Taylor polynomial of (e^{lam dt}-1)/lam."""
    N = 6
    lam, dt = -2.3, 0.2
    D = np.array([[[[lam ** d]] for d in range(N + 1)]])
    I = stages.time_integral(N, D, dt)
    ref = sum(lam ** d * dt ** (d + 1) / np.prod(np.arange(1, d + 2)) for d in range(N + 1))
    assert I[0, 0, 0] == pytest.approx(ref, rel=1e-15)
    assert I[0, 0, 0] == pytest.approx((exp(lam * dt) - 1) / lam, rel=1e-6)


def _homogeneous_setup(N, n=4, relabel=True, seed=0):
    mesh = cube_mesh(n, seed_for(seed), relabel=relabel)
    mat1 = random_materials(1, 3 + seed)[0]
    mats = np.tile(mat1, (mesh.E, 1))
    star = elements.star_matrices(mesh.X, mats)
    Ap, Am = elements.flux_matrices(mesh.X, mats, mesh.neigh)
    rho, lam, mu = elements.lame(mat1)
    Jac = elements.jacobians(rho, lam, mu)
    return mesh, mats, star, Ap, Am, Jac


@pytest.mark.parametrize("N", [2, 3, 5])
def test_predictor_exact_time_derivatives(N):
    """D^d equals the projection of L^d q0 for a polynomial q0 (T10)."""
    mesh, mats, star, Ap, Am, Jac = _homogeneous_setup(N, n=3)
    rng = np.random.default_rng(N)
    q = mf.random_poly(N, 9, rng, np.array([1e7] * 6 + [1.0] * 3))
    Q0 = mf.project(q, mesh.X, N, 9)
    rm = refmat.refmats(N)
    D = stages.predictor(rm, star, Q0)
    # forward rounding-error scale of the recursion: the same recursion run on
    # absolute values, |Kt| |D| |A*|^T (the conditioning grows with d, since a
    # smooth state has derivatives far below this bound)
    absrm = SimpleNamespace(N=N, Ktilde=np.abs(rm.Ktilde))
    Dabs = stages.predictor(absrm, np.abs(star), np.abs(Q0))
    cur = q
    for d in range(N + 1):
        ref = mf.project(cur, mesh.X, N, 9)
        for p in range(9):
            err = np.linalg.norm(D[:, d, p] - ref[:, p])
            assert err <= 2e-11 * np.linalg.norm(Dabs[:, d, p]) + 1e-12 * np.linalg.norm(ref[:, p])
            assert err <= 1e-6 * np.linalg.norm(ref[:, p])
        cur = mf.apply_L(cur, Jac)
    # a constant state has vanishing first derivative
    Qc = np.zeros_like(Q0)
    Qc[:, :, 0] = 1.0
    assert np.max(np.abs(stages.predictor(refmat.refmats(N), star, Qc)[:, 1])) < 1e-12 * np.abs(star).max()


@pytest.mark.parametrize("N", [2, 3, 5])
def test_patch_test_full_step(N):
    """ADER-DG is exact for space-time polynomials of degree N: one step from
    the projection of q0 gives the projection of q(x, dt) on every element
    away from the periodic seam (T12).  Covers all 12 (j, h) face cases."""
    mesh, mats, star, Ap, Am, Jac = _homogeneous_setup(N)
    rng = np.random.default_rng(1)
    q0 = mf.random_poly(N, 9, rng, np.array([1e7] * 6 + [1.0] * 3))
    dt = dt_from_mesh(mesh, mats)
    Q0 = mf.project(q0, mesh.X, N, 9)
    Q1 = stages.step(refmat.refmats(N), dt, Q0, star, Ap, Am, mesh.neigh, mesh.nface, mesh.orient)
    exact = mf.project(mf.taylor_state(q0, Jac, dt, N), mesh.X, N, 9)
    ok = mf.seam_free(mesh)
    assert ok.sum() > mesh.E // 3
    inner = mesh.neigh[ok]
    assert len({(int(j), int(h)) for j, h in zip(mesh.nface[ok].ravel(), mesh.orient[ok].ravel())}) == 12
    del inner
    for p in range(9):
        inc = np.linalg.norm(exact[ok, p] - Q0[ok, p])
        assert np.linalg.norm(Q1[ok, p] - exact[ok, p]) <= 2e-11 * inc


def test_free_stream():
    """A uniform state in a homogeneous periodic medium stays uniform (T13),
    seam included."""
    N = 3
    mesh, mats, star, Ap, Am, Jac = _homogeneous_setup(N, relabel=True)
    rm = refmat.refmats(N)
    Q = np.zeros((mesh.E, 9, rm.B))
    Q[:, :, 0] = np.array([1e7, -2e7, 3e6, 1e6, 5e6, -4e6, 1.0, -0.5, 0.25])
    Q1, parts = stages.step(rm, 1e-6, Q, star, Ap, Am, mesh.neigh, mesh.nface, mesh.orient, return_parts=True)
    for p in range(9):
        ref = np.abs(parts["lf"][:, p]).max() + np.abs(Q[:, p]).max() * 1e-6
        assert np.abs(Q1[:, p] - Q[:, p]).max() <= 1e-12 * max(ref, 1e-300) + 1e-12 * np.abs(Q[:, p]).max()


def test_linearity():
    N = 3
    mesh = cube_mesh(3, seed_for(0), relabel=True)
    mats = random_materials(mesh.E, seed_for(0))
    rm = refmat.refmats(N)
    star = elements.star_matrices(mesh.X, mats)
    Ap, Am = elements.flux_matrices(mesh.X, mats, mesh.neigh)
    dt = dt_from_mesh(mesh, mats)
    Q1 = random_dofs(mesh.E, 9, rm.B, 1)
    Q2 = random_dofs(mesh.E, 9, rm.B, 2)
    a, b = 0.7, -2.5
    args = (star, Ap, Am, mesh.neigh, mesh.nface, mesh.orient)
    lhs = stages.step(rm, dt, a * Q1 + b * Q2, *args)
    rhs = a * stages.step(rm, dt, Q1, *args) + b * stages.step(rm, dt, Q2, *args)
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-12 * np.abs(rhs).max())


def test_step_subset_matches_full():
    N = 2
    mesh = cube_mesh(3, seed_for(0))
    mats = random_materials(mesh.E, seed_for(0))
    rm = refmat.refmats(N)
    star = elements.star_matrices(mesh.X, mats)
    Ap, Am = elements.flux_matrices(mesh.X, mats, mesh.neigh)
    Q = random_dofs(mesh.E, 9, rm.B, 4)
    full = stages.step(rm, 1e-6, Q, star, Ap, Am, mesh.neigh, mesh.nface, mesh.orient)
    ids = np.array([0, 5, 17, 100])
    sub = stages.step_subset(rm, 1e-6, ids, Q, star, Ap, Am, mesh.neigh, mesh.nface, mesh.orient)
    assert np.array_equal(sub, full[ids])
