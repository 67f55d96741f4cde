"""Pins of the viscoelastic oracle (oracle/viscoelastic.py):

  * the factorisation the memory-row flux rests on: the elastic face solvers
    are A_n (I - P) and A_n P with P the jump projector built here;
  * memory rows whose Jacobian equals the stress rows' (omega Y = lambda, mu)
    get flux rows equal to the stress rows of the flux solvers;
  * omega = 0 and Y = 0 reduce the step to the elastic step (memory
    variables stay zero), through all 27 rows;
  * a spatially constant state in a homogeneous periodic medium advances by
    the degree-(N+1) Taylor polynomial of exp(dt E), computed here by matrix
    powers, and stays within the truncation bound of scipy's expm.
"""
import math

import numpy as np
import pytest
from scipy.linalg import expm

from oracle import elements, refmat, stages
from oracle import viscoelastic as ve
from workload import cube_mesh, dt_from_mesh, random_dofs, random_materials, seed_for


def test_elastic_solvers_factor_through_the_jump_projector():
    mats = random_materials(8, seed_for(3))
    matL = np.broadcast_to(mats[:4, None, :], (4, 4, 3))
    matR = np.broadcast_to(mats[4:, None, :], (4, 4, 3))
    Ap, Am = elements.godunov_face_matrices(matL, matR)
    rho, lam, mu = elements.lame(matL)
    AL = elements.jacobians(rho, lam, mu)[..., 0, :, :]
    Pm = ve._jump_projector(matL, matR)
    assert np.allclose(Am, AL @ Pm, rtol=0, atol=1e-10 * np.abs(AL).max())
    assert np.allclose(Ap, AL @ (np.eye(9) - Pm), rtol=0, atol=1e-10 * np.abs(AL).max())


def test_memory_rows_equal_stress_rows_when_jacobians_match():
    mesh = cube_mesh(3, seed_for(1), relabel=True)
    mats = random_materials(mesh.E, seed_for(1))
    omega = np.array([0.5, 2.0, 7.0])
    _, lam, mu = elements.lame(mats)
    Ylam = np.stack([lam / w for w in omega], axis=1)
    Ymu = np.stack([mu / w for w in omega], axis=1)
    Ap, Am = ve.flux_matrices(mesh.X, mats, omega, Ylam, Ymu, mesh.neigh)
    Ap9, Am9 = elements.flux_matrices(mesh.X, mats, mesh.neigh)
    sc = np.abs(Ap9).max()
    assert np.allclose(Ap[:, :, :9, :9], Ap9, rtol=0, atol=1e-12 * sc)
    for l in range(3):
        rows = slice(9 + 6 * l, 15 + 6 * l)
        assert np.allclose(Ap[:, :, rows, :9], Ap9[:, :, :6, :], rtol=0, atol=1e-10 * sc)
        assert np.allclose(Am[:, :, rows, :9], Am9[:, :, :6, :], rtol=0, atol=1e-10 * sc)
    assert np.all(Ap[..., 9:] == 0) and np.all(Am[..., 9:] == 0)


@pytest.mark.parametrize("N", [2, 4])
def test_zero_memory_reduces_to_elastic(N):
    mesh = cube_mesh(3, seed_for(2), relabel=True)
    mats = random_materials(mesh.E, seed_for(2))
    rm = refmat.refmats(N)
    zero = np.zeros(3)
    Yz = np.zeros((mesh.E, 3))
    star = ve.star_matrices(mesh.X, mats, zero, Yz, Yz)
    Ap, Am = ve.flux_matrices(mesh.X, mats, zero, Yz, Yz, mesh.neigh)
    Es = ve.source_matrix(zero)
    dt = dt_from_mesh(mesh, mats)
    Q = np.zeros((mesh.E, 27, rm.B))
    Q[:, :9] = random_dofs(mesh.E, 9, rm.B, 6)
    got = ve.step(rm, dt, Q, star, Ap, Am, Es, mesh.neigh, mesh.nface, mesh.orient)
    s9 = elements.star_matrices(mesh.X, mats)
    Ap9, Am9 = elements.flux_matrices(mesh.X, mats, mesh.neigh)
    ref = stages.step(rm, dt, Q[:, :9], s9, Ap9, Am9, mesh.neigh, mesh.nface, mesh.orient)
    assert np.max(np.abs(got[:, :9] - ref)) <= 1e-12 * np.max(np.abs(ref))
    # the memory rows stay zero except for the source's coupling to stress (none: theta = 0)
    assert np.max(np.abs(got[:, 9:])) <= 1e-14 * np.max(np.abs(ref))


@pytest.mark.parametrize("N", [2, 3, 5])
def test_constant_state_follows_truncated_exponential(N):
    mesh = cube_mesh(3, seed_for(4), relabel=True)
    mat1 = random_materials(1, seed_for(4))[0]
    mats = np.tile(mat1, (mesh.E, 1))
    rm = refmat.refmats(N)
    omega = np.array([1.0e3, 4.0e4, 2.0e5])           # dt omega up to about 0.2 below
    Ylam, Ymu = ve.memory_parameters(mats, omega, [0.02, 0.01, 0.04], [0.03, 0.015, 0.005])
    star = ve.star_matrices(mesh.X, mats, omega, Ylam, Ymu)
    Ap, Am = ve.flux_matrices(mesh.X, mats, omega, Ylam, Ymu, mesh.neigh)
    Es = ve.source_matrix(omega)
    dt = dt_from_mesh(mesh, mats)
    assert 0.05 < dt * omega.max() < 1.0
    rng = np.random.default_rng(N)
    q0 = rng.standard_normal(27) * np.r_[np.full(6, 1e7), np.ones(3), np.full(18, 1e6)]
    Q = np.zeros((mesh.E, 27, rm.B))
    Q[:, :, 0] = q0
    got = ve.step(rm, dt, Q, star, Ap, Am, Es, mesh.neigh, mesh.nface, mesh.orient)
    # the truncated Taylor polynomial by repeated matrix products
    term, ref = q0.copy(), q0.copy()
    for k in range(1, N + 2):
        term = dt * (Es @ term) / k
        ref = ref + term
    # relative to the increment, with a rounding floor at the state's scale
    # (the free-stream flux terms of size |q0| cancel to rounding)
    inc = np.abs(ref - q0)
    for e in (0, mesh.E // 2, mesh.E - 1):
        assert np.all(np.abs(got[e, :, 0] - ref) <= 1e-9 * inc + 1e-14 * np.max(np.abs(q0)))
    assert np.max(np.abs(got[:, :, 1:])) <= 1e-9 * np.max(np.abs(q0))
    # within the truncation bound of the exponential
    ex = expm(dt * Es) @ q0
    bound = (dt * np.linalg.norm(Es, 2)) ** (N + 2) / math.factorial(N + 2) * np.linalg.norm(q0) * 1.5
    assert np.linalg.norm(ref - ex) <= bound


@pytest.mark.parametrize("N", [3, 5])
def test_constant_state_closed_form(N):
    """Against the exact solution of the reading's ODE for a constant state,
    written without the source matrix: theta_l(t) = theta_l e^{-omega_l t},
    sigma(t) = sigma_0 - sum_l theta_l (1 - e^{-omega_l t}) / omega_l,
    velocities constant; within the ADER truncation (omega dt)^{N+2}/(N+2)!."""
    mesh = cube_mesh(3, seed_for(5), relabel=True)
    mat1 = random_materials(1, seed_for(5))[0]
    mats = np.tile(mat1, (mesh.E, 1))
    rm = refmat.refmats(N)
    omega = np.array([3.0e3, 5.0e4, 1.5e5])
    Ylam, Ymu = ve.memory_parameters(mats, omega, [0.02, 0.01, 0.04], [0.03, 0.015, 0.005])
    star = ve.star_matrices(mesh.X, mats, omega, Ylam, Ymu)
    Ap, Am = ve.flux_matrices(mesh.X, mats, omega, Ylam, Ymu, mesh.neigh)
    dt = dt_from_mesh(mesh, mats)
    rng = np.random.default_rng(10 + N)
    sig0, vel0 = rng.standard_normal(6) * 1e7, rng.standard_normal(3)
    th0 = rng.standard_normal((3, 6)) * 1e6
    Q = np.zeros((mesh.E, 27, rm.B))
    Q[:, :, 0] = np.concatenate([sig0, vel0, th0.ravel()])
    got = ve.step(rm, dt, Q, star, Ap, Am, ve.source_matrix(omega), mesh.neigh, mesh.nface, mesh.orient)[0, :, 0]
    decay = np.exp(-omega * dt)
    th_ref = th0 * decay[:, None]
    sig_ref = sig0 - np.sum(th0 * ((1.0 - decay) / omega)[:, None], axis=0)
    trunc = (omega.max() * dt) ** (N + 2) / math.factorial(N + 2)
    assert np.all(np.abs(got[9:].reshape(3, 6) - th_ref) <= 2 * trunc * np.abs(th0) + 1e-12 * np.abs(th0))
    # the first omitted term of sigma's series: theta/omega (omega dt)^{N+2}/(N+2)!
    sig_tr = np.sum(np.abs(th0) / omega[:, None] * ((omega * dt) ** (N + 2) / math.factorial(N + 2))[:, None], axis=0)
    assert np.all(np.abs(got[:6] - sig_ref) <= 2 * sig_tr + 1e-14 * np.abs(sig0).max())
    assert np.all(np.abs(got[6:9] - vel0) <= 1e-9 * np.abs(vel0))
