"""Pins of the oracle's star and flux-solver matrices (homogeneous upwind
splitting, eigen-signs, Godunov interface conditions, rotation covariance)."""
import numpy as np
import pytest

from oracle import elements
from workload import cube_mesh, random_materials, seed_for


def _mats(n, seed):
    return random_materials(n, seed)


def test_rotation_and_normal_jacobian():
    mesh = cube_mesh(3, seed_for(1), relabel=True)
    mats = _mats(mesh.E, 1)
    n, s, t, area = elements.face_frames(mesh.X)
    Qm = np.stack([n, s, t], axis=3)
    assert np.allclose(np.swapaxes(Qm, -1, -2) @ Qm, np.eye(3), atol=1e-14)
    T = elements.rotation_9x9(Qm)
    Ti = elements.rotation_9x9(np.swapaxes(Qm, -1, -2))
    assert np.allclose(T @ Ti, np.eye(9), atol=1e-13)
    rho, lam, mu = elements.lame(mats)
    Jac = elements.jacobians(rho, lam, mu)                 # (E, 3, 9, 9)
    # rotational invariance: sum_j n_j A^(j) = T A_x T^-1
    An = np.einsum("esj,ejpq->espq", n, Jac)
    Ax = np.broadcast_to(Jac[:, None, 0], An.shape)
    assert np.allclose(An, T @ Ax @ Ti, rtol=1e-12, atol=1e-12 * np.abs(An).max())


def test_star_is_chain_rule():
    mesh = cube_mesh(3, seed_for(2))
    mats = _mats(mesh.E, 2)
    star = elements.star_matrices(mesh.X, mats)
    Jm, det, G = elements.geometry(mesh.X)
    assert np.all(det > 0)
    rho, lam, mu = elements.lame(mats)
    Jac = elements.jacobians(rho, lam, mu)
    # sum_d star^d J_dj... : star^d = sum_j G_dj A^(j)  <=>  sum_d Jm_jd star^d = A^(j)
    back = np.einsum("ejd,edpq->ejpq", Jm, star)
    assert np.allclose(back, Jac, rtol=1e-10, atol=1e-9 * np.abs(Jac).max())
    assert np.all(np.count_nonzero(np.abs(star) > 0, axis=(2, 3)) <= 24)


def test_homogeneous_upwind_split():
    mats = _mats(20, 3)
    Ap, Am = elements.godunov_face_matrices(mats, mats)
    rho, lam, mu = elements.lame(mats)
    Ax = elements.jacobians(rho, lam, mu)[:, 0]
    assert np.allclose(Ap + Am, Ax, atol=1e-9 * np.abs(Ax).max())
    for e in range(20):
        ev_p = np.linalg.eigvals(Ap[e]).real
        ev_m = np.linalg.eigvals(Am[e]).real
        scale = mats[e, 1]
        assert ev_p.min() > -1e-9 * scale and ev_m.max() < 1e-9 * scale
        cp, cs = mats[e, 1], mats[e, 2]
        assert np.allclose(np.sort(ev_p), np.sort([0] * 6 + [cs, cs, cp]), atol=1e-6 * cp)


def _godunov_interface_state(F, mat):
    """Traction (s_xx, s_xy, s_xz) and velocity (u, v, w) of the Godunov state
    q* from the flux F = A_x(mat) q* (rows 6..8 give -traction/rho, rows 0, 3,
    5 give -(lambda+2mu) u, -mu v, -mu w)."""
    rho, lam, mu = elements.lame(mat)
    trac = -F[:, 6:9] * rho[:, None]
    vel = np.stack([-F[:, 0] / (lam + 2 * mu), -F[:, 3] / mu, -F[:, 5] / mu], axis=1)
    return trac, vel


def test_heterogeneous_godunov_conditions():
    """Exact Riemann solution between two materials: the interface state seen
    from the left and from the right (mirror problem x -> -x) has the same
    traction and the same velocity; equal states give the physical flux."""
    rng = np.random.default_rng(4)
    mL = _mats(30, 5)
    mR = _mats(30, 6)
    Ap, Am = elements.godunov_face_matrices(mL, mR)
    rho, lam, mu = elements.lame(mL)
    AL = elements.jacobians(rho, lam, mu)[:, 0]
    sc = np.array([1e7] * 6 + [1.0] * 3)
    q = rng.standard_normal((30, 9)) * sc
    F = np.einsum("epq,eq->ep", Ap + Am, q)
    assert np.allclose(F, np.einsum("epq,eq->ep", AL, q), rtol=1e-9, atol=1e-9 * np.abs(F).max())
    qL = rng.standard_normal((30, 9)) * sc
    qR = rng.standard_normal((30, 9)) * sc
    F = np.einsum("epq,eq->ep", Ap, qL) + np.einsum("epq,eq->ep", Am, qR)
    flip = np.diag([1, 1, 1, -1, 1, -1, -1, 1, 1.0])
    Apr, Amr = elements.godunov_face_matrices(mR, mL)
    Fm = np.einsum("epq,eq->ep", Apr, qR @ flip) + np.einsum("epq,eq->ep", Amr, qL @ flip)
    tL, vL = _godunov_interface_state(F, mL)
    tR, vR = _godunov_interface_state(Fm, mR)
    tR = tR * np.array([1, -1, -1.0])
    vR = vR * np.array([-1, 1, 1.0])
    assert np.allclose(tL, tR, rtol=1e-9, atol=1e-9 * np.abs(tL).max())
    assert np.allclose(vL, vR, rtol=1e-9, atol=1e-9 * np.abs(vL).max())
    # the interface state differs from both input states (non-trivial problem)
    assert not np.allclose(vL, qL[:, 6:9])


def test_flux_matrices_scaling_sign():
    mesh = cube_mesh(3, seed_for(3), relabel=True)
    mats = np.tile(_mats(1, 7), (mesh.E, 1))
    Aplus, Aminus = elements.flux_matrices(mesh.X, mats, mesh.neigh)
    n, s, t, area = elements.face_frames(mesh.X)
    _, det, _ = elements.geometry(mesh.X)
    rho, lam, mu = elements.lame(mats)
    Jac = elements.jacobians(rho, lam, mu)
    An = np.einsum("esj,ejpq->espq", n, Jac)
    scale = -(2.0 * area / det[:, None])[..., None, None]
    assert np.allclose(Aplus + Aminus, scale * An, rtol=1e-10, atol=1e-10 * np.abs(scale * An).max())


def test_face_without_neighbour_uses_own_material():
    """A face with neigh = -1 takes the element's own material on the far
    side: its A+ equals the homogeneous upwind flux, whose sum with the
    matching A- is the (scaled) normal Jacobian; its A- is zero; other faces
    are unchanged."""
    mesh = cube_mesh(3, seed_for(4), relabel=True)
    mats = _mats(mesh.E, 4)
    nb = mesh.neigh.copy()
    nb[0, 2] = -1
    nb[5, 0] = -1
    Ap, Am = elements.flux_matrices(mesh.X, mats, nb)
    Ap0, Am0 = elements.flux_matrices(mesh.X, mats, mesh.neigh)
    own = np.broadcast_to(mats[:, None, :], (mesh.E, 4, 3))
    Ap_h, Am_h = elements.flux_matrices(mesh.X, mats, None, neighbour_materials=own)
    _, det, _ = elements.geometry(mesh.X)
    n, _, _, area = elements.face_frames(mesh.X)
    rho, lam, mu = elements.lame(mats)
    An = np.einsum("esj,ejpq->espq", n, elements.jacobians(rho, lam, mu))
    for e, f in ((0, 2), (5, 0)):
        assert np.all(Am[e, f] == 0.0)
        assert np.array_equal(Ap[e, f], Ap_h[e, f])
        ref = -(2.0 * area[e, f] / det[e]) * An[e, f]
        assert np.allclose(Ap_h[e, f] + Am_h[e, f], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    mask = nb >= 0
    assert np.array_equal(Ap[mask], Ap0[mask]) and np.array_equal(Am[mask], Am0[mask])
