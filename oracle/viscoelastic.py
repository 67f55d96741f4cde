"""Oracle of the viscoelastic elements (test infrastructure only).

The paper names viscoelastic rheology for SeisSol (Sec. 5.1) without
equations.  Reading (three mechanisms l = 1..3, 27 quantities: the 9
velocity-stress quantities q_e, then the memory variables theta^l, 6 stress
components each):
    d_t q_e + sum_j A^(j) d_j q_e = -sum_l (theta^l, 0 velocities)
    d_t theta^l + sum_j A^(l,j) d_j q_e = -omega_l theta^l
A^(l,j) (6 x 9) is the stress-row block of A^(j) with the Lame parameters
(lambda, mu) replaced by (omega_l Y^lambda_l, omega_l Y^mu_l).  As one system,
d_t q + sum_j A_full^(j) d_j q = E q with A_full^(j) 27 x 27 (non-zero
columns only for q_e) and the source matrix E (27 x 27).  The ADER step is
that of Sec. 5.1.1 with 27 rows and two source terms:
    Eq. seissol:derivative gains + D^d E^T  (D^{d+1}_kp += D^d_kq E_pq),
    the update gains + I E^T,
and no derivative staircase (the source keeps all degrees).  Star matrices
are sum_j G_dj A_full^(j); the flux solvers' memory rows use the same Godunov
state as the elastic rows: in the face frame the elastic solver is
A_n (I - P) for the own trace and A_n P for the neighbour's, P the
projector of the Godunov state's jump; the memory rows are A^(l)_n (I - P) and
A^(l)_n P, rotated as stresses.  The flux solvers act on the 9 elastic trace
columns only.
"""
from __future__ import annotations

from types import SimpleNamespace

import numpy as np

from . import elements, stages

P = 27
NMECH = 3


def memory_parameters(materials, omega, flam, fmu):
    """Y^lambda, Y^mu (E, 3): the element's Lame parameters times the
    per-mechanism factors flam, fmu (3,)."""
    _, lam, mu = elements.lame(materials)
    return lam[:, None] * np.asarray(flam)[None, :], mu[:, None] * np.asarray(fmu)[None, :]


def jacobians(materials, omega, Ylam, Ymu):
    """(E, 3, 27, 27) full Jacobians."""
    rho, lam, mu = elements.lame(materials)
    J9 = elements.jacobians(rho, lam, mu)                       # (E, 3, 9, 9)
    E = materials.shape[0]
    J = np.zeros((E, 3, P, P))
    J[:, :, :9, :9] = J9
    for l in range(NMECH):
        # the stress rows of the elastic Jacobian are linear in (lambda, mu)
        Jm = elements.jacobians(rho, omega[l] * Ylam[:, l], omega[l] * Ymu[:, l])
        J[:, :, 9 + 6 * l:15 + 6 * l, :9] = Jm[:, :, :6, :]
    return J


def source_matrix(omega):
    """E (27, 27): stress rows -sum_l theta^l, memory rows -omega_l theta^l."""
    Es = np.zeros((P, P))
    for l in range(NMECH):
        for i in range(6):
            Es[i, 9 + 6 * l + i] = -1.0
            Es[9 + 6 * l + i, 9 + 6 * l + i] = -omega[l]
    return Es


def star_matrices(X, materials, omega, Ylam, Ymu):
    """(E, 3, 27, 27): sum_j G_dj A_full^(j), G the inverse Jacobian of the
    element map (as for the elastic star matrices)."""
    _, _, G = elements.geometry(X)
    J = jacobians(materials, omega, Ylam, Ymu)
    return np.einsum("edj,ejpq->edpq", G, J)


def flux_matrices(X, materials, omega, Ylam, Ymu, neigh):
    """(Aplus, Aminus), each (E, 4, 27, 27), non-zero columns 0..8."""
    E = X.shape[0]
    _, det, _ = elements.geometry(X)
    n, s, t, area = elements.face_frames(X)
    Qm = np.stack([n, s, t], axis=3)
    T = elements.rotation_9x9(Qm)
    Tinv = elements.rotation_9x9(np.swapaxes(Qm, -1, -2))
    matL = np.broadcast_to(materials[:, None, :], (E, 4, 3))
    nb = np.asarray(neigh)
    matR = np.where((nb >= 0)[..., None], materials[np.where(nb >= 0, nb, 0)], matL)
    At_p, At_m = elements.godunov_face_matrices(matL, matR)     # (E, 4, 9, 9) = A_n (I - P), A_n P
    scale = -(2.0 * area / det[:, None])[..., None, None]
    Ap = np.zeros((E, 4, P, P))
    Am = np.zeros((E, 4, P, P))
    Ap[:, :, :9, :9] = scale * (T @ At_p @ Tinv)
    Am[:, :, :9, :9] = scale * (T @ At_m @ Tinv)
    # the projector of the Godunov state's jump, from the left-going
    # eigenvectors (the same construction as the elastic solver)
    Pm = _jump_projector(matL, matR)                            # (E, 4, 9, 9)
    Tsig = T[..., :6, :6]
    rho, lam, mu = elements.lame(materials)
    for l in range(NMECH):
        Jm = elements.jacobians(rho, omega[l] * Ylam[:, l], omega[l] * Ymu[:, l])[:, 0, :6, :]   # (E, 6, 9)
        Jm = np.broadcast_to(Jm[:, None], (E, 4, 6, 9))
        rows = slice(9 + 6 * l, 15 + 6 * l)
        Ap[:, :, rows, :9] = scale * (Tsig @ (Jm @ (np.eye(9) - Pm)) @ Tinv)
        Am[:, :, rows, :9] = scale * (Tsig @ (Jm @ Pm) @ Tinv)
    Am[nb < 0] = 0.0
    return Ap, Am


def _jump_projector(matL, matR):
    """P (..., 9, 9) with q* = q_L + P (q_R - q_L) the Godunov state on the
    left of the interface (face frame): P = R_left R^-1 restricted to the
    three left-going waves."""
    rL, lL, mL = elements.lame(matL)
    rR, lR, mR = elements.lame(matR)
    cpL, csL = matL[..., 1], matL[..., 2]
    cpR, csR = matR[..., 1], matR[..., 2]
    shp = rL.shape
    Rm = np.zeros(shp + (9, 9))
    Rm[..., 0, 0] = lL + 2 * mL; Rm[..., 1, 0] = lL; Rm[..., 2, 0] = lL; Rm[..., 6, 0] = cpL
    Rm[..., 3, 1] = mL; Rm[..., 7, 1] = csL
    Rm[..., 5, 2] = mL; Rm[..., 8, 2] = csL
    Rm[..., 1, 3] = 1.0; Rm[..., 2, 4] = 1.0; Rm[..., 4, 5] = 1.0
    Rm[..., 0, 6] = lR + 2 * mR; Rm[..., 1, 6] = lR; Rm[..., 2, 6] = lR; Rm[..., 6, 6] = -cpR
    Rm[..., 3, 7] = mR; Rm[..., 7, 7] = -csR
    Rm[..., 5, 8] = mR; Rm[..., 8, 8] = -csR
    return Rm[..., :, 0:3] @ np.linalg.inv(Rm)[..., 0:3, :]


def predictor(rm, star, Esrc, Q):
    """D^0..D^N (E, N+1, 27, B): one step of Eq. seissol:derivative (the
    stage oracle with N = 1) plus the source term D^d E^T, per order."""
    one = SimpleNamespace(N=1, Ktilde=rm.Ktilde)
    D = [np.asarray(Q, dtype=np.float64)]
    for _ in range(rm.N):
        Dd = D[-1]
        D.append(stages.predictor(one, star, Dd)[:, 1] + np.einsum("pq,eqk->epk", Esrc, Dd))
    return np.stack(D, axis=1)


def step(rm, dt, Q, star, Aplus, Aminus, Esrc, neigh, nface, orient, return_parts=False):
    """One global step with the viscoelastic source terms."""
    D = predictor(rm, star, Esrc, Q)
    I = stages.time_integral(rm.N, D, dt)
    dv = stages.volume(rm, star, I)
    dl = stages.local_flux(rm, Aplus, I)
    dn = stages.neighbour_flux(rm, Aminus, I, neigh, nface, orient)
    ds = np.einsum("pq,eqk->epk", Esrc, I)
    Qn = Q + dv + dl + dn + ds
    if return_parts:
        return Qn, dict(D=D, I=I, vol=dv, lf=dl, nf=dn, src=ds)
    return Qn
