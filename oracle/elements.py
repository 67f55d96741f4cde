"""Oracle per-element static data (test infrastructure).

Implements, in plain numpy FP64:
  * the elastic Jacobians A, B, C of the linear system q_t + A q_x + B q_y +
    C q_z = 0 (Sec. 2, Eq. linearpde) in velocity-stress form with quantity
    order (s_xx, s_yy, s_zz, s_xy, s_yz, s_xz, u, v, w);
  * the star matrices, element-dependent combinations of the Jacobians
    (Sec. 5.1.1): A*^d = sum_j (d xi_d / d x_j) A^(j);
  * the flux-solver matrices A+ and A- that hold the solution of the 1D
    Riemann problem on each face (Sec. 5.1.1, the matrices following Eq.
    seissol:correction_neigh).  Reading: exact Godunov state for two
    isotropic elastic half-spaces, obtained by solving the 9x9 eigenvector
    system of the face-normal problem with numpy.linalg; the face rotation,
    the face-to-volume Jacobian ratio 2|S|/det J and the minus sign of the
    weak form are folded in.
"""
from __future__ import annotations

import numpy as np

FACE_VERTS = ((0, 2, 1), (0, 1, 3), (0, 3, 2), (1, 2, 3))
VOIGT = ((0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2))


def lame(materials):
    rho, cp, cs = materials[..., 0], materials[..., 1], materials[..., 2]
    mu = rho * cs * cs
    lam = rho * cp * cp - 2.0 * mu
    return rho, lam, mu


def jacobians(rho, lam, mu):
    """Returns (..., 3, 9, 9): A, B, C for each material."""
    rho = np.asarray(rho, dtype=float)
    shp = rho.shape
    J = np.zeros(shp + (3, 9, 9))
    lp2m = lam + 2.0 * mu
    ir = 1.0 / rho
    # x
    J[..., 0, 0, 6] = -lp2m; J[..., 0, 1, 6] = -lam; J[..., 0, 2, 6] = -lam
    J[..., 0, 3, 7] = -mu; J[..., 0, 5, 8] = -mu
    J[..., 0, 6, 0] = -ir; J[..., 0, 7, 3] = -ir; J[..., 0, 8, 5] = -ir
    # y
    J[..., 1, 0, 7] = -lam; J[..., 1, 1, 7] = -lp2m; J[..., 1, 2, 7] = -lam
    J[..., 1, 3, 6] = -mu; J[..., 1, 4, 8] = -mu
    J[..., 1, 6, 3] = -ir; J[..., 1, 7, 1] = -ir; J[..., 1, 8, 4] = -ir
    # z
    J[..., 2, 0, 8] = -lam; J[..., 2, 1, 8] = -lam; J[..., 2, 2, 8] = -lp2m
    J[..., 2, 4, 7] = -mu; J[..., 2, 5, 6] = -mu
    J[..., 2, 6, 5] = -ir; J[..., 2, 7, 4] = -ir; J[..., 2, 8, 2] = -ir
    return J


def geometry(X):
    """X (E,4,3) -> (Jmat (E,3,3) with columns x_i - x_0, detJ (E,), G = J^-1)."""
    Jm = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    det = np.linalg.det(Jm)
    G = np.linalg.inv(Jm)
    return Jm, det, G


def star_matrices(X, materials):
    """(E, 3, 9, 9): A*^d = sum_j G[d, j] A^(j)."""
    _, _, G = geometry(X)
    rho, lam, mu = lame(materials)
    Jac = jacobians(rho, lam, mu)                       # (E, 3, 9, 9)
    return np.einsum("edj,ejpq->edpq", G, Jac)


def face_frames(X):
    """Per face: unit normal n, tangents s, t, area |S|.  Shapes (E,4,3), (E,4)."""
    n_list, s_list, area_list = [], [], []
    for (a, b, c) in FACE_VERTS:
        ab = X[:, b] - X[:, a]
        ac = X[:, c] - X[:, a]
        cr = np.cross(ab, ac)
        nrm = np.linalg.norm(cr, axis=1)
        n_list.append(cr / nrm[:, None])
        s_list.append(ab / np.linalg.norm(ab, axis=1)[:, None])
        area_list.append(0.5 * nrm)
    n = np.stack(n_list, axis=1)
    s = np.stack(s_list, axis=1)
    t = np.cross(n, s)
    return n, s, t, np.stack(area_list, axis=1)


def rotation_9x9(Qm):
    """T with T q_face = q_global for the frame matrix Qm = [n s t] (columns):
    velocities v_g = Qm v_f, stresses sigma_g = Qm sigma_f Qm^T (Voigt)."""
    shp = Qm.shape[:-2]
    T = np.zeros(shp + (9, 9))
    for col, (i, j) in enumerate(VOIGT):
        Sf = np.zeros(shp + (3, 3))
        Sf[..., i, j] = 1.0
        Sf[..., j, i] = 1.0
        Sg = Qm @ Sf @ np.swapaxes(Qm, -1, -2)
        for row, (a, b) in enumerate(VOIGT):
            T[..., row, col] = Sg[..., a, b]
    T[..., 6:9, 6:9] = Qm
    return T


def godunov_face_matrices(matL, matR):
    """Face-frame flux matrices (At+, At-) for left material matL and right
    material matR (..., 3) such that the Godunov flux is At+ qL + At- qR."""
    rL, lL, mL = lame(matL)
    rR, lR, mR = lame(matR)
    cpL, csL = matL[..., 1], matL[..., 2]
    cpR, csR = matR[..., 1], matR[..., 2]
    shp = rL.shape
    Rm = np.zeros(shp + (9, 9))

    def p_vec(lam, mu, s, out, col):
        out[..., 0, col] = lam + 2.0 * mu
        out[..., 1, col] = lam
        out[..., 2, col] = lam
        out[..., 6, col] = -s

    p_vec(lL, mL, -cpL, Rm, 0)
    Rm[..., 3, 1] = mL; Rm[..., 7, 1] = csL          # r_S1(-csL)
    Rm[..., 5, 2] = mL; Rm[..., 8, 2] = csL          # r_S2(-csL)
    Rm[..., 1, 3] = 1.0; Rm[..., 2, 4] = 1.0; Rm[..., 4, 5] = 1.0
    p_vec(lR, mR, cpR, Rm, 6)
    Rm[..., 3, 7] = mR; Rm[..., 7, 7] = -csR         # r_S1(+csR)
    Rm[..., 5, 8] = mR; Rm[..., 8, 8] = -csR         # r_S2(+csR)
    Rinv = np.linalg.inv(Rm)
    lamL = np.zeros(shp + (3, 3))
    lamL[..., 0, 0] = -cpL; lamL[..., 1, 1] = -csL; lamL[..., 2, 2] = -csL
    W = Rm[..., :, 0:3] @ lamL @ Rinv[..., 0:3, :]
    AL = jacobians(rL, lL, mL)[..., 0, :, :]
    return AL - W, W


def flux_matrices(X, materials, neigh, neighbour_materials=None):
    """(Aplus, Aminus), each (E, 4, 9, 9), in the form used by the update:
    Q += sum_s Rhat^s (R^s^T I) Aplus^s^T + neighbour analogue with Aminus.
    neighbour_materials (E, 4, 3), if given, replaces materials[neigh].
    Faces with neigh < 0 (no neighbour): A+ uses the element's own material
    on both sides and A- is zero."""
    E = X.shape[0]
    _, det, _ = geometry(X)
    n, s, t, area = face_frames(X)
    Qm = np.stack([n, s, t], axis=3)                     # (E,4,3,3) columns n s t
    T = rotation_9x9(Qm)
    Tinv = rotation_9x9(np.swapaxes(Qm, -1, -2))
    matL = np.broadcast_to(materials[:, None, :], (E, 4, 3))
    if neighbour_materials is None:
        # a face without neighbour (neigh < 0) takes the element's own
        # material on the far side: A+ is then the upwind flux of a
        # homogeneous medium, and A- is zero (no neighbour term)
        nb = np.asarray(neigh)
        matR = np.where((nb >= 0)[..., None], materials[np.where(nb >= 0, nb, 0)], matL)
    else:
        matR = neighbour_materials
    Ap, Am = godunov_face_matrices(matL, matR)
    scale = -(2.0 * area / det[:, None])[..., None, None]
    Aplus = scale * (T @ Ap @ Tinv)
    Aminus = scale * (T @ Am @ Tinv)
    if neighbour_materials is None:
        Aminus[np.asarray(neigh) < 0] = 0.0
    return Aplus, Aminus
