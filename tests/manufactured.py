"""Manufactured polynomial states for pinning the oracle (test helper).

A state q(x) is a dict {(a, b, c): coeff (P,)} for x^a y^b z^c.  For a
homogeneous medium the exact solution of q_t + sum_j A^(j) q_xj = 0 with a
polynomial initial state of degree N is the finite Taylor series
q(x, t) = sum_m t^m / m! L^m q0 with L = -sum_j A^(j) d/dx_j.
"""
from __future__ import annotations

from math import factorial

import numpy as np

from oracle import refmat


def random_poly(N, P, rng, scales=None):
    q = {}
    for a in range(N + 1):
        for b in range(N + 1 - a):
            for c in range(N + 1 - a - b):
                v = rng.standard_normal(P)
                if scales is not None:
                    v = v * scales
                q[(a, b, c)] = v
    return q


def apply_L(q, Jac):
    """L q = -sum_j A^(j) dq/dx_j for constant Jacobians Jac (3, P, P)."""
    out = {}
    for (a, b, c), v in q.items():
        for j, e in enumerate((a, b, c)):
            if e == 0:
                continue
            key = [a, b, c]
            key[j] -= 1
            key = tuple(key)
            out[key] = out.get(key, 0.0) - e * (Jac[j] @ v)
    return out


def taylor_state(q0, Jac, t, N):
    """sum_{m=0}^{N} t^m/m! L^m q0 (exact for a degree-N polynomial)."""
    total = {k: v.copy() for k, v in q0.items()}
    cur = q0
    for m in range(1, N + 1):
        cur = apply_L(cur, Jac)
        for k, v in cur.items():
            total[k] = total.get(k, 0.0) + (t ** m / factorial(m)) * v
    return total


def evaluate(q, pts, P):
    out = np.zeros((pts.shape[0], P))
    for (a, b, c), v in q.items():
        out += np.outer(pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c, v)
    return out


def project(q, X, N, P, nq=None):
    """L2 projection of q onto the Dubiner basis of every element: (E, P, B)."""
    nq = nq or N + 2
    rp, rw = refmat.tet_rule(nq)
    phi = refmat.eval_volume_basis(N, rp).astype(float)      # (B, nqp)
    mass = refmat.refmats(N).mass
    E = X.shape[0]
    Jm = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    phys = X[:, 0][:, None, :] + np.einsum("eij,qj->eqi", Jm, rp)   # (E, nqp, 3)
    vals = evaluate(q, phys.reshape(-1, 3), P).reshape(E, -1, P)     # (E, nqp, P)
    return np.einsum("bq,q,eqp->epb", phi, rw, vals) / mass[None, None, :]


def seam_free(mesh):
    """Elements none of whose faces crosses the periodic boundary."""
    from workload.mesh import FACE_VERTS
    X = mesh.X
    ok = np.ones(mesh.E, dtype=bool)
    fv = np.array(FACE_VERTS)
    for s in range(4):
        own = X[:, fv[s]]                                   # (E, 3, 3)
        nb = mesh.neigh[:, s]
        oth = X[nb[:, None], fv[mesh.nface[:, s].astype(int)]]            # (E, 3, 3)
        ok &= np.isclose(own.sum(axis=1), oth.sum(axis=1)).all(axis=1)
    return ok
