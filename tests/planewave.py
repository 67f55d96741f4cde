"""Plane-wave workload of the precision study (test infrastructure).

Homogeneous isotropic medium (one draw from the random-material
distribution), periodic unit cube; wave vector k = 2 pi m with m an integer
vector of length closest to n/8 (wavelength about 8 h) in a seeded random
direction.  The state is a superposition of the right-going P wave and the
two S waves along k:
    q(x, t) = sum_w a_w r_w sin(k.x - c_w |k| t),
where r_w is an eigenvector of A_k = sum_j khat_j A^(j) with eigenvalue c_w
(c_p, c_s, c_s), so each term solves q_t + sum_j A^(j) q_xj = 0 (Eq. linearpde).
The amplitudes mix P and S in a U[0,1] proportion.

Initial DOFs and the exact solution at a later time are L2 projections onto
the Dubiner basis of each element, by a collapsed-coordinate rule with N+4
points per direction (the oracle's basis and quadrature), evaluated in FP64
with torch on the device in element chunks.
"""
from __future__ import annotations

import numpy as np

from oracle import elements as oel
from oracle import refmat
from workload import cube_mesh, seed_for


class PlaneWave:
    def __init__(self, n, N, seed_index=3, m=None):
        self.n, self.N = n, N
        seed = seed_for(seed_index)
        self.mesh = cube_mesh(n, seed)
        rng = np.random.Generator(np.random.PCG64(seed + 555))
        rho = rng.uniform(2000.0, 3000.0)
        cp = rng.uniform(4000.0, 6000.0)
        cs = cp / rng.uniform(1.6, 2.0)
        self.material = np.array([rho, cp, cs])
        self.mats = np.tile(self.material, (self.mesh.E, 1))
        # wave vector: integer m closest in length to n/8, random direction
        target = n / 8.0
        best = None
        for _ in range(64):
            u = rng.standard_normal(3)
            u /= np.linalg.norm(u)
            mv = np.rint(target * u)
            if np.any(mv != 0):
                d = abs(np.linalg.norm(mv) - target)
                if best is None or d < best[0]:
                    best = (d, mv)
        self.m = best[1] if m is None else np.asarray(m, dtype=float)
        self.k = 2.0 * np.pi * self.m
        kn = np.linalg.norm(self.k)
        khat = self.k / kn
        _, lam, mu = oel.lame(self.material[None])
        Jac = oel.jacobians(np.array([rho]), lam, mu)[0]            # (3, 9, 9)
        Ak = np.einsum("j,jpq->pq", khat, Jac)
        w, V = np.linalg.eig(Ak)
        w, V = w.real, V.real
        iP = int(np.argmin(np.abs(w - cp)))
        iS = np.argsort(np.abs(w - cs))[:2]
        assert abs(w[iP] - cp) < 1e-6 * cp and np.all(np.abs(w[iS] - cs) < 1e-6 * cs)
        mix = rng.uniform(0.0, 1.0)
        sdir = rng.standard_normal(2)
        sdir /= np.linalg.norm(sdir)
        rP = V[:, iP] / np.max(np.abs(V[:, iP]))
        rS = [V[:, i] / np.max(np.abs(V[:, i])) for i in iS]
        self.modes = [(mix * rP, cp * kn), ((1 - mix) * sdir[0] * rS[0], cs * kn),
                      ((1 - mix) * sdir[1] * rS[1], cs * kn)]
        # check: each mode solves A_k r = c r
        for r, om in self.modes:
            assert np.allclose(Ak @ r, (om / kn) * r, atol=1e-8 * np.abs(r).max() * cp)
        # time step: 0.5 h_min / ((2N+1) c_p), h_min the smallest insphere diameter
        X = self.mesh.X
        e1, e2, e3 = X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]
        vol = np.abs(np.einsum("ei,ei->e", e1, np.cross(e2, e3))) / 6.0
        area = np.zeros(X.shape[0])
        for (a, b, c) in oel.FACE_VERTS:
            area += 0.5 * np.linalg.norm(np.cross(X[:, b] - X[:, a], X[:, c] - X[:, a]), axis=1)
        self.hmin = float(np.min(6.0 * vol / area))
        self.dt = 0.5 * self.hmin / ((2 * N + 1) * cp)
        self.detJ = 6.0 * vol

    def project(self, t, device="cuda:0", chunk=65536):
        """DOFs (E, 9, B) float64 numpy of q(., t): per element and basis
        function, (1/m_l) int phi_l(xi) q(x(xi), t) dxi."""
        import torch
        N, X = self.N, self.mesh.X
        pts, wts = (np.asarray(a, dtype=np.float64) for a in refmat.tet_rule(N + 4))
        phi = np.asarray(refmat.eval_volume_basis(N, pts), dtype=np.float64)   # (B, npts)
        mass = np.asarray(refmat.mass_closed_form(N), dtype=np.float64)
        Wphi = torch.from_numpy((phi * wts[None, :] / mass[:, None]).T.copy()).to(device)   # (npts, B)
        P = torch.from_numpy(pts).to(device)                           # (npts, 3)
        k = torch.from_numpy(self.k).to(device)
        E = X.shape[0]
        B = phi.shape[0]
        out = np.empty((E, 9, B))
        for e0 in range(0, E, chunk):
            e1 = min(E, e0 + chunk)
            Xc = torch.from_numpy(X[e0:e1]).to(device)
            J = torch.stack([Xc[:, 1] - Xc[:, 0], Xc[:, 2] - Xc[:, 0], Xc[:, 3] - Xc[:, 0]], dim=2)   # (c,3,3)
            phase0 = Xc[:, 0] @ k                                       # (c,)
            kJ = torch.einsum("i,cij->cj", k, J)                        # (c,3)  (J^T k)
            theta = phase0[:, None] + kJ @ P.T                           # (c, npts)
            acc = torch.zeros((e1 - e0, 9, B), dtype=torch.float64, device=device)
            for r, om in self.modes:
                ang = theta - om * t
                coef = torch.sin(ang) @ Wphi                            # (c, B)
                acc += torch.from_numpy(r).to(device)[None, :, None] * coef[:, None, :]
            out[e0:e1] = acc.cpu().numpy()
        return out

    def mass_weights(self):
        """(E, 1, B) weights of the mass-weighted L2 norm of DOF differences."""
        mass = np.asarray(refmat.mass_closed_form(self.N), dtype=np.float64)
        return (self.detJ[:, None] * mass[None, :])[:, None, :]


class SubsetRows:
    """Global element ids -> rows of a compact array (for oracle.stages.step_subset,
    which indexes its per-element inputs with global ids)."""

    def __init__(self, rows, ids, E):
        self.rows = rows
        self.loc = np.full(E, -1, dtype=np.int64)
        self.loc[np.asarray(ids)] = np.arange(len(ids))

    def __getitem__(self, idx):
        li = self.loc[np.asarray(idx)]
        assert np.all(li >= 0), "element outside the subset"
        return self.rows[li]
