"""Pins of the oracle's reference matrices against closed forms, identities and
the sparsity facts stated in the paper (Sec. 5.1: B = C(N+3,3), B~ = C(N+2,2),
derivative staircase C(N-d+3,3))."""
import json
import os
from math import comb, factorial, gamma

import numpy as np
import pytest

from oracle import refmat
from workload import cube_mesh, seed_for
from workload.mesh import FACE_VERTS

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_jacobi_closed_forms():
    x = np.linspace(-1, 1, 7)
    for a in (0, 1, 2, 5):
        assert np.allclose(refmat.jacobi_eval(1, a, 0, x), ((a + 2) * x + a) / 2, atol=1e-15)
        for n in range(8):
            assert refmat.jacobi_eval(n, a, 0, 1.0) == pytest.approx(comb(n + a, n), rel=1e-13)
            # P_n^(a,0)(-1) = (-1)^n
            assert refmat.jacobi_eval(n, a, 0, -1.0) == pytest.approx((-1) ** n, abs=1e-12)
    # norm 2^{a+1}/(2n+a+1) and orthogonality under (1-x)^a
    for a in (0, 1, 2, 4):
        xq, wq = refmat.gauss_jacobi(12, a)
        for n in range(7):
            for m in range(7):
                v = np.sum(wq * refmat.jacobi_eval(n, a, 0, xq) * refmat.jacobi_eval(m, a, 0, xq))
                ref = 2.0 ** (a + 1) / (2 * n + a + 1) if n == m else 0.0
                assert v == pytest.approx(ref, abs=1e-13)


@pytest.mark.parametrize("a", [0, 1, 2, 3])
@pytest.mark.parametrize("nq", [1, 3, 6])
def test_gauss_jacobi_exactness(a, nq):
    x, w = refmat.gauss_jacobi(nq, a)
    for m in range(2 * nq):
        beta = 2.0 ** (a + m + 1) * gamma(a + 1) * gamma(m + 1) / gamma(a + m + 2)
        assert np.sum(w * (1 + x) ** m) == pytest.approx(beta, rel=1e-13)


def test_simplex_rules_exact():
    p, w = refmat.tet_rule(5)
    assert w.sum() == pytest.approx(1 / 6, rel=1e-14)
    for a in range(5):
        for b in range(5 - a):
            for c in range(5 - a - b):
                exact = factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 3)
                v = np.sum(w * p[:, 0] ** a * p[:, 1] ** b * p[:, 2] ** c)
                assert v == pytest.approx(exact, rel=1e-12)
    p, w = refmat.tri_rule(5)
    assert w.sum() == pytest.approx(0.5, rel=1e-14)
    for a in range(8):
        for b in range(8 - a):
            exact = factorial(a) * factorial(b) / factorial(a + b + 2)
            assert np.sum(w * p[:, 0] ** a * p[:, 1] ** b) == pytest.approx(exact, rel=1e-12)


def test_sizes_match_paper_golden():
    with open(os.path.join(GOLDEN, "paper_sizes.json")) as fh:
        g = json.load(fh)
    for row in g["rows"]:
        N = row["N"]
        assert refmat.n_basis(N) == row["B"]
        assert refmat.n_face_basis(N) == row["Bf"]


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6])
def test_mass_closed_form_and_orthogonality(N):
    rm = refmat.refmats(N)
    assert np.allclose(rm.mass, refmat.mass_closed_form(N), rtol=1e-13, atol=0)
    off = rm.mass_full - np.diag(rm.mass)
    assert np.max(np.abs(off)) < 1e-14 * np.max(rm.mass)
    assert np.allclose(rm.face_mass, refmat.face_mass_closed_form(N), rtol=1e-13, atol=0)
    offf = rm.face_mass_full - np.diag(rm.face_mass)
    assert np.max(np.abs(offf)) < 1e-14 * np.max(rm.face_mass)


def _face_raw(N, s):
    fp, fw = refmat.tri_rule(N + 2)
    phis = refmat.eval_volume_basis(N, refmat.face_map(s, fp)).astype(float)
    return (phis * fw) @ phis.T


@pytest.mark.parametrize("N", [2, 3, 5, 6])
def test_stiffness_integration_by_parts(N):
    """S^d + S^d^T = boundary integral of n_d phi_k phi_l (divergence theorem on
    the reference tetrahedron, whose faces 0/1/2 have normals -e_z, -e_y, -e_x)."""
    rm = refmat.refmats(N)
    F = [_face_raw(N, s) for s in range(4)]
    scale = np.max(np.abs(rm.S))
    for d, s in ((0, 2), (1, 1), (2, 0)):
        lhs = rm.S[d] + rm.S[d].T
        assert np.max(np.abs(lhs - (F[3] - F[s]))) < 1e-13 * scale


@pytest.mark.parametrize("N", [2, 3, 5])
def test_ktilde_is_exact_negative_derivative(N):
    """Ktilde^d c(p) = -c(d p/d xi_d) for polynomials p of degree <= N."""
    rm = refmat.refmats(N)
    rng = np.random.default_rng(3)
    pts, w = refmat.tet_rule(N + 2)
    phi = refmat.eval_volume_basis(N, pts).astype(float)
    mono = [(a, b, c) for a in range(N + 1) for b in range(N + 1 - a) for c in range(N + 1 - a - b)]
    coef = rng.standard_normal(len(mono))

    def poly(pts, deriv=None):
        out = np.zeros(len(pts))
        for cf, (a, b, c) in zip(coef, mono):
            e = [a, b, c]
            f = cf
            if deriv is not None:
                f *= e[deriv]
                if e[deriv] == 0:
                    continue
                e[deriv] -= 1
            out += f * pts[:, 0] ** e[0] * pts[:, 1] ** e[1] * pts[:, 2] ** e[2]
        return out

    proj = lambda vals: (phi * w) @ vals / rm.mass
    c = proj(poly(pts))
    for d in range(3):
        assert np.allclose(rm.Ktilde[d] @ c, -proj(poly(pts, d)), rtol=0, atol=1e-11 * np.max(np.abs(c)))
        # Khat is the transpose partner: Khat^d = -M^-1 (M Ktilde^d)^T
        assert np.allclose(rm.Khat[d], -(np.diag(rm.mass) @ rm.Ktilde[d]).T / rm.mass[:, None], atol=1e-14 * np.max(np.abs(rm.Khat[d])))


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6])
def test_sparsity_staircase_and_zero_columns(N):
    """Degree structure: Ktilde^d_kl != 0 only for deg(k) < deg(l); the d-th
    derivative keeps C(N-d+3,3) coefficients (paper Sec. 5.1.2); Khat has
    C(N+2,3) non-zero columns (our reading of the zero-block remark)."""
    rm = refmat.refmats(N)
    deg = np.array([i + j + k for (i, j, k) in refmat.basis_indices(N)])
    for d in range(3):
        nz = np.argwhere(rm.Ktilde[d] != 0)
        assert np.all(deg[nz[:, 0]] < deg[nz[:, 1]])
        ncols = np.nonzero(np.any(rm.Khat[d] != 0, axis=0))[0]
        assert ncols.max() + 1 == comb(N + 2, 3)
    rng = np.random.default_rng(0)
    D = rng.standard_normal(rm.B)
    for dd in range(N + 1):
        rows = np.nonzero(np.abs(D) > 1e-12 * np.max(np.abs(D)))[0]
        assert len(rows) == comb(N - dd + 3, 3)
        assert rows.max() + 1 == comb(N - dd + 3, 3)
        D = sum(rm.Ktilde[d] @ D for d in range(3))


@pytest.mark.parametrize("N", [2, 3, 5, 6])
def test_face_matrices(N):
    rm = refmat.refmats(N)
    rng = np.random.default_rng(5)
    chi = rng.uniform(0, 1, (40, 2))
    chi = chi[chi.sum(1) < 1]
    psi = refmat.eval_face_basis(N, chi).astype(float)        # (Bf, n)
    for s in range(4):
        # R^s holds the exact trace: phi_l(xi^s(chi)) = sum_n R_ln psi_n(chi)
        phis = refmat.eval_volume_basis(N, refmat.face_map(s, chi)).astype(float)
        assert np.allclose(phis, rm.R[s] @ psi, atol=1e-12)
        assert np.allclose(rm.Rhat[s], (rm.R[s] * rm.face_mass[None, :]) / rm.mass[:, None], rtol=1e-13, atol=0)
    Mt = np.diag(rm.face_mass)
    for h in range(3):
        f = rm.f[h]
        psih = refmat.eval_face_basis(N, refmat.orient_map(h, chi)).astype(float)
        assert np.allclose(psih, f.T @ psi, atol=1e-12)
        assert np.allclose(f @ f, np.eye(rm.Bf), atol=1e-12)
        assert np.allclose(f.T @ Mt @ f, Mt, atol=1e-14)
    # f^1 maps chi1 -> 1-chi1-chi2: psi_ij -> (-1)^i psi_ij (diagonal)
    sign = np.array([(-1.0) ** i for (i, j) in refmat.face_basis_indices(N)])
    assert np.allclose(rm.f[1], np.diag(sign), atol=1e-13)


def test_orientation_maps_match_mesh_geometry():
    """A point on face s of element e, mapped with chi~^h, is the same point on
    face j of the neighbour (up to the periodic shift)."""
    mesh = cube_mesh(4, seed_for(0), relabel=True)
    rng = np.random.default_rng(2)
    chi = rng.uniform(0, 1, (10, 2))
    chi = chi[chi.sum(1) < 1]
    fv = np.array(FACE_VERTS)
    seen = set()
    for e in range(0, mesh.E, 3):
        for s in range(4):
            nu, j, h = mesh.neigh[e, s], int(mesh.nface[e, s]), int(mesh.orient[e, s])
            seen.add((j, h))
            a, b, c = mesh.X[e, fv[s]]
            x1 = a + chi[:, :1] * (b - a) + chi[:, 1:] * (c - a)
            ch2 = refmat.orient_map(h, chi)
            a2, b2, c2 = mesh.X[nu, fv[j]]
            x2 = a2 + ch2[:, :1] * (b2 - a2) + ch2[:, 1:] * (c2 - a2)
            d = x1 - x2
            d = d - np.round(d)
            assert np.max(np.abs(d)) < 1e-12
    assert len(seen) == 12
