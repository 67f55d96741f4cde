"""Oracle reference matrices on the reference tetrahedron (test infrastructure).

Follows the paper's Sec. 2 (weak form, stiffness matrices as integrals of
basis-function derivatives against basis functions) and Sec. 5.1 (Dubiner
basis with B = C(N+3,3) functions, K-hat / K-tilde B x B, R / R-hat B x B~,
f B~ x B~ with B~ = C(N+2,2)).  The paper gives no formulas for these
matrices; the readings used here are:

  phi_ijk  = P_i^(0,0)(2xi/(1-eta-zeta)-1) (1-eta-zeta)^i
           * P_j^(2i+1,0)(2eta/(1-zeta)-1) (1-zeta)^j * P_k^(2i+2j+2,0)(2zeta-1)
  psi_ij   = P_i^(0,0)(2chi1/(1-chi2)-1) (1-chi2)^i * P_j^(2i+1,0)(2chi2-1)
  ordering : degree-major; inside total degree d, k ascending, then j
             ascending (i = d-j-k); faces: j ascending (i = d-j)
  S^d_kl   = int dphi_k/dxi_d phi_l ;  Khat^d = M^-1 S^d ; Ktilde^d = -M^-1 S^d^T
  R^s_ln   = (1/mt_n) int_T~ phi_l(xi^s(chi)) psi_n(chi)
  Rhat^s_km= (1/m_k)  int_T~ phi_k(xi^s(chi)) psi_m(chi)
  f^h_mn   = (1/mt_m) int_T~ psi_n(chi~^h(chi)) psi_m(chi)

Method (deliberately plain): every basis function is built as an explicit
polynomial in the monomials xi^a eta^b zeta^c (dense coefficient arrays in
x87 extended precision, so that the cancellation between the large monomial
coefficients of high-order Jacobi polynomials stays below FP64 rounding),
differentiated exactly, and integrated with collapsed-coordinate
Gauss-Jacobi rules whose nodes/weights come from the Golub-Welsch
eigenvalue method.  Entries below 1e-13 * max|matrix| are set to exact 0.
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np

LD = np.longdouble

SNAP = 1e-13

# Reference tetrahedron vertices and faces.  Face s is the vertex triple
# (a, b, c); its outward normal is (b-a) x (c-a).
REF_VERTS = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
FACE_VERTS = ((0, 2, 1), (0, 1, 3), (0, 3, 2), (1, 2, 3))


def n_basis(N: int) -> int:
    return (N + 1) * (N + 2) * (N + 3) // 6


def n_face_basis(N: int) -> int:
    return (N + 1) * (N + 2) // 2


def basis_indices(N: int):
    """(i, j, k) triples in the volume ordering."""
    out = []
    for d in range(N + 1):
        for k in range(d + 1):
            for j in range(d - k + 1):
                out.append((d - j - k, j, k))
    return out


def face_basis_indices(N: int):
    out = []
    for d in range(N + 1):
        for j in range(d + 1):
            out.append((d - j, j))
    return out


# ----------------------------------------------------------------------------
# 1D Jacobi polynomials as coefficient vectors (ascending powers of x)
# ----------------------------------------------------------------------------
def jacobi_coeffs(n: int, alpha: float, beta: float) -> np.ndarray:
    """Coefficients of P_n^(alpha,beta)(x) from the three-term recurrence
    (Abramowitz & Stegun 22.7.1)."""
    alpha = LD(alpha)
    beta = LD(beta)
    p0 = np.array([1.0], dtype=LD)
    if n == 0:
        return p0
    p1 = np.array([(alpha - beta) / 2, (alpha + beta + 2) / 2], dtype=LD)
    for m in range(2, n + 1):
        c = 2 * m + alpha + beta
        a1 = 2 * m * (m + alpha + beta) * (c - 2)
        a2 = (c - 1) * (alpha * alpha - beta * beta)
        a3 = (c - 2) * (c - 1) * c
        a4 = 2 * (m + alpha - 1) * (m + beta - 1) * c
        z1 = np.zeros(1, dtype=LD)
        xp1 = np.concatenate([z1, p1])
        p1e = np.concatenate([p1, z1])
        p0e = np.concatenate([p0, z1, z1])
        p2 = (a2 * p1e + a3 * xp1 - a4 * p0e) / a1
        p0, p1 = p1, p2
    return p1


def jacobi_eval(n: int, alpha: float, beta: float, x):
    x = np.asarray(x, dtype=LD)
    r = np.zeros_like(x)
    for c in jacobi_coeffs(n, alpha, beta)[::-1]:
        r = r * x + c
    return r.astype(float)


def gauss_jacobi(n: int, alpha: float, beta: float = 0.0):
    """n-point Gauss-Jacobi rule for int_{-1}^{1} (1-x)^alpha (1+x)^beta g(x) dx,
    via the Golub-Welsch eigenvalue problem of the Jacobi matrix."""
    k = np.arange(n, dtype=float)
    ab = alpha + beta
    diag = np.empty(n)
    for i in range(n):
        if i == 0:
            diag[0] = (beta - alpha) / (ab + 2.0)
        else:
            diag[i] = (beta * beta - alpha * alpha) / ((2 * i + ab) * (2 * i + ab + 2.0))
    off = np.empty(max(n - 1, 0))
    for i in range(1, n):
        num = 4.0 * i * (i + alpha) * (i + beta) * (i + ab)
        den = (2 * i + ab) ** 2 * (2 * i + ab + 1.0) * (2 * i + ab - 1.0)
        off[i - 1] = math.sqrt(num / den)
    J = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
    x, V = np.linalg.eigh(J)
    mu0 = 2.0 ** (ab + 1.0) * math.gamma(alpha + 1.0) * math.gamma(beta + 1.0) / math.gamma(ab + 2.0)
    w = mu0 * V[0, :] ** 2
    del k
    return x, w


def tet_rule(nq: int):
    """Collapsed-coordinate rule on the reference tetrahedron: points (npts,3),
    weights (npts,) with sum = 1/6."""
    x0, w0 = gauss_jacobi(nq, 0.0)
    x1, w1 = gauss_jacobi(nq, 1.0)
    x2, w2 = gauss_jacobi(nq, 2.0)
    pts, wts = [], []
    for a in range(nq):
        for b in range(nq):
            for c in range(nq):
                zeta = (1.0 + x2[c]) / 2.0
                eta = (1.0 + x1[b]) / 2.0 * (1.0 - zeta)
                xi = (1.0 + x0[a]) / 2.0 * (1.0 - eta - zeta)
                pts.append((xi, eta, zeta))
                wts.append(w0[a] * w1[b] * w2[c] / 64.0)
    return np.array(pts), np.array(wts)


def tri_rule(nq: int):
    """Collapsed-coordinate rule on the reference triangle: sum w = 1/2."""
    x0, w0 = gauss_jacobi(nq, 0.0)
    x1, w1 = gauss_jacobi(nq, 1.0)
    pts, wts = [], []
    for a in range(nq):
        for b in range(nq):
            chi2 = (1.0 + x1[b]) / 2.0
            chi1 = (1.0 + x0[a]) / 2.0 * (1.0 - chi2)
            pts.append((chi1, chi2))
            wts.append(w0[a] * w1[b] / 8.0)
    return np.array(pts), np.array(wts)


# ----------------------------------------------------------------------------
# Dense multivariate polynomials: coefficient array c[a, b, (c)] of x^a y^b z^c
# ----------------------------------------------------------------------------
def _pmul(p, q):
    shape = tuple(a + b - 1 for a, b in zip(p.shape, q.shape))
    r = np.zeros(shape, dtype=LD)
    for idx in zip(*np.nonzero(p)):
        sl = tuple(slice(i, i + s) for i, s in zip(idx, q.shape))
        r[sl] += p[idx] * q
    return r


def _padd(p, q):
    shape = tuple(max(a, b) for a, b in zip(p.shape, q.shape))
    r = np.zeros(shape, dtype=LD)
    r[tuple(slice(0, s) for s in p.shape)] += p
    r[tuple(slice(0, s) for s in q.shape)] += q
    return r


def _ppow(p, m, dim):
    r = np.ones((1,) * dim, dtype=LD)
    for _ in range(m):
        r = _pmul(r, p)
    return r


def _homog(coeffs, num, den, deg, dim):
    """sum_m coeffs[m] * (2*num - den)^m * den^(deg-m): the polynomial
    p(2 num/den - 1) den^deg with num, den polynomials."""
    base = _padd(2 * num, -den)
    r = np.zeros((1,) * dim, dtype=LD)
    for m, c in enumerate(coeffs):
        if c == 0.0:
            continue
        r = _padd(r, c * _pmul(_ppow(base, m, dim), _ppow(den, deg - m, dim)))
    return r


def _pderiv(p, axis):
    n = p.shape[axis]
    if n == 1:
        return np.zeros_like(p)
    idx = np.arange(1, n, dtype=LD)
    sl = [slice(None)] * p.ndim
    sl[axis] = slice(1, n)
    shape = [1] * p.ndim
    shape[axis] = n - 1
    return p[tuple(sl)] * idx.reshape(shape)


def _peval(p, pts):
    """Evaluate polynomial p at points pts (npts, dim)."""
    pts = np.atleast_2d(np.asarray(pts, dtype=LD))
    out = np.zeros(pts.shape[0], dtype=LD)
    for idx in zip(*np.nonzero(p)):
        term = np.full(pts.shape[0], p[idx], dtype=LD)
        for ax, e in enumerate(idx):
            if e:
                term = term * pts[:, ax] ** e
        out += term
    return out


@lru_cache(maxsize=None)
def volume_basis_polys(N: int):
    """Dubiner volume basis as dense coefficient arrays in (xi, eta, zeta)."""
    one = np.ones((1, 1, 1), dtype=LD)
    xi = np.zeros((2, 1, 1), dtype=LD); xi[1, 0, 0] = 1.0
    eta = np.zeros((1, 2, 1), dtype=LD); eta[0, 1, 0] = 1.0
    zeta = np.zeros((1, 1, 2), dtype=LD); zeta[0, 0, 1] = 1.0
    s = _padd(one, _padd(-eta, -zeta))          # 1 - eta - zeta
    t = _padd(one, -zeta)                        # 1 - zeta
    polys = []
    for (i, j, k) in basis_indices(N):
        a = _homog(jacobi_coeffs(i, 0.0, 0.0), xi, s, i, 3)
        b = _homog(jacobi_coeffs(j, 2.0 * i + 1.0, 0.0), eta, t, j, 3)
        c = _homog(jacobi_coeffs(k, 2.0 * i + 2.0 * j + 2.0, 0.0), zeta, one, k, 3)
        polys.append(_pmul(_pmul(a, b), c))
    return polys


@lru_cache(maxsize=None)
def face_basis_polys(N: int):
    one = np.ones((1, 1), dtype=LD)
    c1 = np.zeros((2, 1), dtype=LD); c1[1, 0] = 1.0
    c2 = np.zeros((1, 2), dtype=LD); c2[0, 1] = 1.0
    t = _padd(one, -c2)
    polys = []
    for (i, j) in face_basis_indices(N):
        a = _homog(jacobi_coeffs(i, 0.0, 0.0), c1, t, i, 2)
        b = _homog(jacobi_coeffs(j, 2.0 * i + 1.0, 0.0), c2, one, j, 2)
        polys.append(_pmul(a, b))
    return polys


def eval_volume_basis(N: int, pts) -> np.ndarray:
    """phi_l(pts) as array (B, npts)."""
    return np.array([_peval(p, pts) for p in volume_basis_polys(N)])


def eval_volume_basis_grad(N: int, pts) -> np.ndarray:
    """d phi_l / d xi_d at pts, array (3, B, npts)."""
    polys = volume_basis_polys(N)
    return np.array([[_peval(_pderiv(p, d), pts) for p in polys] for d in range(3)])


def eval_face_basis(N: int, pts) -> np.ndarray:
    return np.array([_peval(p, pts) for p in face_basis_polys(N)])


def face_map(sigma: int, chi) -> np.ndarray:
    """xi^sigma(chi) = a + chi1 (b - a) + chi2 (c - a) for face sigma."""
    a, b, c = (REF_VERTS[v] for v in FACE_VERTS[sigma])
    chi = np.atleast_2d(chi)
    return a[None, :] + chi[:, 0:1] * (b - a)[None, :] + chi[:, 1:2] * (c - a)[None, :]


def orient_map(h: int, chi) -> np.ndarray:
    """chi~^h: the neighbour's face coordinates of the point with local face
    coordinates chi, when the first local face vertex sits at position h of
    the neighbour's face triple."""
    chi = np.atleast_2d(chi)
    c1, c2 = chi[:, 0], chi[:, 1]
    if h == 0:
        return np.stack([c2, c1], axis=1)
    if h == 1:
        return np.stack([1.0 - c1 - c2, c2], axis=1)
    if h == 2:
        return np.stack([c1, 1.0 - c1 - c2], axis=1)
    raise ValueError(h)


def _snap(A: np.ndarray) -> np.ndarray:
    A = A.copy()
    m = np.max(np.abs(A)) if A.size else 0.0
    A[np.abs(A) < SNAP * m] = 0.0
    return A


class RefMats:
    """All reference matrices for degree N (FP64 numpy arrays; products are
    accumulated in extended precision and rounded once)."""

    def __init__(self, N: int):
        if not 1 <= N <= 8:
            raise ValueError("degree out of range")
        self.N = N
        self.B = n_basis(N)
        self.Bf = n_face_basis(N)
        nq = N + 2
        vp, vw = tet_rule(nq)
        vw = vw.astype(LD)
        phi = eval_volume_basis(N, vp)                # (B, nv)
        dphi = eval_volume_basis_grad(N, vp)          # (3, B, nv)
        mass_full = (phi * vw) @ phi.T
        mass = np.diag(mass_full).copy()
        S = np.einsum('dkq,lq,q->dkl', dphi, phi, vw)
        self.mass_full = mass_full.astype(float)
        self.mass = mass.astype(float)
        self.S = S.astype(float)
        self.Khat = _snap_each((S / mass[None, :, None]).astype(float))
        self.Ktilde = _snap_each((-np.transpose(S, (0, 2, 1)) / mass[None, :, None]).astype(float))
        fp, fw = tri_rule(nq)
        fw = fw.astype(LD)
        psi = eval_face_basis(N, fp)                  # (Bf, nf)
        face_mass_full = (psi * fw) @ psi.T
        fmass = np.diag(face_mass_full).copy()
        self.face_mass_full = face_mass_full.astype(float)
        self.face_mass = fmass.astype(float)
        R = []
        Rhat = []
        for s in range(4):
            phis = eval_volume_basis(N, face_map(s, fp))   # (B, nf)
            raw = (phis * fw) @ psi.T                     # (B, Bf)
            R.append(_snap((raw / fmass[None, :]).astype(float)))
            Rhat.append(_snap((raw / mass[:, None]).astype(float)))
        self.R = np.array(R)
        self.Rhat = np.array(Rhat)
        f = []
        for h in range(3):
            psih = eval_face_basis(N, orient_map(h, fp))   # (Bf, nf): psi_n(chi~^h)
            raw = (psi * fw) @ psih.T                     # [m, n]
            f.append(_snap((raw / fmass[:, None]).astype(float)))
        self.f = np.array(f)


def _snap_each(A):
    return np.array([_snap(a) for a in A])


@lru_cache(maxsize=None)
def refmats(N: int) -> RefMats:
    return RefMats(N)


def mass_closed_form(N: int) -> np.ndarray:
    return np.array([1.0 / ((2 * i + 1) * (2 * i + 2 * j + 2) * (2 * i + 2 * j + 2 * k + 3))
                     for (i, j, k) in basis_indices(N)])


def face_mass_closed_form(N: int) -> np.ndarray:
    return np.array([1.0 / ((2 * i + 1) * (2 * i + 2 * j + 2)) for (i, j) in face_basis_indices(N)])
