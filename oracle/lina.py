"""Oracle of the LinA ADER-DG-SEM scheme on cuboids (test infrastructure only).

The paper's LinA application (Sec. 5.2): linearised acoustics in three
dimensions, quantities (pressure p, velocities u, v, w), a uniform periodic
grid of cubic elements, a tensor-product nodal basis on the Gauss-Lobatto
points of each direction, and the ADER scheme
  Eq. lina:derivative   D^{d+1}_xyzp = Kt_xl D^d_lyzq A*_pq + Kt_ym D^d_xmzq B*_pq
                                       + Kt_zn D^d_xynq C*_pq,   D^0 = Q
  Eq. lina:integration  I = sum_{d=0}^{N} dt^{d+1}/(d+1)! D^d
  weak derivatives      Q* = Q + Kh_xl I_lyzq A*_pq + Kh_ym I_xmzq B*_pq + Kh_zn I_xynq C*_pq
  Eq. lin3d_evaluateSide  X^s = F^s_l I_lyzp (left/right), Y, Z alike,
                        F^left = delta_{l0}, F^right = delta_{lN}
  Eq. lina3d_flux       Q_new = Q* + sum_s Fh^s_x (X^s_yzq Ap^s_pq + X^{Neigh(s)}_yzq Am^s_pq) + (y, z)
The paper leaves the matrices to the reader; the readings used here (each
one a textbook DG-SEM fact, restated):
  * nodes and weights: the N+1 Gauss-Lobatto-Legendre points of [0, 1]; the
    mass matrix is the lumped (collocated) one, h w_i per direction;
  * Kt = -Dm with Dm_il = psi_l'(x_i) the collocation derivative (the strong
    derivative of Eq. lina:derivative), Kh_kl = (w_l / w_k) Dm_lk (the weak
    derivative M^-1 S, S_kl = int psi_k' psi_l, exact in GLL quadrature);
  * A* = A / h, B* = B / h, C* = C / h with the acoustic Jacobians of
    q_t + A q_x + B q_y + C q_z = 0: p_t + K0 div(u) = 0, u_t + grad(p)/rho0 = 0;
  * side s with outward normal n: upwind flux A_n^+ q_own + A_n^- q_nb,
    A_n^{+-} = (A_n +- |A_n|)/2, |A_n| = c times the projector on (p, u.n);
    Ap^s = -A_n^+ / h, Am^s = -A_n^- / h, and the lift Fh^s_x = delta_{x,e}/w_e
    for the node index e of the side (0 or N);
  * the neighbour's side data X^{Neigh(s)} is the neighbour element's side
    facing this element (its right side for this element's left side).
Layout: Q[e][p][z][y][x] (x fastest; the paper's Q_xyzp in column-major
order); elements of an n x n x n grid numbered e = (i_z n + i_y) n + i_x.
"""
from __future__ import annotations

from math import factorial

import numpy as np
from numpy.polynomial import legendre as L

SIDES = ("left", "right", "bottom", "top", "back", "front")   # -x, +x, -y, +y, -z, +z


def gll(N):
    """Nodes (ascending) and weights of the (N+1)-point Gauss-Lobatto rule on
    [0, 1]: the endpoints and the roots of P_N', weights 2/(N(N+1) P_N(x)^2)
    on [-1, 1], mapped."""
    cN = np.zeros(N + 1)
    cN[N] = 1.0
    inner = np.sort(np.real(L.legroots(L.legder(cN)))) if N >= 2 else np.array([])
    x = np.concatenate([[-1.0], inner, [1.0]])
    w = 2.0 / (N * (N + 1) * L.legval(x, cN) ** 2)
    return (x + 1.0) / 2.0, w / 2.0


def lagrange_derivative(nodes):
    """Dm[i][j] = psi_j'(nodes[i]) for the Lagrange polynomials psi_j of the
    nodes, in barycentric form: with b_j = 1 / prod_{k != j} (x_j - x_k),
    Dm_ij = (b_j / b_i) / (x_i - x_j) for i != j, and Dm_ii = -sum_{j != i}
    Dm_ij (the derivatives of the psi_j sum to that of 1, zero)."""
    n = len(nodes)
    diff = nodes[:, None] - nodes[None, :]
    np.fill_diagonal(diff, 1.0)
    b = 1.0 / np.prod(diff, axis=1)
    Dm = (b[None, :] / b[:, None]) / diff
    np.fill_diagonal(Dm, 0.0)
    np.fill_diagonal(Dm, -Dm.sum(axis=1))
    return Dm


def matrices(N):
    """dict: nodes x, weights w, Dm, Kt = -Dm, Kh = W^-1 Dm^T W."""
    x, w = gll(N)
    Dm = lagrange_derivative(x)
    Kh = (w[None, :] / w[:, None]) * Dm.T
    return dict(N=N, x=x, w=w, Dm=Dm, Kt=-Dm, Kh=Kh)


def jacobians(rho0, K0):
    """A, B, C (4 x 4) for q = (p, u, v, w)."""
    J = np.zeros((3, 4, 4))
    for d in range(3):
        J[d, 0, 1 + d] = K0
        J[d, 1 + d, 0] = 1.0 / rho0
    return J


def element_matrices(rho0, K0, h):
    """Star matrices (3, 4, 4) and the side flux solvers Ap, Am (6, 4, 4) in
    SIDES order."""
    J = jacobians(rho0, K0)
    c = np.sqrt(K0 / rho0)
    star = J / h
    Ap = np.zeros((6, 4, 4))
    Am = np.zeros((6, 4, 4))
    for s in range(6):
        d, sign = s // 2, (-1.0 if s % 2 == 0 else 1.0)
        An = sign * J[d]
        absA = np.zeros((4, 4))
        absA[0, 0] = c
        absA[1 + d, 1 + d] = c
        Ap[s] = -(An + absA) / 2.0 / h
        Am[s] = -(An - absA) / 2.0 / h
    return star, Ap, Am


def grid_neighbours(n):
    """neigh[e][s] for the periodic n x n x n grid, s in SIDES order."""
    E = n ** 3
    e = np.arange(E)
    ix, iy, iz = e % n, (e // n) % n, e // (n * n)
    idx = lambda a, b, c: ((c % n) * n + (b % n)) * n + (a % n)
    return np.stack([idx(ix - 1, iy, iz), idx(ix + 1, iy, iz), idx(ix, iy - 1, iz), idx(ix, iy + 1, iz),
                     idx(ix, iy, iz - 1), idx(ix, iy, iz + 1)], axis=1).astype(np.int32)


# -- the stages, in the paper's notation (arrays Q[e, p, z, y, x]) -----------
def contract_x(K, T):
    """K_xl T_e,q,z,y,l"""
    return np.einsum("xl,eqzyl->eqzyx", K, T)


def contract_y(K, T):
    return np.einsum("ym,eqzmx->eqzyx", K, T)


def contract_z(K, T):
    return np.einsum("zn,eqnyx->eqzyx", K, T)


def mix(S, T):
    """S_pq T_e,q,... (quantity mixing)"""
    return np.einsum("pq,eq...->ep...", S, T)


def derivatives(m, star, Q):
    """D^0..D^N (Eq. lina:derivative): shape (E, N+1, 4, O, O, O)."""
    D = [np.asarray(Q, dtype=np.float64)]
    for _ in range(m["N"]):
        Dd = D[-1]
        D.append(mix(star[0], contract_x(m["Kt"], Dd)) + mix(star[1], contract_y(m["Kt"], Dd))
                 + mix(star[2], contract_z(m["Kt"], Dd)))
    return np.stack(D, axis=1)


def time_integral(D, dt):
    """Eq. lina:integration."""
    N1 = D.shape[1]
    return sum(dt ** (d + 1) / factorial(d + 1) * D[:, d] for d in range(N1))


def weak_derivatives(m, star, I):
    """Kh_xl I_lyzq A*_pq + Kh_ym I_xmzq B*_pq + Kh_zn I_xynq C*_pq."""
    return (mix(star[0], contract_x(m["Kh"], I)) + mix(star[1], contract_y(m["Kh"], I))
            + mix(star[2], contract_z(m["Kh"], I)))


def sides(I):
    """Eq. lin3d_evaluateSide: (E, 6, 4, O, O) boundary nodes of I per side
    in SIDES order, each a 2D array over the two remaining directions in the
    order (z, y), (z, x) or (y, x)."""
    N = I.shape[-1] - 1
    return np.stack([I[..., 0], I[..., N], I[..., 0, :], I[..., N, :], I[:, :, 0], I[:, :, N]], axis=1)


def flux(m, Ap, Am, X, neigh):
    """Eq. lina3d_flux without Q*: the update of every element's boundary
    nodes from its own and its neighbours' sides."""
    E, _, P, O, _ = X.shape
    N = O - 1
    w = m["w"]
    out = np.zeros((E, P, O, O, O))
    for s in range(6):
        opp = s ^ 1                              # the neighbour's side facing us
        Xo, Xn = X[:, s], X[neigh[:, s], opp]
        g = np.einsum("pq,eqab->epab", Ap[s], Xo) + np.einsum("pq,eqab->epab", Am[s], Xn)
        edge = 0 if s % 2 == 0 else N
        g = g / w[edge]
        if s < 2:
            out[..., edge] += g
        elif s < 4:
            out[..., edge, :] += g
        else:
            out[:, :, edge] += g
    return out


def step(m, star, Ap, Am, neigh, Q, dt):
    """One ADER-DG-SEM time step: Q^{tau+1}."""
    I = time_integral(derivatives(m, star, Q), dt)
    return Q + weak_derivatives(m, star, I) + flux(m, Ap, Am, sides(I), neigh)


def brute_derivative(Kt, star, D):
    """One recursion step of Eq. lina:derivative for one element, as the
    literal index sum (nested loops; tiny inputs only)."""
    P, O = D.shape[0], D.shape[1]
    out = np.zeros_like(D)
    for p in range(P):
        for z in range(O):
            for y in range(O):
                for x in range(O):
                    s = 0.0
                    for q in range(P):
                        for l in range(O):
                            s += Kt[x, l] * D[q, z, y, l] * star[0, p, q]
                            s += Kt[y, l] * D[q, z, l, x] * star[1, p, q]
                            s += Kt[z, l] * D[q, l, y, x] * star[2, p, q]
                    out[p, z, y, x] = s
    return out
