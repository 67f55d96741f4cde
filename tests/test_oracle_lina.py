"""Pins of the LinA oracle (oracle/lina.py) against facts that do not come
from it: Gauss-Lobatto closed forms and exactness, exact differentiation of
polynomials, the summation-by-parts identity of the collocation derivative,
the literal index sum of Eq. lina:derivative, conservation and free stream
of the upwind scheme on a periodic grid, and convergence on an exact
acoustic plane wave (order above N in h)."""
import math

import numpy as np
import pytest

from oracle import lina


def test_gll_closed_forms():
    x, w = lina.gll(2)
    assert np.allclose(x, [0.0, 0.5, 1.0], atol=1e-15) and np.allclose(w, [1 / 6, 2 / 3, 1 / 6], atol=1e-15)
    x, w = lina.gll(3)
    a = (1.0 - 1.0 / math.sqrt(5.0)) / 2.0
    assert np.allclose(x, [0.0, a, 1.0 - a, 1.0], atol=1e-15)
    assert np.allclose(w, [1 / 12, 5 / 12, 5 / 12, 1 / 12], atol=1e-15)


@pytest.mark.parametrize("N", [2, 3, 5, 7, 11, 15])
def test_gll_exactness(N):
    """Exact for x^k, k <= 2N-1, and (where the error is above rounding) not
    for k = 2N: Lobatto, not Gauss."""
    x, w = lina.gll(N)
    for k in range(2 * N):
        assert abs(np.dot(w, x ** k) - 1.0 / (k + 1)) <= 1e-13
    if N <= 5:
        assert abs(np.dot(w, x ** (2 * N)) - 1.0 / (2 * N + 1)) > 1e-6


@pytest.mark.parametrize("N", [1, 2, 4, 7, 11, 15])
def test_derivative_matrix_exact_on_polynomials(N):
    m = lina.matrices(N)
    rng = np.random.default_rng(N)
    c = rng.standard_normal(N + 1)
    f = np.polynomial.Polynomial(c)
    got = m["Dm"] @ f(m["x"])
    ref = f.deriv()(m["x"])
    assert np.max(np.abs(got - ref)) <= 1e-10 * max(1.0, np.max(np.abs(ref))) * N ** 2


@pytest.mark.parametrize("N", [2, 3, 7, 15])
def test_summation_by_parts(N):
    """W Dm + (W Dm)^T = diag(-1, 0, ..., 0, 1): the GLL collocation
    derivative integrates by parts exactly."""
    m = lina.matrices(N)
    Q = np.diag(m["w"]) @ m["Dm"]
    Bd = np.zeros((N + 1, N + 1))
    Bd[0, 0], Bd[N, N] = -1.0, 1.0
    assert np.max(np.abs(Q + Q.T - Bd)) <= 1e-11 * N


def test_derivative_recursion_literal_index_sum():
    N = 2
    m = lina.matrices(N)
    rng = np.random.default_rng(5)
    star = rng.standard_normal((3, 4, 4))
    D = rng.standard_normal((1, 4, N + 1, N + 1, N + 1))
    got = lina.derivatives(m, star, D)[0, 1]
    ref = lina.brute_derivative(m["Kt"], star, D[0])
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    # the weak derivatives are the same sum with Kh
    got = lina.weak_derivatives(m, star, D)[0]
    ref = lina.brute_derivative(m["Kh"], star, D[0])
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def _setup(N, n, rho0=1.2, K0=1.4e5):
    m = lina.matrices(N)
    h = 1.0 / n
    star, Ap, Am = lina.element_matrices(rho0, K0, h)
    c = math.sqrt(K0 / rho0)
    dt = 0.3 * h / (c * (2 * N + 1))
    return m, star, Ap, Am, lina.grid_neighbours(n), c, dt


def test_conservation_and_free_stream():
    N, n = 3, 3
    m, star, Ap, Am, neigh, c, dt = _setup(N, n)
    rng = np.random.default_rng(2)
    Q = rng.standard_normal((n ** 3, 4, N + 1, N + 1, N + 1))
    Q1 = lina.step(m, star, Ap, Am, neigh, Q, dt)
    w3 = np.einsum("z,y,x->zyx", m["w"], m["w"], m["w"])
    before = np.einsum("epzyx,zyx->p", Q, w3)
    after = np.einsum("epzyx,zyx->p", Q1, w3)
    scale = np.einsum("epzyx,zyx->p", np.abs(Q1 - Q), w3)
    assert np.all(np.abs(after - before) <= 1e-12 * scale)
    Qc = np.zeros_like(Q)
    Qc[:, :] = np.array([3.0, -1.0, 0.5, 2.0])[None, :, None, None, None]
    # rows of the collocation derivative sum to zero up to rounding
    assert np.max(np.abs(lina.step(m, star, Ap, Am, neigh, Qc, dt) - Qc)) <= 1e-11 * np.max(np.abs(Qc))


def _wave(N, n, T, rho0=1.2, K0=1.4e5):
    """Max nodal error after T of an acoustic plane wave along k = 2 pi (1, 1, 1)."""
    m, star, Ap, Am, neigh, c, dt = _setup(N, n, rho0, K0)
    Z = rho0 * c
    kv = 2 * np.pi * np.array([1.0, 1.0, 1.0])
    kn = np.linalg.norm(kv)
    khat = kv / kn
    r = np.concatenate([[Z], khat])             # A_k r = c r
    h = 1.0 / n
    E = n ** 3
    e = np.arange(E)
    ix, iy, iz = e % n, (e // n) % n, e // (n * n)
    X = (ix[:, None] + m["x"][None, :]) * h
    Y = (iy[:, None] + m["x"][None, :]) * h
    Zc = (iz[:, None] + m["x"][None, :]) * h
    phase = (kv[0] * X[:, None, None, :] + kv[1] * Y[:, None, :, None] + kv[2] * Zc[:, :, None, None])

    def exact(t):
        return r[None, :, None, None, None] * np.sin(phase - c * kn * t)[:, None]
    steps = int(round(T / dt))
    Q = exact(0.0)
    for _ in range(steps):
        Q = lina.step(m, star, Ap, Am, neigh, Q, dt)
    return np.max(np.abs(Q - exact(steps * dt))) / Z, steps * dt


@pytest.mark.parametrize("N", [3, 5])
def test_plane_wave_convergence(N):
    """Same simulated time on n = 4 and n = 8 (dt halves with h): the error
    falls by more than 2^N, and is small at n = 8."""
    T = 8 * _setup(N, 4)[-1]
    e4, t4 = _wave(N, 4, T)
    e8, t8 = _wave(N, 8, T)
    assert abs(t4 - t8) <= 1e-12 * t4
    assert e8 < 1e-2
    assert e4 / e8 > 2 ** N, (e4, e8)
