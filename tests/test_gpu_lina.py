"""GPU parity of the LinA ADER-DG-SEM step (dg_lina_step, Sec. 5.2) through
the C ABI against the LinA oracle (oracle/lina.py) on the same seeded inputs.

Each side computes its own coefficients (the product's blob from
dg_lina_coefficients, the oracle's from oracle.lina).  Inputs: periodic
n x n x n grids, air-like acoustics (rho0 1.2, K0 1.4e5), dt = 0.3 h /
(c (2 order - 1)), DOFs N(0,1).  Bars on the step increment, per quantity
and per element (dgtest): FP64 1e-12, FP32 1e-5 (the increment of random
data is of the size of the data, so its FP32 rounding is a few 2^-24 per
term summed over the order's line contractions).
"""
import sys

import numpy as np
import pytest

from dgtest import assert_close
from oracle import lina

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RHO0, K0 = 1.2, 1.4e5


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _case(order, n, seed):
    h = 1.0 / n
    c = np.sqrt(K0 / RHO0)
    dt = 0.3 * h / (c * (2 * order - 1))
    rng = np.random.default_rng(seed)
    Q = rng.standard_normal((n ** 3, 4, order, order, order))
    return h, dt, Q, lina.grid_neighbours(n)


def _gpu(order, dtype, h, dt, Q, neigh, steps):
    import paper_1903_11521_amd as dg
    coef = torch.from_numpy(dg.lina_coefficients(order, RHO0, K0, h)["blob"]).to(dtype).to("cuda:0")
    Qg = torch.from_numpy(Q).to(dtype).to("cuda:0")
    E = Q.shape[0]
    sides = torch.empty((E, 6, 4, order, order), dtype=dtype, device="cuda:0")
    dg.lina_step(Qg, sides, coef, torch.from_numpy(neigh).to("cuda:0"), dt, steps)
    torch.cuda.synchronize()
    return Qg.double().cpu().numpy(), sides.double().cpu().numpy()


def _oracle(order, h, dt, Q, neigh, steps):
    m = lina.matrices(order - 1)
    star, Ap, Am = lina.element_matrices(RHO0, K0, h)
    for _ in range(steps):
        I = lina.time_integral(lina.derivatives(m, star, Q), dt)
        Q = Q + lina.weak_derivatives(m, star, I) + lina.flux(m, Ap, Am, lina.sides(I), neigh)
    return Q, lina.sides(I)


@pytest.mark.parametrize("dtype,order,n", [(torch.float64, 2, 3), (torch.float64, 3, 3), (torch.float64, 5, 4),
                                           (torch.float64, 8, 3), (torch.float64, 12, 3),
                                           (torch.float32, 4, 3), (torch.float32, 8, 3), (torch.float32, 16, 3)])
def test_lina_step_matches_oracle(dtype, order, n):
    _say(f"test_lina_step_matches_oracle {dtype} order={order} n={n}")
    h, dt, Q, neigh = _case(order, n, 100 + order)
    if dtype == torch.float32:
        Q = Q.astype(np.float32).astype(np.float64)
    got, gs = _gpu(order, dtype, h, dt, Q, neigh, 1)
    ref, rs = _oracle(order, h, dt, Q, neigh, 1)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    E = Q.shape[0]
    assert_close((got - Q).reshape(E, 4, -1), (ref - Q).reshape(E, 4, -1), tol, "step increment")
    assert_close(gs.reshape(E, 24, -1), rs.reshape(E, 24, -1), tol, "side values of I")


def test_lina_three_steps_order8():
    _say("test_lina_three_steps_order8")
    order, n = 8, 3
    h, dt, Q, neigh = _case(order, n, 7)
    got, _ = _gpu(order, torch.float64, h, dt, Q, neigh, 3)
    ref, _ = _oracle(order, h, dt, Q, neigh, 3)
    E = Q.shape[0]
    assert_close((got - Q).reshape(E, 4, -1), (ref - Q).reshape(E, 4, -1), 1e-12, "3-step increment")


def test_lina_missing_neighbours():
    """Neighbour indices outside [0, E) drop that side's neighbour term."""
    _say("test_lina_missing_neighbours")
    order, n = 4, 3
    h, dt, Q, neigh = _case(order, n, 9)
    nb = neigh.copy()
    nb[0, 1] = -1
    nb[5, 4] = 10 ** 6
    got, _ = _gpu(order, torch.float64, h, dt, Q, nb, 1)
    m = lina.matrices(order - 1)
    star, Ap, Am = lina.element_matrices(RHO0, K0, h)
    I = lina.time_integral(lina.derivatives(m, star, Q), dt)
    X = lina.sides(I)
    ref = Q + lina.weak_derivatives(m, star, I) + lina.flux(m, Ap, Am, X, neigh)
    # remove the dropped neighbour terms from the oracle's result
    for e, s in ((0, 1), (5, 4)):
        g = np.einsum("pq,qab->pab", Am[s], X[neigh[e, s], s ^ 1]) / m["w"][0 if s % 2 == 0 else order - 1]
        edge = 0 if s % 2 == 0 else order - 1
        if s < 2:
            ref[e][..., edge] -= g
        elif s < 4:
            ref[e][..., edge, :] -= g
        else:
            ref[e][:, edge] -= g
    E = Q.shape[0]
    assert_close((got - Q).reshape(E, 4, -1), (ref - Q).reshape(E, 4, -1), 1e-12, "step increment")
