"""Pins of the MADNESS contraction oracle (Sec. 7, Eq. stock_mra).

  * the literal nine-index sum on tiny tensors;
  * every other association order (operator pairs first, then one
    p x p matrix per mode, in any mode order) gives the same result;
  * rank one (q = 1) has the closed form
    R_ijk = (sum_xyz S_xyz a_x b_y c_z) u_i v_j w_k;
  * identity factors (q = p, X^L = X^R = I, ...) return S.
"""
import itertools

import numpy as np
import pytest

from oracle import madness


def _ops(rng, p, q):
    return [rng.standard_normal(sh) for sh in ((p, q), (q, p)) * 3]


@pytest.mark.parametrize("p,q", [(3, 2), (2, 2), (3, 1)])
def test_brute_force(p, q):
    rng = np.random.default_rng(11 + p + q)
    S = rng.standard_normal((p, p, p))
    ops = _ops(rng, p, q)
    ref = madness.brute(S.tolist(), *[o.tolist() for o in ops])
    got = madness.apply(S[None], *ops)[0]
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_association_orders():
    rng = np.random.default_rng(5)
    p, q = 7, 3
    S = rng.standard_normal((4, p, p, p))
    XL, XR, YL, YR, ZL, ZR = _ops(rng, p, q)
    ref = madness.apply(S, XL, XR, YL, YR, ZL, ZR)
    mats = {"x": XL @ XR, "y": YL @ YR, "z": ZL @ ZR}
    for order in itertools.permutations("xyz"):
        T = S.copy()
        for mode in order:
            ax = {"x": 1, "y": 2, "z": 3}[mode]
            T = np.moveaxis(np.tensordot(T, mats[mode], axes=([ax], [0])), -1, ax)
        assert np.max(np.abs(T - ref)) <= 1e-12 * np.max(np.abs(ref)), order


def test_rank_one_closed_form():
    rng = np.random.default_rng(9)
    p = 6
    S = rng.standard_normal((3, p, p, p))
    a, b, c, u, v, w = (rng.standard_normal(p) for _ in range(6))
    R = madness.apply(S, a[:, None], u[None, :], b[:, None], v[None, :], c[:, None], w[None, :])
    s = np.einsum("nxyz,x,y,z->n", S, a, b, c)
    ref = s[:, None, None, None] * u[None, :, None, None] * v[None, None, :, None] * w[None, None, None, :]
    assert np.max(np.abs(R - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_identity_factors():
    rng = np.random.default_rng(3)
    p = 5
    S = rng.standard_normal((2, p, p, p))
    I = np.eye(p)
    assert np.array_equal(madness.apply(S, I, I, I, I, I, I), S)
