"""Oracle of the MADNESS separable contraction (test infrastructure: only the
tests, the smoke check and the benchmark's CPU-baseline leg use it).

Sec. 7, Eq. stock_mra: for a p x p x p tensor S and three low-rank operator
pairs (X^L p x q, X^R q x p, and likewise Y, Z),
    R_ijk = sum_{x,y,z,l,m,n} S_xyz X^L_xl X^R_li Y^L_ym Y^R_mj Z^L_zn Z^R_nk.
The paper evaluates it as a chain of binary contractions, one index at a
time: x with X^L, then l with X^R, then y, m, z, n.  `apply` takes exactly
those six steps, each a library tensordot (a matrix product over one index),
for a batch of tensors sharing the operators.  `brute` is the literal
nine-index sum, pure Python, for tiny sizes.
"""
from __future__ import annotations

import numpy as np


def apply(S, XL, XR, YL, YR, ZL, ZR):
    """S (nb, p, p, p) -> R (nb, p, p, p), FP64."""
    S = np.asarray(S, dtype=np.float64)
    T = np.tensordot(S, XL, axes=([1], [0]))          # (nb, y, z, l)     sum over x
    T = np.tensordot(T, XR, axes=([3], [0]))          # (nb, y, z, i)     sum over l
    T = np.tensordot(T, YL, axes=([1], [0]))          # (nb, z, i, m)     sum over y
    T = np.tensordot(T, YR, axes=([3], [0]))          # (nb, z, i, j)     sum over m
    T = np.tensordot(T, ZL, axes=([1], [0]))          # (nb, i, j, n)     sum over z
    T = np.tensordot(T, ZR, axes=([3], [0]))          # (nb, i, j, k)     sum over n
    return T


def brute(S, XL, XR, YL, YR, ZL, ZR):
    """The nine-index sum of Eq. stock_mra for one tensor S (p, p, p), loops."""
    p = len(S)
    q = len(XL[0])
    R = [[[0.0] * p for _ in range(p)] for _ in range(p)]
    for i in range(p):
        for j in range(p):
            for k in range(p):
                acc = 0.0
                for x in range(p):
                    for y in range(p):
                        for z in range(p):
                            s = S[x][y][z]
                            for l in range(q):
                                for m in range(q):
                                    for n in range(q):
                                        acc += (s * XL[x][l] * XR[l][i] * YL[y][m] * YR[m][j]
                                                * ZL[z][n] * ZR[n][k])
                R[i][j][k] = acc
    return np.array(R)


def flops(p, q):
    """Non-zero flops of the six-step evaluation per tensor (a multiply and
    an add per term): each step is a p x p x p (or p x p x q) output with a
    sum over p or q, 12 p^3 q in total."""
    return 12 * p ** 3 * q
