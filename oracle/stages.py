"""Oracle stages: ctypes binding of oracle/stages.c plus brute-force index sums.

Test infrastructure only (see the package docstring).  Every function takes
and returns FP64 numpy arrays in the element-major layouts listed in
stages.c, and follows the paper's Sec. 5.1.1:
  predictor        Eq. seissol:derivative     (unscaled derivatives D^0..D^N)
  time_integral    Eq. seissol:timeint
  volume           Eq. seissol:correction_local, stiffness terms
  local_flux       Eq. seissol:correction_local, face terms (R-tilde = R)
  neighbour_flux   Eq. seissol:correction_neigh
  step             Q + volume + local_flux + neighbour_flux of the time
                   integral of the predictor (one global time step)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from math import factorial

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stages.c")
_LIB = os.path.join(_HERE, "_oracle_stages.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle loop nests with gcc (plain -O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            dp = ctypes.POINTER(ctypes.c_double)
            i32p = ctypes.POINTER(ctypes.c_int32)
            i8p = ctypes.POINTER(ctypes.c_int8)
            I, L, D = ctypes.c_int, ctypes.c_int64, ctypes.c_double
            lib.oracle_predictor.argtypes = [I, I, I, L, dp, dp, dp, dp]
            lib.oracle_time_integral.argtypes = [I, I, I, L, D, dp, dp]
            lib.oracle_volume.argtypes = [I, I, L, dp, dp, dp, dp]
            lib.oracle_local_flux.argtypes = [I, I, I, L, dp, dp, dp, dp, dp]
            lib.oracle_neighbour_flux.argtypes = [I, I, I, L, dp, dp, dp, i32p, i8p, i8p, dp, dp, dp]
            lib.oracle_set_threads.argtypes = [I]
            lib.oracle_max_threads.restype = I
            _lib = lib
    return _lib


def set_threads(n: int) -> None:
    """OpenMP thread count of the loop nests (for timing runs)."""
    _load().oracle_set_threads(int(n))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def _p(a, ctype=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


def predictor(rm, star, Q):
    """D^0..D^N, shape (E, N+1, P, B)."""
    lib = _load()
    Q = _c(Q); star = _c(star); Kt = _c(rm.Ktilde)
    E, P, B = Q.shape
    D = np.empty((E, rm.N + 1, P, B))
    lib.oracle_predictor(rm.N, B, P, E, _p(Kt), _p(star), _p(Q), _p(D))
    return D


def time_integral(N, D, dt):
    lib = _load()
    D = _c(D)
    E, _, P, B = D.shape
    I = np.empty((E, P, B))
    lib.oracle_time_integral(N, B, P, E, float(dt), _p(D), _p(I))
    return I


def volume(rm, star, I):
    lib = _load()
    I = _c(I); star = _c(star); Kh = _c(rm.Khat)
    E, P, B = I.shape
    dQ = np.empty_like(I)
    lib.oracle_volume(B, P, E, _p(Kh), _p(star), _p(I), _p(dQ))
    return dQ


def local_flux(rm, Aplus, I):
    lib = _load()
    I = _c(I); Ap = _c(Aplus)
    E, P, B = I.shape
    dQ = np.empty_like(I)
    lib.oracle_local_flux(B, rm.Bf, P, E, _p(_c(rm.Rhat)), _p(_c(rm.R)), _p(Ap), _p(I), _p(dQ))
    return dQ


def neighbour_flux(rm, Aminus, I_all, neigh, nface, orient, E=None):
    """Neighbour term for elements 0..E-1 (default: all of I_all); neighbour
    indices point into I_all."""
    lib = _load()
    I_all = _c(I_all); Am = _c(Aminus)
    neigh = _c(neigh, np.int32); nface = _c(nface, np.int8); orient = _c(orient, np.int8)
    E = neigh.shape[0] if E is None else E
    P, B = I_all.shape[1], I_all.shape[2]
    dQ = np.empty((E, P, B))
    lib.oracle_neighbour_flux(B, rm.Bf, P, E, _p(_c(rm.Rhat)), _p(_c(rm.R)), _p(_c(rm.f)),
                              _p(neigh, ctypes.c_int32), _p(nface, ctypes.c_int8),
                              _p(orient, ctypes.c_int8), _p(Am), _p(I_all), _p(dQ))
    return dQ


def step(rm, dt, Q, star, Aplus, Aminus, neigh, nface, orient, return_parts=False):
    """One global ADER-DG time step on all elements."""
    D = predictor(rm, star, Q)
    I = time_integral(rm.N, D, dt)
    dv = volume(rm, star, I)
    dl = local_flux(rm, Aplus, I)
    dn = neighbour_flux(rm, Aminus, I, neigh, nface, orient)
    Qn = Q + dv + dl + dn
    if return_parts:
        return Qn, dict(D=D, I=I, vol=dv, lf=dl, nf=dn)
    return Qn


def step_subset(rm, dt, ids, Q, star, Aplus, Aminus, neigh, nface, orient):
    """Q^{n+1} of the elements `ids` only: the predictor runs on `ids` and their
    face neighbours, the corrector on `ids`.  Returns (len(ids), P, B)."""
    ids = np.asarray(ids, dtype=np.int64)
    nb = neigh[ids].ravel()
    allids = np.unique(np.concatenate([ids, nb[nb >= 0]]))
    pos = {int(g): i for i, g in enumerate(allids)}
    D = predictor(rm, star[allids], Q[allids])
    I = time_integral(rm.N, D, dt)
    loc = np.array([pos[int(g)] for g in ids])
    Iown = I[loc]
    dv = volume(rm, star[ids], Iown)
    dl = local_flux(rm, Aplus[ids], Iown)
    nloc = np.array([[pos[int(v)] if v >= 0 else -1 for v in row] for row in neigh[ids]], dtype=np.int32)
    dn = neighbour_flux(rm, Aminus[ids], I, nloc, nface[ids], orient[ids])
    return Q[ids] + dv + dl + dn


# ----------------------------------------------------------------------------
# Brute force: the fully expanded multi-index sums (paper Sec. 4.2, the
# generic tensor-operation formula U_i = sum_j prod_k T^k), pure Python.
# ----------------------------------------------------------------------------
def brute_derivative(Kt, star, Dd):
    """One recursion step for one element: returns D^{d+1}[p][k]."""
    B = len(Kt[0])
    P = len(star[0])
    out = [[0.0] * B for _ in range(P)]
    for k in range(B):
        for p in range(P):
            s = 0.0
            for xi in range(3):
                for l in range(B):
                    for q in range(P):
                        s += Kt[xi][k][l] * Dd[q][l] * star[xi][p][q]
            out[p][k] = s
    return out


def brute_time_integral(N, D, dt):
    P, B = len(D[0]), len(D[0][0])
    return [[sum(dt ** (d + 1) / factorial(d + 1) * D[d][p][k] for d in range(N + 1))
             for k in range(B)] for p in range(P)]


def brute_volume(Kh, star, I):
    return brute_derivative(Kh, star, I)


def brute_face(Rh, F, R, I, A):
    """sum_{k,m,n,l,q} Rh_km F_mn R_ln I_lq A_pq for one face (F may be None)."""
    B, Bf = len(Rh), len(Rh[0])
    P = len(A)
    out = [[0.0] * B for _ in range(P)]
    for k in range(B):
        for p in range(P):
            s = 0.0
            for m in range(Bf):
                for n in range(Bf):
                    fmn = (1.0 if m == n else 0.0) if F is None else F[m][n]
                    if fmn == 0.0:
                        continue
                    for l in range(B):
                        for q in range(P):
                            s += Rh[k][m] * fmn * R[l][n] * I[q][l] * A[p][q]
            out[p][k] = s
    return out
