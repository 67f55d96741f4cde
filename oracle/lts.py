"""Oracle of clustered local time stepping (test infrastructure only).

The paper reports time-to-solution with local time stepping (Sec. 6.4, Table
tab:loh1: GTS against LTS) and gives no equations for it.  Reading (clustered
LTS of rate 2): element e belongs to cluster c_e and steps with
dt_c = 2^c dt0; face neighbours differ by at most one cluster.  Each step of an
element is the ADER step of Sec. 5.1.1 with one change: in the neighbour term
(Eq. seissol:correction_neigh) the neighbour's time integral is taken over
the receiving element's own step interval.  A neighbour's predicted solution
in time is piecewise: over each of its own steps it is the Taylor expansion of
its predictor (Eq. seissol:derivative) about that step's start.  The integral
over the receiver's interval sums the pieces that overlap it.

This module evaluates exactly that definition, plainly: it keeps every
element's pieces and integrates the overlaps.  Time advances in ticks of
dt0.  At tick tau the clusters with tau % 2^c == 0 predict from their current
state; then the clusters whose step ends at tau + 1 are corrected (the
corrections read predictions only, never another element's new state).
"""
from __future__ import annotations

from math import factorial

import numpy as np

from . import stages


def piece_integral(D, lo, hi):
    """Integral over local time u in [lo, hi] of sum_d D^d u^d / d!
    (D: (..., N+1, P, B), u measured from the piece's start)."""
    N1 = D.shape[-3]
    w = np.array([(hi ** (d + 1) - lo ** (d + 1)) / factorial(d + 1) for d in range(N1)])
    return np.einsum("d,...dpb->...pb", w, D)


def run(rm, cluster, dt0, Q, star, Aplus, Aminus, neigh, nface, orient, n_cycles):
    """Advances Q by n_cycles cycles of 2^(C-1) ticks (C = number of
    clusters, the largest cluster takes one step per cycle).  Returns Q."""
    cluster = np.asarray(cluster, dtype=np.int64)
    C = int(cluster.max()) + 1
    ticks = n_cycles * 2 ** (C - 1)
    E = Q.shape[0]
    Q = np.array(Q, dtype=np.float64, copy=True)
    members = [np.nonzero(cluster == c)[0] for c in range(C)]
    # pieces[e] = list of (start tick, length in ticks, D^0..D^N)
    pieces = [[] for _ in range(E)]
    for tau in range(ticks):
        for c in range(C):
            ids = members[c]
            if tau % 2 ** c == 0 and len(ids):
                D = stages.predictor(rm, star[ids], Q[ids])
                for i, e in enumerate(ids):
                    pieces[e].append((tau, 2 ** c, D[i]))
        for c in range(C):
            ids = members[c]
            if (tau + 1) % 2 ** c != 0 or not len(ids):
                continue
            a, b = tau + 1 - 2 ** c, tau + 1            # receiver interval in ticks
            J = np.zeros_like(Q)
            nb = neigh[ids].ravel()
            for v in np.unique(np.concatenate([ids, nb[nb >= 0]])):
                for (s, n, D) in pieces[v]:
                    lo, hi = max(a, s), min(b, s + n)
                    if hi > lo:
                        J[v] += piece_integral(D, (lo - s) * dt0, (hi - s) * dt0)
            Iown = J[ids]                              # own piece covers [a, b] exactly
            dQ = (stages.volume(rm, star[ids], Iown) + stages.local_flux(rm, Aplus[ids], Iown)
                  + stages.neighbour_flux(rm, Aminus[ids], J, neigh[ids], nface[ids], orient[ids]))
            Q[ids] += dQ
    return Q
