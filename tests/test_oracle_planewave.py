"""Oracle pin: convergence on a smooth exact solution.

ADER-DG of degree N is accurate of order N+1 in space and time for smooth
solutions (the paper's plane-wave validation, Sec. 5).  The oracle's full
step (predictor, time integral, volume, local and neighbour flux with the
exact Godunov flux) is run on the periodic plane wave of tests/planewave.py
(wave vector 2 pi (1, 1, 0), homogeneous medium) on jittered meshes with
n = 8 and n = 16 cubes per direction, to the same final time with dt
proportional to h; the mass-weighted L2 error against the exact wave must
fall by close to 2^(N+1) (measured orders 2.85 at degree 2 and 3.83 at
degree 3; they approach N+1 from below as the mesh is refined).  A dropped term, a wrong sign or a transposed
operand anywhere in the step destroys the convergence.
"""
import numpy as np
import pytest

from oracle import elements as oel
from oracle import refmat, stages


def _error(n, N, T, steps):
    from planewave import PlaneWave
    pw = PlaneWave(n, N, m=(1, 1, 0))
    dt = T / steps
    assert dt <= pw.dt
    Q = pw.project(0.0, device="cpu", chunk=2048)
    exact = pw.project(T, device="cpu", chunk=2048)
    star = oel.star_matrices(pw.mesh.X, pw.mats)
    Ap, Am = oel.flux_matrices(pw.mesh.X, pw.mats, pw.mesh.neigh)
    rm = refmat.refmats(N)
    for _ in range(steps):
        Q = stages.step(rm, dt, Q, star, Ap, Am, pw.mesh.neigh, pw.mesh.nface, pw.mesh.orient)
    w = pw.mass_weights()
    return float(np.sqrt(np.sum(w * (Q - exact) ** 2) / np.sum(w * exact ** 2)))


@pytest.mark.parametrize("N", [2, 3])
def test_plane_wave_convergence_order(N):
    pytest.importorskip("torch")
    from planewave import PlaneWave
    # the same final time on both meshes, dt halved with h (below both
    # meshes' stability limit 0.5 h_min / ((2N+1) c_p))
    T = 16 * 0.9 * PlaneWave(8, N, m=(1, 1, 0)).dt
    e8 = _error(8, N, T, 16)
    e16 = _error(16, N, T, 32)
    order = np.log2(e8 / e16)
    print("degree %d: L2 errors %.3e (n=8) %.3e (n=16), observed order %.2f" % (N, e8, e16, order))
    assert e16 < e8
    assert order > N + 1 - 0.3
