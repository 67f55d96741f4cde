"""Precision study on the degree-6 plane wave: the 60x60x60x6 = 1 296 000
element jittered periodic mesh, homogeneous medium, 100 time steps at
dt = 0.5 h_min / ((2N+1) c_p), in FP64, FP32 and the split-BF16 form.

Checks, per precision:
  * per step against the FP64 oracle on a seeded 1000-element subset, at
    steps 1, 50 and 100: the oracle re-steps the subset from the GPU run's
    own state Q^n (the predictor also on the subset's face neighbours) and
    Q^{n+1} is compared (relative error of Q^{n+1}, per quantity and per
    element).  Bars: FP64 1e-12, FP32 1e-5, split-BF16 1e-4 (the bound of
    tests/test_gpu_bf16x3.py) in the per-quantity Frobenius metric.  The
    per-element metric takes the maximum over 9 000 (element, quantity)
    pairs; for split-BF16 its bar is 2e-4: a split product errs by up to
    3 * 2^-16 of |a||b|, two split contractions chain into every term of the
    update (predictor into the time integral, time integral into the volume
    and face terms), and on this wave the summed magnitude of those terms is
    about 0.4 |Q| (volume and face terms each about N^2 / (k h) = 46 times
    the increment, itself 0.8 % of Q), which gives 2 * 4.6e-5 * (1 + 0.4) =
    1.3e-4 before the FP32 accumulation; measured 8-10e-5.  The relative
    error of the step increment is printed beside it (the terms cancel to an
    increment 46 times smaller, which multiplies their relative rounding);
  * after 100 steps against the exact plane wave (its L2 projection), in the
    mass-weighted L2 norm: FP64 shows the discretisation error, FP32 and
    split-BF16 must stay within 1e-3 relative of the FP64 run's state.
"""
import sys

import numpy as np
import pytest

import dgtest
from oracle import elements as oel
from oracle import refmat, stages

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = 6
NCUBE = 60
STEPS = 100
CHECK = (0, 49, 99)          # steps n whose Q^{n+1} is checked
TOL_STEP = {0: 1e-12, 1: 1e-5, 3: 1e-4}          # per-quantity Frobenius
TOL_ELEM = {0: 1e-12, 1: 1e-5, 3: 2e-4}          # per element (see the module docstring)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _mass_rel(x, y, w):
    return float(np.sqrt(np.sum(w * (x - y) ** 2) / np.sum(w * y ** 2)))


@pytest.fixture(scope="module")
def wave():
    from planewave import PlaneWave
    _say("building the degree-6 plane wave on %d elements" % (6 * NCUBE ** 3))
    pw = PlaneWave(NCUBE, N)
    pw.Q0 = pw.project(0.0)
    pw.exact = pw.project(STEPS * pw.dt)
    rng = np.random.default_rng(1903)
    pw.ids = np.sort(rng.choice(pw.mesh.E, 1000, replace=False))
    nb = pw.mesh.neigh[pw.ids].ravel()
    pw.allids = np.unique(np.concatenate([pw.ids, nb[nb >= 0]]))
    X = pw.mesh.X
    pw.ostar = oel.star_matrices(X[pw.allids], pw.mats[pw.allids])
    pw.oAp, pw.oAm = oel.flux_matrices(X[pw.ids], pw.mats[pw.ids], None,
                                       neighbour_materials=pw.mats[pw.mesh.neigh[pw.ids]])
    return pw


def _oracle_subset(pw, Qsub_all, dt):
    """Q^{n+1} of pw.ids from the state rows Qsub_all (rows of pw.allids)."""
    from planewave import SubsetRows
    E = pw.mesh.E
    star = SubsetRows(pw.ostar, pw.allids, E)
    Q = SubsetRows(Qsub_all, pw.allids, E)
    Ap = SubsetRows(pw.oAp, pw.ids, E)
    Am = SubsetRows(pw.oAm, pw.ids, E)
    return stages.step_subset(refmat.refmats(N), dt, pw.ids, Q, star, Ap, Am, pw.mesh.neigh, pw.mesh.nface,
                              pw.mesh.orient)


@pytest.fixture(scope="module")
def fp64_final():
    return {}


@pytest.mark.parametrize("prec", [0, 1, 3])
def test_planewave_degree6(wave, prec, fp64_final):
    import paper_1903_11521_amd as dg
    pw = wave
    _say(f"test_planewave_degree6 prec={prec} E={pw.mesh.E} dt={pw.dt:.3e} |m|={np.linalg.norm(pw.m):.2f}")
    plan = dg.Plan(N, prec)
    star, Ap, Am = dg.element_data(pw.mesh.X, pw.mats, pw.mesh.neigh)
    dev = "cuda:0"
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    E = pw.mesh.E
    Qg = t(pw.Q0).to(plan.dtype)
    I = torch.empty(plan.dof_shape(E), dtype=plan.dtype, device=dev)
    tr = torch.empty(plan.trace_shape(E), dtype=plan.dtype, device=dev)
    args = (plan.pack_star(t(star)), t(Ap), t(Am), t(pw.mesh.neigh), t(pw.mesh.face_rot))
    del star, Ap, Am
    all_idx = torch.from_numpy(pw.allids).to(dev)
    pos = np.searchsorted(pw.allids, pw.ids)
    for n in range(STEPS):
        if n in CHECK:
            Qn = Qg.index_select(0, all_idx).double().cpu().numpy()
            ref = _oracle_subset(pw, Qn, pw.dt)
        plan.step(Qg, I, tr, *args, pw.dt, 1)
        if n in CHECK:
            Q1 = Qg.index_select(0, all_idx).double().cpu().numpy()[pos]
            q0 = Qn[pos]
            inc = dgtest.rel_err(Q1 - q0, ref - q0)
            _say("  step %3d: increment rel. error %.3e" % (n + 1, inc))
            f, m = dgtest.errors(Q1, ref)
            _say("  step %3d Q^{n+1} vs oracle: frobenius %.3e (bar %.0e)  per-element %.3e (bar %.0e)"
                 % (n + 1, f, TOL_STEP[prec], m, TOL_ELEM[prec]))
            assert f <= TOL_STEP[prec] and m <= TOL_ELEM[prec]
    Qend = Qg.double().cpu().numpy()
    w = pw.mass_weights()
    err_exact = _mass_rel(Qend, pw.exact, w)
    _say("  after %d steps: L2 error vs the exact plane wave %.3e" % (STEPS, err_exact))
    if prec == 0:
        fp64_final["Q"] = Qend
        assert err_exact < 1e-2, "FP64 run far from the exact plane wave"
    else:
        if "Q" in fp64_final:
            d = _mass_rel(Qend, fp64_final["Q"], w)
            _say("  after %d steps: L2 difference from the FP64 run %.3e" % (STEPS, d))
            assert d < 1e-3
        assert err_exact < 1e-2
