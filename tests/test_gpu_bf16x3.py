"""GPU parity of the split-BF16 matrix-core form (DG_BF16X3) through the C ABI
against the FP64 oracle on the same seeded inputs.

Bar: the step increment Q^{n+1} - Q^n (and several steps' increment) within
1e-4 relative, both in the per-quantity Frobenius metric and in the
per-element metric of dgtest.  Derivation: one split product
a b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi drops a_lo b_lo and the two lo
representation errors, at most 3 * 2^-16 = 4.6e-5 of |a||b| (bf16 keeps 8
significant bits, so |x - x_hi| <= 2^-8 |x| and |x - x_hi - x_lo| <= 2^-16 |x|);
FP32 accumulation adds about K * 2^-24 for K terms (K <= 84), and the flux
products run in FP64.  A step chains at most N+1 such contractions whose
errors add, against increments of the size of their largest terms, so 1e-4
is the stated bound per step; the measured values are printed.
"""
import sys

import numpy as np
import pytest

import dgtest
from dgtest import assert_close
from oracle import refmat, stages

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_B = 1e-4
BF = 3   # DG_BF16X3


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def _host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy() if t.is_floating_point() else t.cpu().numpy()


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _r32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _run(dg, plan, mesh, mats, Q, dt, n_steps):
    star, Ap, Am = dg.element_data(mesh.X, mats, mesh.neigh)
    E = mesh.E
    Qg = _dev(Q, torch.float32)
    I = torch.empty(plan.dof_shape(E), dtype=torch.float32, device="cuda:0")
    tr = torch.empty(plan.trace_shape(E), dtype=torch.float32, device="cuda:0")
    plan.step(Qg, I, tr, plan.pack_star(_dev(star)), _dev(Ap), _dev(Am), _dev(mesh.neigh),
              _dev(mesh.face_rot), dt, n_steps)
    return _host(Qg)


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6])
def test_bf16x3_steps_all_degrees(N):
    """One and three steps on a relabelled 162-element mesh (all 12
    neighbour face/orientation cases, a ragged last tile of 2 elements)."""
    import paper_1903_11521_amd as dg
    _say(f"test_bf16x3_steps_all_degrees N={N}")
    mesh, mats, Q, dt = dgtest.mesh_inputs(3, N, 40 + N, relabel=True)
    rm = refmat.refmats(N)
    ostar, oAp, oAm = dgtest.oracle_element_data(mesh, mats)
    plan = dg.Plan(N, BF)
    Q0 = _r32(Q)
    ref = Q0.copy()
    for k in range(3):
        ref = stages.step(rm, dt, ref, ostar, oAp, oAm, mesh.neigh, mesh.nface, mesh.orient)
        if k == 0:
            ref1 = ref.copy()
    Q1 = _run(dg, plan, mesh, mats, Q, dt, 1)
    assert_close(Q1 - Q0, ref1 - Q0, TOL_B, "degree %d step increment" % N)
    Q3 = _run(dg, plan, mesh, mats, Q, dt, 3)
    assert_close(Q3 - Q0, ref - Q0, TOL_B, "degree %d 3-step increment" % N)


def test_bf16x3_config0():
    """One step of the 3072-element degree-3 workload (8x8x8x6 jittered
    periodic mesh, random materials)."""
    import paper_1903_11521_amd as dg
    _say("test_bf16x3_config0")
    N = 3
    mesh, mats, Q, dt = dgtest.mesh_inputs(8, N, 0)
    ostar, oAp, oAm = dgtest.oracle_element_data(mesh, mats)
    Q0 = _r32(Q)
    ref = stages.step(refmat.refmats(N), dt, Q0, ostar, oAp, oAm, mesh.neigh, mesh.nface, mesh.orient)
    Q1 = _run(dg, dg.Plan(N, BF), mesh, mats, Q, dt, 1)
    assert_close(Q1 - Q0, ref - Q0, TOL_B, "step increment")


@pytest.mark.parametrize("E", [1, 15, 16, 17, 33])
def test_bf16x3_edge_sizes(E):
    """Tile edges (one element, one short of a tile, one tile, one past, two
    tiles and one past), random neighbour tables with faces without a
    neighbour (-1), random star and flux-solver matrices."""
    import paper_1903_11521_amd as dg
    _say(f"test_bf16x3_edge_sizes E={E}")
    N = 4
    d = dgtest.random_stage_inputs(N, E, seed=70 + E)
    neigh = d["neigh"].copy()
    neigh[0, 1] = -1
    if E > 2:
        neigh[E - 1, 3] = -1
    rm = refmat.refmats(N)
    Q0 = _r32(d["Q"])
    star = _r32(d["star"])
    ref = stages.step(rm, 0.05, Q0, star, d["Ap"], d["Am"], neigh, d["nface"], d["orient"])
    plan = dg.Plan(N, BF)
    Qg = _dev(d["Q"], torch.float32)
    I = torch.empty(plan.dof_shape(E), dtype=torch.float32, device="cuda:0")
    tr = torch.empty(plan.trace_shape(E), dtype=torch.float32, device="cuda:0")
    plan.step(Qg, I, tr, plan.pack_star(_dev(d["star"])), _dev(d["Ap"]), _dev(d["Am"]), _dev(neigh),
              _dev(d["face_rot"]), 0.05, 1)
    assert_close(_host(Qg) - Q0, ref - Q0, TOL_B, "step increment E=%d" % E)


def test_bf16x3_split_launches_equal_step():
    """dg_step_predict + dg_step_correct is bitwise dg_step (degree 5, 2 steps)."""
    import paper_1903_11521_amd as dg
    _say("test_bf16x3_split_launches_equal_step")
    N = 5
    mesh, mats, Q, dt = dgtest.mesh_inputs(3, N, 9, relabel=True)
    plan = dg.Plan(N, BF)
    star, Ap, Am = dg.element_data(mesh.X, mats, mesh.neigh)
    E = mesh.E
    args = [plan.pack_star(_dev(star)), _dev(Ap), _dev(Am), _dev(mesh.neigh), _dev(mesh.face_rot)]
    Qa, Qb = _dev(Q, torch.float32), _dev(Q, torch.float32)
    Ia, Ib = (torch.empty(plan.dof_shape(E), dtype=torch.float32, device="cuda:0") for _ in range(2))
    ta, tb = (torch.empty(plan.trace_shape(E), dtype=torch.float32, device="cuda:0") for _ in range(2))
    plan.step(Qa, Ia, ta, *args, dt, 2, traces_b=torch.empty_like(ta))
    for _ in range(2):
        plan.step_predict(Qb, args[0], dt, Ib, tb)
        plan.step_correct(Ib, tb, *args, Qb)
    assert torch.equal(Qa, Qb) and torch.equal(Ia, Ib) and torch.equal(ta, tb)


def test_bf16x3_unsupported_calls():
    """The per-stage calls, the fused launch and batches are refused for this
    form (synchronously, nothing enqueued)."""
    import paper_1903_11521_amd as dg
    plan = dg.Plan(3, BF)
    E = 4
    Q = torch.zeros(plan.dof_shape(E), dtype=torch.float32, device="cuda:0")
    with pytest.raises(dg.DGError, match="not available"):
        plan.volume(Q, torch.zeros((E, 9, 3, 3), dtype=torch.float32, device="cuda:0"), Q)
    with pytest.raises(dg.DGError):
        plan.set_fusion(True)
    assert plan.tune(E=128) is False
