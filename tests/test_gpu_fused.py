"""GPU parity of the fused-simulation step (dg_fused_step, 16 simulations per
element on the matrix cores; the extra simulation index s of Sec. 3 and
5.1.1) through the C ABI.

  * Each simulation's result equals, bit for bit, dg_step of the same
    split-BF16 plan on that simulation's DOFs alone (same arithmetic per
    MFMA column and per lane; the fused tiling only shares the element data).
  * Every simulation matches the FP64 oracle stepped on it (the fused form's
    definition: independent simulations under the same operators) within the
    split-BF16 bar of 1e-4 on the step increment (tests/test_gpu_bf16x3.py).
"""
import sys

import numpy as np
import pytest

import dgtest
from dgtest import assert_close
from oracle import refmat, stages

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

S = 16
BF = 3


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6])
def test_fused_equals_single_and_oracle(N):
    import paper_1903_11521_amd as dg
    from workload import random_dofs, seed_for
    _say(f"test_fused_equals_single_and_oracle N={N}")
    mesh, mats, _, dt = dgtest.mesh_inputs(3, N, 60 + N, relabel=True)
    E = mesh.E
    plan = dg.Plan(N, BF)
    B = plan.B
    Qs = np.stack([random_dofs(E, 9, B, seed_for(700 + s)) for s in range(S)], axis=-1)   # (E, 9, B, S)
    Qs = Qs.astype(np.float32).astype(np.float64)
    star, Ap, Am = dg.element_data(mesh.X, mats, mesh.neigh)
    args = [plan.pack_star(_dev(star)), _dev(Ap), _dev(Am), _dev(mesh.neigh), _dev(mesh.face_rot)]
    Qf = _dev(Qs, torch.float32)
    If = torch.empty(plan.fused_dof_shape(E), dtype=torch.float32, device="cuda:0")
    tf = torch.empty(plan.fused_trace_shape(E), dtype=torch.float32, device="cuda:0")
    steps = 2
    plan.fused_step(Qf, If, tf, *args, dt, steps)
    I = torch.empty(plan.dof_shape(E), dtype=torch.float32, device="cuda:0")
    tr = torch.empty(plan.trace_shape(E), dtype=torch.float32, device="cuda:0")
    for s in range(S):
        q = _dev(Qs[..., s], torch.float32)
        plan.step(q, I, tr, *args, dt, steps)
        assert torch.equal(Qf[..., s], q), "simulation %d differs from dg_step" % s
        assert torch.equal(If[..., s], I), "simulation %d: time integral differs" % s
    Q2 = Qf.double().cpu().numpy()
    rm = refmat.refmats(N)
    ostar, oAp, oAm = dgtest.oracle_element_data(mesh, mats)
    for s in (0, 7, 15):
        ref = Qs[..., s]
        for _ in range(steps):
            ref = stages.step(rm, dt, ref, ostar, oAp, oAm, mesh.neigh, mesh.nface, mesh.orient)
        assert_close(Q2[..., s] - Qs[..., s], ref - Qs[..., s], 1e-4,
                     "degree %d simulation %d, %d-step increment" % (N, s, steps))


def test_fused_refused_for_other_precisions():
    import paper_1903_11521_amd as dg
    plan = dg.Plan(3, dg.DG_FP32)
    E = 2
    z = lambda *sh, dt=torch.float32: torch.zeros(sh, dtype=dt, device="cuda:0")
    with pytest.raises(dg.DGError, match="fused"):
        plan.fused_step(z(*plan.fused_dof_shape(E)), z(*plan.fused_dof_shape(E)), z(*plan.fused_trace_shape(E)),
                        z(E, 9, 3, 3), z(E, 4, 9, 9, dt=torch.float64), z(E, 4, 9, 9, dt=torch.float64),
                        z(E, 4, dt=torch.int32), z(E, 4, dt=torch.uint8), 1e-3, 1)
