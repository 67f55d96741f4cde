"""dg_step_noalloc (face traces in the library's fixed device buffer, no
device allocation) against dg_step through the C ABI.

Both run the same kernels on the same data, so the bar is bit-for-bit
equality of Q and I (the FP64 oracle bar of 1e-12 is then implied by dg_step's
own parity tests).  Two calls in a row on one device, the second with a
smaller mesh, so the second call runs over the first call's leftover traces;
and a call above the buffer's capacity is refused before anything runs.
"""
import sys

import numpy as np
import pytest

import dgtest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run_pair(plan, n, seed_index, n_steps):
    """dg_step (caller's trace arrays, two of them) and dg_step_noalloc on
    the same mesh; returns (Q, I) of both."""
    import paper_1903_11521_amd as dg
    mesh, mats, Q, dt = dgtest.mesh_inputs(n, plan.degree, seed_index, relabel=True)
    star, Ap, Am = dg.element_data(mesh.X, mats, mesh.neigh)
    E = mesh.E
    assert E <= plan.noalloc_max_elements()
    args = [plan.pack_star(_dev(star)), _dev(Ap), _dev(Am), _dev(mesh.neigh), _dev(mesh.face_rot)]
    Qa, Qb = _dev(Q).to(plan.dtype), _dev(Q).to(plan.dtype)
    Ia, Ib = (torch.empty(plan.dof_shape(E), dtype=plan.dtype, device="cuda:0") for _ in range(2))
    ta, tb = (torch.empty(plan.trace_shape(E), dtype=plan.dtype, device="cuda:0") for _ in range(2))
    plan.step(Qa, Ia, ta, *args, dt, n_steps, traces_b=tb)
    plan.step_noalloc(Qb, Ib, *args, dt, n_steps)
    plan.sync()
    return Qa, Ia, Qb, Ib


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
@pytest.mark.parametrize("N", [3, 5])
def test_noalloc_equals_step_twice_shrinking(N, prec):
    import paper_1903_11521_amd as dg
    _say(f"test_noalloc_equals_step_twice_shrinking N={N} prec={prec}")
    plan = dg.Plan(N, prec)
    # first call: 6*5^3 = 750 elements, 3 steps; second: 6*3^3 = 162, 2 steps
    for n, seed, steps in ((5, 21, 3), (3, 22, 2)):
        _say(f"  mesh n={n} E={6 * n ** 3} steps={steps}")
        Qa, Ia, Qb, Ib = _run_pair(plan, n, seed, steps)
        assert torch.equal(Qa, Qb), "Q differs from dg_step"
        assert torch.equal(Ia, Ib), "I differs from dg_step"


def test_noalloc_both_schedules():
    """The fused (one launch per step) and the two-launch schedule both go
    through the fixed buffer and give dg_step's result."""
    import paper_1903_11521_amd as dg
    _say("test_noalloc_both_schedules")
    for fused in (True, False):
        plan = dg.Plan(4, 0)
        plan.set_fusion(fused)
        Qa, Ia, Qb, Ib = _run_pair(plan, 4, 23, 3)
        assert torch.equal(Qa, Qb) and torch.equal(Ia, Ib)


def test_noalloc_rejects_above_capacity():
    """E one above the capacity: DG_EINVAL with the limit in the message,
    and Q untouched (nothing was enqueued)."""
    import paper_1903_11521_amd as dg
    _say("test_noalloc_rejects_above_capacity")
    plan = dg.Plan(6, 0)
    E = plan.noalloc_max_elements() + 1
    assert E == (256 << 20) // (4 * 9 * 28 * 8) + 1
    Q = torch.ones(plan.dof_shape(E), dtype=torch.float64, device="cuda:0")
    I = torch.empty_like(Q)
    star = torch.zeros((E, 9, 3, 3), dtype=torch.float64, device="cuda:0")
    A = torch.zeros((E, 4, 9, 9), dtype=torch.float64, device="cuda:0")
    neigh = torch.full((E, 4), -1, dtype=torch.int32, device="cuda:0")
    rot = torch.zeros((E, 4), dtype=torch.uint8, device="cuda:0")
    with pytest.raises(dg.DGError, match="fixed scratch"):
        plan.step_noalloc(Q, I, star, A, A, neigh, rot, 1e-3, 1)
    plan.sync()
    assert bool(torch.all(Q == 1.0))
