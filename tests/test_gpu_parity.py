"""GPU parity: every stage and the full step through the C ABI against the
FP64 oracle on the same seeded inputs.

Bars (both the per-quantity Frobenius metric and the per-element metric of
dgtest must pass): FP64 1e-12, FP32 and mixed 1e-5, for every stage (each
derivative order of the predictor, the time integral, the volume, local and
neighbour flux increments), for Q after one or more full steps, and for the
full-step increment Q^{n+1} - Q^n (relative to the increment).
"""
import math
import sys

import numpy as np
import pytest

import dgtest
from dgtest import assert_close
from oracle import refmat, stages

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5, 2: 1e-5}
TOL_INC = TOL                               # full-step increments: the same bars


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def _host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy() if t.is_floating_point() else t.cpu().numpy()


def _plan(N, prec):
    import paper_1903_11521_amd as dg
    return dg.Plan(N, prec)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rounded(Q, prec):
    """The initial DOFs as the GPU holds them (FP32 plans round once)."""
    return Q.astype(np.float32).astype(np.float64) if prec else Q


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("N,E", [(2, 30), (3, 52), (4, 17), (5, 52), (6, 23)])
def test_stages(N, E, prec):
    _say(f"test_stages N={N} E={E} prec={prec}")
    d = dgtest.random_stage_inputs(N, E, seed=100 + N)
    rm = refmat.refmats(N)
    plan = _plan(N, prec)
    dt = 0.13
    tol = TOL[prec]
    fdt = plan.dtype
    star_p = plan.pack_star(_dev(d["star"]))
    # predictor (Taylor-scaled derivatives), every order at the stage bar
    T = plan.predictor(_dev(d["Q"], fdt), star_p, dt)
    D = stages.predictor(rm, d["star"], d["Q"])
    scale = np.array([dt ** k / math.factorial(k) for k in range(N + 1)])
    Tref = D * scale[None, :, None, None]
    Tg = _host(T)
    for k in range(N + 1):
        assert_close(Tg[:, k], Tref[:, k], tol, f"derivative {k}")
    # time integral from the oracle's derivatives
    I = plan.time_integral(_dev(Tref, fdt), dt)
    assert_close(_host(I), stages.time_integral(N, D, dt), tol, "time integral")
    # update stages as increments on Q = 0
    Iin = _dev(d["I"], fdt)
    zero = lambda: torch.zeros(plan.dof_shape(E), dtype=fdt, device="cuda:0")
    q = plan.volume(Iin, star_p, zero())
    assert_close(_host(q), stages.volume(rm, d["star"], d["I"]), tol, "volume")
    q = plan.local_flux(Iin, _dev(d["Ap"]), zero())
    assert_close(_host(q), stages.local_flux(rm, d["Ap"], d["I"]), tol, "local flux")
    q = plan.neighbour_flux(Iin, _dev(d["neigh"]), _dev(d["face_rot"]), _dev(d["Am"]), zero())
    ref = stages.neighbour_flux(rm, d["Am"], d["I"], d["neigh"], d["nface"], d["orient"])
    assert_close(_host(q), ref, tol, "neighbour flux")
    # add-to-Q path with a non-zero Q: Q + volume, compared as Q^{n+1}
    Q0 = _dev(d["Q"], fdt)
    plan.volume(Iin, star_p, Q0)
    assert_close(_host(Q0), _rounded(d["Q"], prec) + stages.volume(rm, d["star"], d["I"]), tol, "Q + volume")


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("N,E", [(3, 29), (5, 52)])
def test_time_integral_reads_only_the_staircase(N, E, prec):
    """dg_time_integral takes the rows of T^d at and past C(N-d+3, 3) as the
    zeros the predictor leaves there: with those rows filled with noise the
    result is the oracle's on the staircase-truncated T (stage bar)."""
    _say(f"test_time_integral_reads_only_the_staircase N={N} E={E} prec={prec}")
    rng = np.random.default_rng(700 + N)
    B = refmat.n_basis(N)
    T = rng.standard_normal((E, N + 1, 9, B))
    Tz = T.copy()
    for d in range(N + 1):
        Tz[:, d, :, refmat.n_basis(N - d):] = 0.0
    plan = _plan(N, prec)
    dt = 0.07
    I = plan.time_integral(_dev(T, plan.dtype), dt)
    D = Tz / np.array([dt ** k / math.factorial(k) for k in range(N + 1)])[None, :, None, None]
    assert_close(_host(I), stages.time_integral(N, D, dt), TOL[prec], "time integral")


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_step_config0(prec):
    """One full time step on the 8x8x8x6 = 3072-element jittered periodic mesh,
    degree 3, random materials; element data built by the library itself."""
    import paper_1903_11521_amd as dg
    N = 3
    _say(f"test_step_config0 prec={prec}")
    mesh, mats, Q, dt = dgtest.mesh_inputs(8, N, 0)
    E = mesh.E
    rm = refmat.refmats(N)
    ostar, oAp, oAm = dgtest.oracle_element_data(mesh, mats)
    ref = stages.step(rm, dt, Q, ostar, oAp, oAm, mesh.neigh, mesh.nface, mesh.orient)
    plan = dg.Plan(N, prec)
    star, Ap, Am = dg.element_data(mesh.X, mats, mesh.neigh)
    Qg = _dev(Q, plan.dtype)
    I = torch.empty(plan.dof_shape(E), dtype=plan.dtype, device="cuda:0")
    tr = torch.empty(plan.trace_shape(E), dtype=plan.dtype, device="cuda:0")
    plan.step(Qg, I, tr, plan.pack_star(_dev(star)), _dev(Ap), _dev(Am), _dev(mesh.neigh),
              _dev(mesh.face_rot), dt, 1)
    Q1 = _host(Qg)
    assert_close(Q1 - _rounded(Q, prec), ref - Q, TOL_INC[prec], "step increment")
    assert_close(Q1, ref, TOL[prec], "Q^{n+1}")


@pytest.mark.parametrize("fused", [False, True])
def test_step_multi_relabelled_degree5(fused):
    """Three steps on a mesh with all 12 neighbour face/orientation cases
    (fused: one launch per step, traces alternating between two arrays)."""
    import paper_1903_11521_amd as dg
    N = 5
    _say(f"test_step_multi_relabelled_degree5 fused={fused}")
    mesh, mats, Q, dt = dgtest.mesh_inputs(4, N, 2, relabel=True)
    rm = refmat.refmats(N)
    ostar, oAp, oAm = dgtest.oracle_element_data(mesh, mats)
    ref = Q.copy()
    for _ in range(3):
        ref = stages.step(rm, dt, ref, ostar, oAp, oAm, mesh.neigh, mesh.nface, mesh.orient)
    plan = dg.Plan(N, 0)
    if fused:
        plan.set_fusion(True)
    star, Ap, Am = dg.element_data(mesh.X, mats, mesh.neigh)
    E = mesh.E
    Qg = _dev(Q)
    I = torch.empty(plan.dof_shape(E), dtype=plan.dtype, device="cuda:0")
    tr = torch.empty(plan.trace_shape(E), dtype=plan.dtype, device="cuda:0")
    plan.step(Qg, I, tr, plan.pack_star(_dev(star)), _dev(Ap), _dev(Am), _dev(mesh.neigh),
              _dev(mesh.face_rot), dt, 3, traces_b=torch.empty_like(tr) if fused else None)
    assert_close(_host(Qg) - Q, ref - Q, 1e-12, "3-step increment")


@pytest.mark.parametrize("E", [0, 1, 7, 8])
def test_edge_sizes(E):
    """Empty input, a single element (its own neighbour), one exact wave, one
    element past a wave; faces without neighbour (-1) contribute nothing."""
    N = 3
    _say(f"test_edge_sizes E={E}")
    plan = _plan(N, 0)
    rm = refmat.refmats(N)
    if E == 0:
        Q = torch.zeros((0, 9, plan.B), dtype=torch.float64, device="cuda:0")
        I = torch.zeros_like(Q)
        tr = torch.zeros(plan.trace_shape(0), dtype=torch.float64, device="cuda:0")
        z = lambda *s, dt=torch.float64: torch.zeros(s, dtype=dt, device="cuda:0")
        plan.step(Q, I, tr, z(0, 9, 3, 3), z(0, 4, 9, 9), z(0, 4, 9, 9), z(0, 4, dt=torch.int32),
                  z(0, 4, dt=torch.uint8), 0.1, 2)
        plan.sync()
        return
    d = dgtest.random_stage_inputs(N, E, seed=7 + E)
    neigh = d["neigh"].copy()
    neigh[0, 1] = -1
    if E > 2:
        neigh[E - 1, 3] = -1
    ref = stages.step(rm, 0.05, d["Q"], d["star"], d["Ap"], d["Am"], neigh, d["nface"], d["orient"])
    Qg = _dev(d["Q"])
    I = torch.empty(plan.dof_shape(E), dtype=torch.float64, device="cuda:0")
    tr = torch.empty(plan.trace_shape(E), dtype=torch.float64, device="cuda:0")
    args = (plan.pack_star(_dev(d["star"])), _dev(d["Ap"]), _dev(d["Am"]), _dev(neigh), _dev(d["face_rot"]))
    plan.step(Qg, I, tr, *args, 0.05, 1)
    assert_close(_host(Qg) - d["Q"], ref - d["Q"], 1e-12, "step increment")
    # two more steps, fused, against the oracle
    ref2 = ref
    for _ in range(2):
        ref2 = stages.step(rm, 0.05, ref2, d["star"], d["Ap"], d["Am"], neigh, d["nface"], d["orient"])
    plan.step(Qg, I, tr, *args, 0.05, 2, traces_b=torch.empty_like(tr))
    assert_close(_host(Qg) - ref, ref2 - ref, 1e-12, "fused 2-step increment")


def test_step_split_equals_step():
    """dg_step_predict + dg_step_correct is bitwise dg_step."""
    import paper_1903_11521_amd as dg
    N = 4
    mesh, mats, Q, dt = dgtest.mesh_inputs(4, N, 3)
    plan = dg.Plan(N, 0)
    star, Ap, Am = dg.element_data(mesh.X, mats, mesh.neigh)
    E = mesh.E
    args = [plan.pack_star(_dev(star)), _dev(Ap), _dev(Am), _dev(mesh.neigh), _dev(mesh.face_rot)]
    Qa, Qb = _dev(Q), _dev(Q)
    I = torch.empty(plan.dof_shape(E), dtype=torch.float64, device="cuda:0")
    tr = torch.empty(plan.trace_shape(E), dtype=torch.float64, device="cuda:0")
    plan.step(Qa, I, tr, *args, dt, 2)
    for _ in range(2):
        plan.step_predict(Qb, args[0], dt, I, tr)
        plan.step_correct(I, tr, args[0], args[1], args[2], args[3], args[4], Qb)
    assert torch.equal(Qa, Qb)


@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("N", [2, 3, 4, 5, 6])
def test_fused_step_equals_split(N, prec, fused):
    """dg_step with a second trace array is bitwise the sequence of
    dg_step_predict + dg_step_correct, for Q, I and the last step's traces,
    with odd and even step counts, with the launch schedule forced either way
    (fused: the one-launch kernel runs at every degree and precision)."""
    import paper_1903_11521_amd as dg
    _say(f"test_fused_step_equals_split N={N} prec={prec} fused={fused}")
    mesh, mats, Q, dt = dgtest.mesh_inputs(3, N, 11, relabel=True)
    plan = dg.Plan(N, prec)
    default = plan.fuses_steps
    assert default == (N <= 3)
    plan.set_fusion(fused)
    assert plan.fuses_steps == fused
    from paper_1903_11521_amd import _lib as L
    assert bool(L._load().dg_plan_fuses_steps(plan._h)) == fused
    star, Ap, Am = dg.element_data(mesh.X, mats, mesh.neigh)
    E = mesh.E
    args = [plan.pack_star(_dev(star)), _dev(Ap), _dev(Am), _dev(mesh.neigh), _dev(mesh.face_rot)]
    for n in (2, 3):
        Qa, Qb = _dev(Q).to(plan.dtype), _dev(Q).to(plan.dtype)
        Ia, Ib = (torch.empty(plan.dof_shape(E), dtype=plan.dtype, device="cuda:0") for _ in range(2))
        ta, tb, tc = (torch.empty(plan.trace_shape(E), dtype=plan.dtype, device="cuda:0") for _ in range(3))
        plan.step(Qa, Ia, ta, *args, dt, n, traces_b=tb)
        for _ in range(n):
            plan.step_predict(Qb, args[0], dt, Ib, tc)
            plan.step_correct(Ib, tc, args[0], args[1], args[2], args[3], args[4], Qb)
        assert torch.equal(Qa, Qb)
        assert torch.equal(Ia, Ib)
        assert torch.equal(ta, tc)
    # the exported launches: predict, fused (one launch or two, per plan), correct
    Qa, Qb = _dev(Q).to(plan.dtype), _dev(Q).to(plan.dtype)
    Ia, Ib = (torch.empty(plan.dof_shape(E), dtype=plan.dtype, device="cuda:0") for _ in range(2))
    ta, tb, tc = (torch.empty(plan.trace_shape(E), dtype=plan.dtype, device="cuda:0") for _ in range(3))
    plan.step_predict(Qa, args[0], dt, Ia, ta)
    plan.step_fused(Qa, Ia, ta, tb, *args, dt)
    plan.step_fused(Qa, Ia, tb, ta, *args, dt)
    plan.step_correct(Ia, ta, *args, Qa)
    for _ in range(3):
        plan.step_predict(Qb, args[0], dt, Ib, tc)
        plan.step_correct(Ib, tc, *args, Qb)
    assert torch.equal(Qa, Qb)
    assert torch.equal(ta, tc)
    if fused and prec == 0:
        # and the fused schedule against the oracle (3 steps)
        rm = refmat.refmats(N)
        ostar, oAp, oAm = dgtest.oracle_element_data(mesh, mats)
        ref = Q.copy()
        for _ in range(3):
            ref = stages.step(rm, dt, ref, ostar, oAp, oAm, mesh.neigh, mesh.nface, mesh.orient)
        assert_close(_host(Qa) - Q, ref - Q, 1e-12, "fused 3-step increment")


@pytest.mark.parametrize("N", [3, 5, 6])
def test_plan_tune(N):
    """The launch-schedule tuner picks one of the two schedules, the plan
    reports it, and dg_step with two trace arrays still equals the split
    launches bitwise under either choice."""
    import paper_1903_11521_amd as dg
    _say(f"test_plan_tune N={N}")
    plan = dg.Plan(N, 0)
    choice = plan.tune(20_000)
    assert isinstance(choice, bool)
    from paper_1903_11521_amd import _lib as L
    assert bool(L._load().dg_plan_fuses_steps(plan._h)) == choice
    mesh, mats, Q, dt = dgtest.mesh_inputs(3, N, 12)
    star, Ap, Am = dg.element_data(mesh.X, mats, mesh.neigh)
    E = mesh.E
    args = [plan.pack_star(_dev(star)), _dev(Ap), _dev(Am), _dev(mesh.neigh), _dev(mesh.face_rot)]
    Qa, Qb = _dev(Q), _dev(Q)
    I = torch.empty(plan.dof_shape(E), dtype=plan.dtype, device="cuda:0")
    ta, tb = (torch.empty(plan.trace_shape(E), dtype=plan.dtype, device="cuda:0") for _ in range(2))
    plan.step(Qa, I, ta, *args, dt, 3, traces_b=tb)
    for _ in range(3):
        plan.step_predict(Qb, args[0], dt, I, ta)
        plan.step_correct(I, ta, *args, Qb)
    assert torch.equal(Qa, Qb)


def test_debug_neighbour_checks():
    """With the debug checks on, a neighbour index outside [-1, E) is rejected
    synchronously (nothing enqueued); with them off it is treated like -1."""
    import paper_1903_11521_amd as dg
    from paper_1903_11521_amd import _lib as L
    N = 3
    mesh, mats, Q, dt = dgtest.mesh_inputs(3, N, 13)
    plan = dg.Plan(N, 0)
    star, Ap, Am = dg.element_data(mesh.X, mats, mesh.neigh)
    E = mesh.E
    bad = mesh.neigh.copy()
    bad[E // 2, 1] = E            # one past the end
    args = [plan.pack_star(_dev(star)), _dev(Ap), _dev(Am), _dev(bad), _dev(mesh.face_rot)]
    Qg = _dev(Q)
    I = torch.empty(plan.dof_shape(E), dtype=torch.float64, device="cuda:0")
    tr = torch.empty(plan.trace_shape(E), dtype=torch.float64, device="cuda:0")
    prev = L.set_debug_checks(True)
    try:
        with pytest.raises(dg.DGError, match="neighbour index"):
            plan.step(Qg, I, tr, *args, dt, 1)
        with pytest.raises(dg.DGError, match="element %d face 1" % (E // 2)):
            plan.step_correct(I, tr, *args, Qg)
        assert torch.equal(Qg, _dev(Q))          # nothing ran
    finally:
        L.set_debug_checks(prev)
    # checks off: the entry acts as "no neighbour", equal to an explicit -1
    none = mesh.neigh.copy()
    none[E // 2, 1] = -1
    Qa, Qb = _dev(Q), _dev(Q)
    plan.step(Qa, I, tr, *args, dt, 1)
    plan.step(Qb, I, tr, args[0], args[1], args[2], _dev(none), args[4], dt, 1)
    assert torch.equal(Qa, Qb)


@pytest.fixture(scope="module")
def config1_data():
    """The 40x40x40x6 = 384000-element degree-5 workload and its element data
    (built once for the full-size tests)."""
    import paper_1903_11521_amd as dg
    mesh, mats, Q, dt = dgtest.mesh_inputs(40, 5, 1)
    star, Ap, Am = dg.element_data(mesh.X, mats, mesh.neigh)
    rng = np.random.default_rng(5)
    E = mesh.E
    ids = np.sort(np.concatenate([rng.choice(E, 90, replace=False), [0, 1, 2, E - 3, E - 2, E - 1]]))
    ostar, oAp, oAm = dgtest.oracle_element_data_subset(mesh, mats, ids)
    rm = refmat.refmats(5)
    ref1 = stages.step_subset(rm, dt, ids, Q, ostar, oAp, oAm, mesh.neigh, mesh.nface, mesh.orient)
    return dict(mesh=mesh, mats=mats, Q=Q, dt=dt, star=star, Ap=Ap, Am=Am, ids=ids, ref1=ref1)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_full_size_config1_sampled(config1_data, prec):
    """Degree 5 on the 40x40x40x6 = 384000-element mesh, one step in the launch
    configuration the benchmark times (second trace array); 96 sampled
    elements re-stepped by the oracle (predictor on them and their
    neighbours), in every precision."""
    import paper_1903_11521_amd as dg
    _say(f"test_full_size_config1_sampled prec={prec}")
    c = config1_data
    mesh, Q, dt, ids = c["mesh"], c["Q"], c["dt"], c["ids"]
    E = mesh.E
    plan = dg.Plan(5, prec)
    Qg = _dev(Q, plan.dtype)
    I = torch.empty(plan.dof_shape(E), dtype=plan.dtype, device="cuda:0")
    tr = torch.empty(plan.trace_shape(E), dtype=plan.dtype, device="cuda:0")
    args = (plan.pack_star(_dev(c["star"])), _dev(c["Ap"]), _dev(c["Am"]), _dev(mesh.neigh), _dev(mesh.face_rot))
    plan.step(Qg, I, tr, *args, dt, 1, traces_b=torch.empty_like(tr))
    Q1 = _host(Qg)
    ref = c["ref1"]
    Qr = _rounded(Q[ids], prec)
    assert_close(Q1[ids] - Qr, ref - Q[ids], TOL_INC[prec], "sampled step increment")
    assert_close(Q1[ids], ref, TOL[prec], "sampled Q^{n+1}")
    # two steps with the benchmark's arguments equal two split steps bitwise
    Qa, Qb = _dev(Q, plan.dtype), _dev(Q, plan.dtype)
    plan.step(Qa, I, tr, *args, dt, 2, traces_b=torch.empty_like(tr))
    for _ in range(2):
        plan.step_predict(Qb, args[0], dt, I, tr)
        plan.step_correct(I, tr, *args, Qb)
    assert torch.equal(Qa, Qb)


def _mesh_tensors(dg, N, n, seed_index, prec, relabel=True):
    mesh, mats, Q, dt = dgtest.mesh_inputs(n, N, seed_index, relabel=relabel)
    plan = dg.Plan(N, prec)
    star, Ap, Am = dg.element_data(mesh.X, mats, mesh.neigh)
    E = mesh.E
    m = dict(degree=N, E=E, dt=dt, Q=_dev(Q, plan.dtype),
             I=torch.empty(plan.dof_shape(E), dtype=plan.dtype, device="cuda:0"),
             traces=torch.empty(plan.trace_shape(E), dtype=plan.dtype, device="cuda:0"),
             star_packed=plan.pack_star(_dev(star)), Aplus=_dev(Ap), Aminus=_dev(Am),
             neigh=_dev(mesh.neigh), face_rot=_dev(mesh.face_rot))
    return plan, m, (mesh, mats, Q, dt)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_batch_mixed_degrees(prec):
    """Five meshes of degrees 2..6 stepped as one batch (graph replay): each
    mesh equals its own single-mesh dg_step bitwise, and the FP64 oracle."""
    import paper_1903_11521_amd as dg
    _say(f"test_batch_mixed_degrees prec={prec}")
    meshes, singles, raw = [], [], []
    for i, (N, n) in enumerate([(2, 4), (5, 3), (3, 3), (6, 3), (4, 4)]):
        plan, m, r = _mesh_tensors(dg, N, n, 10 + i, prec)
        meshes.append(m)
        raw.append(r)
        q = m["Q"].clone()
        plan.step(q, torch.empty_like(m["I"]), torch.empty_like(m["traces"]), m["star_packed"], m["Aplus"],
                  m["Aminus"], m["neigh"], m["face_rot"], m["dt"], 3)
        singles.append(q)
    batch = dg.Batch(prec, meshes)
    batch.step(2)
    batch.step(1)
    torch.cuda.synchronize()
    for m, q, (mesh, mats, Q, dt) in zip(meshes, singles, raw):
        assert torch.equal(m["Q"], q), "batch differs from single-mesh step (degree %d)" % m["degree"]
        N = m["degree"]
        ostar, oAp, oAm = dgtest.oracle_element_data(mesh, mats)
        ref = Q.copy()
        for _ in range(3):
            ref = stages.step(refmat.refmats(N), dt, ref, ostar, oAp, oAm, mesh.neigh, mesh.nface, mesh.orient)
        Q3 = _host(m["Q"])
        assert_close(Q3 - _rounded(Q, prec), ref - Q, TOL_INC[prec], "degree %d 3-step increment" % N)
        assert_close(Q3, ref, TOL[prec], "degree %d Q after 3 steps" % N)
    batch.close()


def test_mixed_is_at_least_as_accurate_as_fp32():
    """The mixed form (FP64 time integral and flux products) is not less
    accurate than plain FP32 against the FP64 oracle (degree 5, 3 steps)."""
    import paper_1903_11521_amd as dg
    N = 5
    errs = {}
    for prec in (1, 2):
        plan, m, (mesh, mats, Q, dt) = _mesh_tensors(dg, N, 3, 30, prec)
        plan.step(m["Q"], m["I"], m["traces"], m["star_packed"], m["Aplus"], m["Aminus"], m["neigh"],
                  m["face_rot"], dt, 3)
        ostar, oAp, oAm = dgtest.oracle_element_data(mesh, mats)
        ref = Q.copy()
        for _ in range(3):
            ref = stages.step(refmat.refmats(N), dt, ref, ostar, oAp, oAm, mesh.neigh, mesh.nface, mesh.orient)
        errs[prec] = dgtest.rel_err(_host(m["Q"]) - _rounded(Q, prec), ref - Q)
    _say("fp32 %.3e mixed %.3e" % (errs[1], errs[2]))
    assert errs[2] <= 1e-5 and errs[1] <= 1e-5
    assert errs[2] <= errs[1] * 1.5
