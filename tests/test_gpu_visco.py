"""GPU parity of the viscoelastic step (dg_visco_step, 27 quantities)
through the C ABI against the viscoelastic oracle (oracle/viscoelastic.py).

The GPU runs on the product's element data (dg_visco_element_data_host) and
reference matrices, the oracle on its own.  Relaxation frequencies are
chosen so that omega dt is 0.02-0.3 (the source terms matter); memory
coefficients as the workload draws them.  Bar: FP64 1e-12 on the step
increment, per quantity and per element (dgtest), over all 27 quantities.
"""
import sys

import numpy as np
import pytest

from dgtest import assert_close
from oracle import refmat
from oracle import viscoelastic as ve
from workload import cube_mesh, dt_from_mesh, random_dofs, random_materials, seed_for

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _case(N, n, seed, relabel=True):
    mesh = cube_mesh(n, seed_for(seed), relabel=relabel)
    mats = random_materials(mesh.E, seed_for(seed))
    dt = dt_from_mesh(mesh, mats)
    omega = np.array([0.02, 0.1, 0.3]) / dt
    Ylam, Ymu = ve.memory_parameters(mats, omega, [0.02, 0.01, 0.04], [0.03, 0.015, 0.005])
    B = refmat.refmats(N).B
    Q = random_dofs(mesh.E, 27, B, seed)
    return mesh, mats, dt, omega, Ylam, Ymu, Q


def _gpu(N, mesh, mats, dt, omega, Ylam, Ymu, Q, steps, neigh=None):
    import paper_1903_11521_amd as dg
    nb = mesh.neigh if neigh is None else neigh
    star, Ap, Am = dg.visco_element_data(mesh.X, mats, omega, Ylam, Ymu, nb)
    ref = _dev(dg.reference_blob(N))
    E = mesh.E
    Qg = _dev(Q)
    I = torch.empty_like(Qg)
    Bf = refmat.refmats(N).Bf
    tr = torch.empty((E, 4, 9, Bf), dtype=torch.float64, device="cuda:0")
    dg.visco_step(N, Qg, I, tr, _dev(star), _dev(Ap), _dev(Am), omega, ref, _dev(nb.astype(np.int32)), _dev(mesh.face_rot), dt,
                  steps)
    torch.cuda.synchronize()
    return Qg.cpu().numpy()


def _oracle(N, mesh, mats, dt, omega, Ylam, Ymu, Q, steps, neigh=None):
    nb = mesh.neigh if neigh is None else neigh
    rm = refmat.refmats(N)
    star = ve.star_matrices(mesh.X, mats, omega, Ylam, Ymu)
    Ap, Am = ve.flux_matrices(mesh.X, mats, omega, Ylam, Ymu, nb)
    Es = ve.source_matrix(omega)
    for _ in range(steps):
        Q = ve.step(rm, dt, Q, star, Ap, Am, Es, nb, mesh.nface, mesh.orient)
    return Q


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6])
def test_visco_step_matches_oracle(N):
    _say(f"test_visco_step_matches_oracle N={N}")
    case = _case(N, 3, 20 + N)
    got = _gpu(N, *case, 1)
    ref = _oracle(N, *case, 1)
    Q = case[-1]
    assert_close(got - Q, ref - Q, 1e-12, "viscoelastic step increment")


def test_visco_two_steps_and_missing_neighbours():
    _say("test_visco_two_steps_and_missing_neighbours")
    N = 4
    case = _case(N, 3, 31)
    mesh = case[0]
    nb = mesh.neigh.copy()
    nb[0, 1] = -1
    nb[7, 3] = -1
    got = _gpu(N, *case, 2, neigh=nb)
    ref = _oracle(N, *case, 2, neigh=nb)
    Q = case[-1]
    assert_close(got - Q, ref - Q, 1e-12, "two-step increment")


def _visco_mesh(dg, N, n, seed):
    """Device arrays of one viscoelastic mesh as a batch item."""
    mesh, mats, dt, omega, Ylam, Ymu, Q = _case(N, n, seed)
    star, Ap, Am = dg.visco_element_data(mesh.X, mats, omega, Ylam, Ymu, mesh.neigh)
    E, Bf = mesh.E, refmat.refmats(N).Bf
    item = dict(degree=N, E=E, dt=dt, n_quant=27, omega=omega, Q=_dev(Q), I=torch.empty((E, 27, Q.shape[2]),
                dtype=torch.float64, device="cuda:0"),
                traces=torch.empty((E, 4, 9, Bf), dtype=torch.float64, device="cuda:0"), star=_dev(star),
                Aplus=_dev(Ap), Aminus=_dev(Am), neigh=_dev(mesh.neigh.astype(np.int32)), face_rot=_dev(mesh.face_rot))
    return item, (mesh, mats, dt, omega, Ylam, Ymu, Q)


def test_visco_meshes_in_a_mixed_batch():
    """Two viscoelastic meshes (degrees 3 and 5) and an elastic one (degree 4)
    in one FP64 batch, two steps: each viscoelastic mesh equals
    dg_visco_step alone bitwise and the oracle to the bar; the elastic mesh
    equals dg_step alone bitwise."""
    _say("test_visco_meshes_in_a_mixed_batch")
    import paper_1903_11521_amd as dg
    from workload import cube_mesh, dt_from_mesh, random_dofs, random_materials, seed_for
    v3, c3 = _visco_mesh(dg, 3, 3, 41)
    v5, c5 = _visco_mesh(dg, 5, 3, 42)
    mesh = cube_mesh(3, seed_for(43), relabel=True)
    mats = random_materials(mesh.E, seed_for(43))
    plan = dg.Plan(4, dg.DG_FP64)
    star, Ap, Am = dg.element_data(mesh.X, mats, mesh.neigh)
    Qe = random_dofs(mesh.E, 9, plan.B, 43)
    el = dict(degree=4, E=mesh.E, dt=dt_from_mesh(mesh, mats), Q=_dev(Qe),
              I=torch.empty(plan.dof_shape(mesh.E), dtype=torch.float64, device="cuda:0"),
              traces=torch.empty(plan.trace_shape(mesh.E), dtype=torch.float64, device="cuda:0"),
              star_packed=plan.pack_star(_dev(star)), Aplus=_dev(Ap), Aminus=_dev(Am), neigh=_dev(mesh.neigh),
              face_rot=_dev(mesh.face_rot))
    batch = dg.Batch(dg.DG_FP64, [v3, el, v5])
    batch.step(2)
    torch.cuda.synchronize()
    for item, case in ((v3, c3), (v5, c5)):
        N = item["degree"]
        alone = _gpu(N, *case, 2)
        got = item["Q"].cpu().numpy()
        assert np.array_equal(got, alone), "degree %d: batch differs from dg_visco_step" % N
        ref = _oracle(N, *case, 2)
        assert_close(got - case[-1], ref - case[-1], 1e-12, "degree %d in batch" % N)
    Qa = _dev(Qe)
    plan.step(Qa, torch.empty_like(el["I"]), torch.empty_like(el["traces"]), el["star_packed"], el["Aplus"],
              el["Aminus"], el["neigh"], el["face_rot"], el["dt"], 2)
    torch.cuda.synchronize()
    assert torch.equal(Qa, el["Q"])
    batch.close()


def test_visco_tune_keeps_results_bitwise():
    """The tuner picks a launch shape per degree; the step's results do not
    depend on it."""
    _say("test_visco_tune_keeps_results_bitwise")
    import paper_1903_11521_amd as dg
    from paper_1903_11521_amd._lib import DGError
    N = 4
    case = _case(N, 3, 51)
    before = _gpu(N, *case, 2)
    waves, per_cu = dg.visco_tune(N, 3000)
    assert waves in (4, 8) and per_cu >= 1
    after = _gpu(N, *case, 2)
    assert np.array_equal(before, after)
    with pytest.raises(DGError):
        dg.visco_tune(9, 3000)


@pytest.mark.parametrize("N,n", [(3, 8), (5, 6), (6, 4)])
def test_visco_many_elements_per_workgroup(N, n):
    """Work lists several times the persistent grid (3072, 1296 and 384
    elements; the grid has CUs x resident workgroups), so every workgroup
    walks several elements and runs the prefetch of the next one: one step
    against the oracle."""
    _say(f"test_visco_many_elements_per_workgroup N={N} n={n}")
    case = _case(N, n, 60 + N)
    got = _gpu(N, *case, 1)
    ref = _oracle(N, *case, 1)
    Q = case[-1]
    assert_close(got - Q, ref - Q, 1e-12, "viscoelastic step increment, %d elements" % case[0].E)


def test_visco_batch_of_one_degree_walks_item_boundaries():
    """Three degree-3 viscoelastic meshes in one batch (162, 1296 and 384
    elements): one work list whose workgroups cross item boundaries; each
    mesh equals dg_visco_step alone bitwise, and the largest the oracle."""
    _say("test_visco_batch_of_one_degree_walks_item_boundaries")
    import paper_1903_11521_amd as dg
    items, cases = [], []
    for n, seed in ((3, 71), (6, 72), (4, 73)):
        it, c = _visco_mesh(dg, 3, n, seed)
        items.append(it)
        cases.append(c)
    batch = dg.Batch(dg.DG_FP64, items)
    batch.step(2)
    torch.cuda.synchronize()
    for it, c in zip(items, cases):
        alone = _gpu(3, *c, 2)
        assert np.array_equal(it["Q"].cpu().numpy(), alone), "mesh of %d elements" % c[0].E
    ref = _oracle(3, *cases[1], 2)
    Q = cases[1][-1]
    assert_close(items[1]["Q"].cpu().numpy() - Q, ref - Q, 1e-12, "batched mesh of 1296 elements")
    batch.close()


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6])
def test_visco_every_launch_shape_bitwise(N):
    """Both wave counts, one workgroup per CU and all that fit: the same
    bits (the 27x element data of a 1296-element mesh, two steps)."""
    _say(f"test_visco_every_launch_shape_bitwise N={N}")
    import paper_1903_11521_amd as dg
    case = _case(N, 6, 80 + N)
    keep = dg.visco_shape(N)
    try:
        runs = []
        for shape in ((4, 0), (4, 1), (8, 0), (8, 1)):
            dg.visco_shape(N, shape)
            runs.append(_gpu(N, *case, 2))
    finally:
        dg.visco_shape(N, keep)
    shapes = ((4, 0), (4, 1), (8, 0), (8, 1))
    bad = [(sh, float(np.abs(r - runs[0]).max()), int((r != runs[0]).sum())) for sh, r in zip(shapes[1:], runs[1:])
           if not np.array_equal(runs[0], r)]
    assert not bad, "shapes differing from (4, 0): %s" % bad
