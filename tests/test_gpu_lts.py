"""GPU parity of clustered local time stepping (dg_lts_*, the LTS of Sec.
6.4) through the C ABI against the LTS oracle (oracle/lts.py) on the same
seeded inputs.

Workload: x-graded periodic cube meshes (cell widths growing by the factor
64 across the cube, all 12 neighbour face/orientation cases), random
materials, per-element CFL steps grouped into rate-2 clusters (3 or 4
clusters), elements numbered cluster by cluster.  Bars as for the global
step's multi-step increments: FP64 1e-12, FP32 and mixed 1e-5 (per
quantity and per element, dgtest).
"""
import sys

import numpy as np
import pytest

from dgtest import assert_close, oracle_element_data
from oracle import lts as olts
from oracle import refmat, stages
from workload import (element_time_steps, graded_cube_mesh, permute_elements, random_dofs, random_materials,
                      rate2_clusters, seed_for)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5, 2: 1e-5}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def _host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def _graded(n, N, seed, split=False):
    """split=False numbers elements by cluster only (boundary elements spread
    through each cluster); split=True puts each cluster's interior elements
    (no neighbour in another cluster) before its boundary elements."""
    mesh = graded_cube_mesh(n, seed_for(seed), 64.0, relabel=True)
    mats = random_materials(mesh.E, seed_for(seed))
    c, dt0 = rate2_clusters(element_time_steps(mesh, mats), mesh.neigh)
    bnd = np.any(c[mesh.neigh] != c[:, None], axis=1)
    down = np.any(c[mesh.neigh] < c[:, None], axis=1)
    order = np.lexsort((down, bnd, c)) if split else np.argsort(c, kind="stable")
    mesh = permute_elements(mesh, order)
    mats, c = mats[order], c[order]
    Q = random_dofs(mesh.E, 9, refmat.refmats(N).B, 50 + seed)
    return mesh, mats, c, dt0, Q


def _gpu_run(dg, plan, mesh, mats, c, dt0, Q, cycles, calls=1):
    star, Ap, Am = dg.element_data(mesh.X, mats, mesh.neigh)
    Qg = _dev(Q, plan.dtype)
    L = dg.Lts(plan, c, mesh.neigh, dt0)
    args = (plan.pack_star(_dev(star)), _dev(Ap), _dev(Am), _dev(mesh.neigh), _dev(mesh.face_rot))
    for _ in range(calls):
        L.advance(cycles, Qg, *args)
    out = _host(Qg)
    return out, L


def _r(a, prec):
    return a if prec == 0 else np.asarray(a, dtype=np.float32).astype(np.float64)


@pytest.mark.parametrize("prec,split", [(0, False), (0, True), (1, True), (2, False)])
def test_lts_cycle_matches_oracle(prec, split):
    """One cycle (8 steps of the smallest cluster) at degree 3 on a 384-element
    graded mesh with 4 clusters, in both element orders."""
    import paper_1903_11521_amd as dg
    N = 3
    mesh, mats, c, dt0, Q = _graded(4, N, 1, split)
    _say(f"test_lts_cycle_matches_oracle prec={prec} split={split} E={mesh.E} clusters={np.bincount(c).tolist()}")
    plan = dg.Plan(N, prec)
    got, L = _gpu_run(dg, plan, mesh, mats, c, dt0, Q, 1)
    assert L.n_clusters == 4
    assert L.updates_per_cycle == int(np.sum(2 ** (3 - c)))
    ostar, oAp, oAm = oracle_element_data(mesh, mats)
    Q0 = _r(Q, prec)
    ref = olts.run(refmat.refmats(N), c, dt0, Q0, ostar, oAp, oAm, mesh.neigh, mesh.nface, mesh.orient, 1)
    assert_close(got - Q0, ref - Q0, TOL[prec], "cycle increment")


def test_lts_two_cycles_degree5():
    """Two cycles at degree 5 (FP64) on a 162-element graded mesh with 3
    clusters, advanced by two calls of one cycle (the handle's work arrays
    carry nothing between calls)."""
    import paper_1903_11521_amd as dg
    N = 5
    mesh, mats, c, dt0, Q = _graded(3, N, 1, True)
    _say(f"test_lts_two_cycles_degree5 E={mesh.E} clusters={np.bincount(c).tolist()}")
    plan = dg.Plan(N, 0)
    got, _ = _gpu_run(dg, plan, mesh, mats, c, dt0, Q, 1, calls=2)
    got2, _ = _gpu_run(dg, plan, mesh, mats, c, dt0, Q, 2)
    assert np.array_equal(got, got2)
    ostar, oAp, oAm = oracle_element_data(mesh, mats)
    ref = olts.run(refmat.refmats(N), c, dt0, Q, ostar, oAp, oAm, mesh.neigh, mesh.nface, mesh.orient, 2)
    assert_close(got - Q, ref - Q, TOL[0], "two-cycle increment")


@pytest.mark.parametrize("level", [0, 1])
def test_lts_one_cluster_is_global_step(level):
    """All elements in one cluster (level 0, or level 1 with cluster 0 empty):
    LTS cycles are global steps of dt0 * 2^level; against dg_step and the
    oracle's global step."""
    import paper_1903_11521_amd as dg
    N = 4
    mesh, mats, _, dt0, Q = _graded(3, N, 2)
    c = np.full(mesh.E, level, np.int32)
    _say(f"test_lts_one_cluster_is_global_step level={level}")
    plan = dg.Plan(N, 0)
    got, L = _gpu_run(dg, plan, mesh, mats, c, dt0, Q, 2)
    assert L.n_clusters == level + 1 and L.updates_per_cycle == mesh.E
    dt = dt0 * 2 ** level
    star, Ap, Am = dg.element_data(mesh.X, mats, mesh.neigh)
    Qg = _dev(Q)
    I = torch.empty(plan.dof_shape(mesh.E), dtype=torch.float64, device="cuda:0")
    tr = torch.empty(plan.trace_shape(mesh.E), dtype=torch.float64, device="cuda:0")
    plan.step(Qg, I, tr, plan.pack_star(_dev(star)), _dev(Ap), _dev(Am), _dev(mesh.neigh), _dev(mesh.face_rot),
              dt, 2)
    ref_step = _host(Qg)
    assert_close(got - Q, ref_step - Q, TOL[0], "LTS vs dg_step")
    ostar, oAp, oAm = oracle_element_data(mesh, mats)
    ref = Q
    for _ in range(2):
        ref = stages.step(refmat.refmats(N), dt, ref, ostar, oAp, oAm, mesh.neigh, mesh.nface, mesh.orient)
    assert_close(got - Q, ref - Q, TOL[0], "LTS vs oracle global steps")


def test_lts_bf16x3_refused():
    import paper_1903_11521_amd as dg
    mesh, mats, c, dt0, Q = _graded(3, 3, 1)
    with pytest.raises(dg.DGError, match="not available"):
        dg.Lts(dg.Plan(3, dg.DG_BF16X3), c, mesh.neigh, dt0)
