"""Serving loop: admission by HBM footprint, continuous batching, accounting
(host executor on the CPU), and on the GPU: each request's result is bitwise
the same alone and in the mix."""
import numpy as np
import pytest

from paper_1903_11521_amd.serving import Request, Server, footprint_bytes


class HostExecutor:
    """Stands in for the GPU: a step multiplies every active request's state
    by a per-request factor, so results show how many steps each got."""

    def __init__(self):
        self.state, self.batches, self.t = {}, [], 0.0

    def start(self, t0):
        pass

    def add(self, req):
        self.state[req.rid] = 1.0

    def rebuild(self, rids):
        self.batches.append(sorted(rids))
        self.cur = list(rids)

    def step(self, rids):
        assert sorted(rids) == sorted(self.cur)
        for r in rids:
            self.state[r] *= 2.0
        self.t += 1.0
        return self.t

    def wait(self, token):
        return token

    def remove(self, req):
        return np.array([self.state.pop(req.rid)])

    def finish(self):
        pass


def _req(rid, E, steps, arrival, degree=3):
    return Request(rid=rid, degree=degree, E=E, n_steps=steps, arrival=arrival, build=lambda: {})


def test_each_request_gets_exactly_its_steps_and_batches_change():
    ex = HostExecutor()
    budget = footprint_bytes(1000, 3, 8) * 2
    clock = iter(np.arange(0, 1e6, 0.5))
    srv = Server(ex, budget, 8, clock=lambda: next(clock))
    srv.submit(_req(0, 1000, 3, 0.0))
    srv.submit(_req(1, 1000, 5, 0.0))
    srv.submit(_req(2, 1000, 2, 0.0))      # waits for memory
    srv.run()
    res = {r.rid: r.result[0] for r in srv.done}
    assert res == {0: 2.0 ** 3, 1: 2.0 ** 5, 2: 2.0 ** 2}
    assert [len(r.step_done) for r in sorted(srv.done, key=lambda r: r.rid)] == [3, 5, 2]
    assert len(ex.batches) >= 3 and [0, 1] in ex.batches
    s = srv.summary()
    assert s["requests"] == 3 and s["rejected"] == 0 and s["p50_step_ms"] is not None


def test_admission_rejects_and_budget_never_exceeded():
    ex = HostExecutor()
    budget = footprint_bytes(1000, 4, 4) * 3
    clock = iter(np.arange(0, 1e6, 0.25))
    srv = Server(ex, budget, 4, clock=lambda: next(clock))
    srv.submit(_req(0, 10 ** 6, 2, 0.0, degree=4))     # never fits -> rejected
    for i in range(1, 7):
        srv.submit(_req(i, 1000, 1 + i % 3, 0.1 * i, degree=4))
    peak = []
    orig = srv._admit

    def spy(now):
        orig(now)
        peak.append(srv.used)
    srv._admit = spy
    srv.run()
    assert max(peak) <= budget
    assert sum(r.rejected for r in srv.done) == 1
    assert all(r.result is not None for r in srv.done if not r.rejected)
    assert srv.used == 0


class CountingClock:
    """Deterministic clock: every reading advances it by `tick` seconds, so
    arrivals become admission points a fixed number of loop iterations in."""

    def __init__(self, tick=1e-3):
        self.t, self.tick = 0.0, tick

    def __call__(self):
        self.t += self.tick
        return self.t


def _gpu_request(dg, rid, n, N, steps, arrival):
    from math import comb

    from workload import cube_mesh, dt_from_mesh, random_dofs, random_materials, seed_for

    def build():
        mesh = cube_mesh(n, seed_for(50 + rid))
        mats = random_materials(mesh.E, seed_for(50 + rid))
        star, Ap, Am = dg.element_data(mesh.X, mats, mesh.neigh)
        return dict(dt=dt_from_mesh(mesh, mats), Q=random_dofs(mesh.E, 9, comb(N + 3, 3), seed_for(50 + rid)),
                    star=star, Aplus=Ap, Aminus=Am, neigh=mesh.neigh, face_rot=mesh.face_rot)
    return Request(rid=rid, degree=N, E=6 * n ** 3, n_steps=steps, arrival=arrival, build=build)


@pytest.mark.gpu
def test_alone_equals_mixed_on_gpu():
    """Requests that arrive while others are on the GPU join the running
    batch (dg_batch_update, no device-wide wait); each result is bitwise the
    same as the request served alone, and every one matches the FP64 oracle
    within the mixed form's bar (1e-5 on the increment, as in the parity
    tests)."""
    pytest.importorskip("torch")
    import dgtest
    import paper_1903_11521_amd as dg
    from oracle import refmat, stages
    from paper_1903_11521_amd.serving import GpuExecutor
    from workload import cube_mesh, dt_from_mesh, random_dofs, random_materials, seed_for

    # (rid, n, degree, steps, arrival): arrivals staggered by a few loop
    # iterations of the counting clock, long runs, so later requests are
    # admitted while earlier ones are mid-run
    specs = [(0, 4, 3, 12, 0.0), (1, 3, 5, 6, 0.004), (2, 5, 2, 9, 0.008), (3, 3, 6, 4, 0.012)]
    alone = {}
    for s in specs:
        srv = Server(GpuExecutor(dg.DG_MIXED), 1 << 34, 4, clock=CountingClock())
        srv.submit(_gpu_request(dg, *s))
        srv.run()
        alone[s[0]] = srv.done[0].result
    ex = GpuExecutor(dg.DG_MIXED)
    srv = Server(ex, 1 << 34, 4, clock=CountingClock())
    for s in specs:
        srv.submit(_gpu_request(dg, *s))
    srv.run()
    assert len(srv.done) == 4
    for r in srv.done:
        assert len(r.step_done) == r.n_steps
        assert np.array_equal(r.result, alone[r.rid]), r.rid
    # requests joined a batch that was already running
    sets = [set(h) for h in ex.history]
    assert any(len(a) < len(b) and a < b for a, b in zip(sets, sets[1:])), sets
    # every served request against the FP64 oracle (its own number of steps)
    for rid, n, N, steps, _ in specs:
        mesh = cube_mesh(n, seed_for(50 + rid))
        mats = random_materials(mesh.E, seed_for(50 + rid))
        Q0 = random_dofs(mesh.E, 9, refmat.n_basis(N), seed_for(50 + rid))
        ostar, oAp, oAm = dgtest.oracle_element_data(mesh, mats)
        ref = Q0.copy()
        for _ in range(steps):
            ref = stages.step(refmat.refmats(N), dt_from_mesh(mesh, mats), ref, ostar, oAp, oAm, mesh.neigh,
                              mesh.nface, mesh.orient)
        served = next(r for r in srv.done if r.rid == rid).result
        dgtest.assert_close(served - Q0.astype(np.float32).astype(np.float64), ref - Q0, 1e-5,
                            "served request %d vs oracle (%d-step increment)" % (rid, steps))
