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


@pytest.mark.gpu
def test_alone_equals_mixed_on_gpu():
    torch = pytest.importorskip("torch")
    import paper_1903_11521_amd as dg
    from paper_1903_11521_amd.serving import GpuExecutor
    from workload import cube_mesh, dt_from_mesh, random_dofs, random_materials, seed_for
    from math import comb

    def make(rid, n, N, steps, arrival):
        def build():
            mesh = cube_mesh(n, seed_for(50 + rid))
            mats = random_materials(mesh.E, seed_for(50 + rid))
            star, Ap, Am = dg.element_data(mesh.X, mats, mesh.neigh)
            return dict(dt=dt_from_mesh(mesh, mats), Q=random_dofs(mesh.E, 9, comb(N + 3, 3), seed_for(50 + rid)),
                        star=star, Aplus=Ap, Aminus=Am, neigh=mesh.neigh, face_rot=mesh.face_rot)
        return Request(rid=rid, degree=N, E=6 * n ** 3, n_steps=steps, arrival=arrival, build=build)

    specs = [(0, 4, 3, 6, 0.0), (1, 3, 5, 4, 0.0), (2, 5, 2, 7, 0.0), (3, 3, 6, 3, 0.0)]
    alone = {}
    for s in specs:
        srv = Server(GpuExecutor(dg.DG_MIXED), 1 << 34, 4)
        srv.submit(make(*s))
        srv.run()
        alone[s[0]] = srv.done[0].result
    srv = Server(GpuExecutor(dg.DG_MIXED), 1 << 34, 4)
    for s in specs:
        srv.submit(make(*s))
    srv.run()
    assert len(srv.done) == 4
    for r in srv.done:
        assert len(r.step_done) == r.n_steps
        assert np.array_equal(r.result, alone[r.rid]), r.rid
