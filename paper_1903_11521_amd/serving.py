"""Continuous-batching request loop for ensembles of elastic ADER-DG runs.

A request is one independent simulation: a mesh (cube-split, any size),
a polynomial degree, materials, initial DOFs and a number of time steps.
The loop
  * admits arrived requests in arrival order while their HBM footprint fits
    the budget; a request that does not fit is passed by later, smaller ones,
    unless it needs more than half of the budget, in which case admission
    stops at it so that it is served as soon as memory frees up;
  * keeps the DOFs and static data of admitted requests resident on the GPU;
  * steps all admitted requests together: one dg_batch step (one predictor
    and one corrector launch per degree present, a replayed HIP graph); when
    a request joins or leaves, the batch's mesh list is replaced in stream
    order (dg_batch_update: the batch's second table slot and graph), with no
    device-wide synchronisation;
  * records, for every request, the completion time of each of its steps and
    returns the final DOFs when it finishes.
Per-step latency of a request = time between its consecutive step
completions (the first measured from admission).  Each element's arithmetic
does not depend on which other requests share the launch, so a request's
result is bitwise the same alone and in any mix.

The executor is separate from the scheduling logic so that admission and
accounting can be exercised without a GPU (tests use a host executor).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from math import comb
from typing import Callable, Dict, List, Optional

import numpy as np


def footprint_bytes(E: int, degree: int, itemsize: int) -> int:
    """Resident bytes of one request: Q, I, traces, packed star (plan type),
    A+ and A- (FP64), neighbour tables."""
    B, Bf = comb(degree + 3, 3), comb(degree + 2, 2)
    return E * (itemsize * (2 * 9 * B + 4 * 9 * Bf + 81) + 2 * 4 * 81 * 8 + 4 * 4 + 4)


@dataclass
class Request:
    rid: int
    degree: int
    E: int
    n_steps: int
    arrival: float                      # seconds since the loop started
    build: Callable[[], dict]           # host inputs: dt, Q, star, Aplus, Aminus, neigh, face_rot
    admitted_at: Optional[float] = None
    step_done: List[float] = field(default_factory=list)
    result: Optional[np.ndarray] = None
    rejected: bool = False


class Server:
    """Scheduling and accounting; the executor does the device work."""

    def __init__(self, executor, budget_bytes: int, itemsize: int, clock=time.perf_counter, log=None):
        self.ex = executor
        self.log = log                   # optional progress callback (one line per finished request)
        self.budget = int(budget_bytes)
        self.itemsize = itemsize
        self.clock = clock
        self.queue: List[Request] = []
        self.active: Dict[int, Request] = {}
        self.done: List[Request] = []
        self.used = 0

    def submit(self, req: Request):
        if footprint_bytes(req.E, req.degree, self.itemsize) > self.budget:
            req.rejected = True          # can never fit
            self.done.append(req)
            return
        self.queue.append(req)
        prepare = getattr(self.ex, "prepare", None)
        if prepare is not None:
            prepare(req)                 # host-side setup may start early

    def _admit(self, now):
        for req in list(self.queue):
            if req.arrival > now:
                continue
            need = footprint_bytes(req.E, req.degree, self.itemsize)
            if self.used + need <= self.budget:
                self.queue.remove(req)
                self.ex.add(req)
                self.used += need
                req.admitted_at = self.clock() - self.t0
                self.active[req.rid] = req
                self.enqueued[req.rid] = 0
            elif need * 2 > self.budget:
                break                    # a large request at the head: keep order

    def run(self, until_idle=True, max_iters=10 ** 9):
        self.t0 = self.clock()
        self.ex.start(self.t0)
        self.enqueued = {}
        batch_set = None
        pending = None   # (token, rids) of the step in flight
        it = 0
        while it < max_iters:
            it += 1
            self._admit(self.clock() - self.t0)
            runnable = [rid for rid, r in self.active.items() if self.enqueued[rid] < r.n_steps]
            token = None
            if runnable:
                if batch_set != set(runnable):
                    self.ex.rebuild(runnable)
                    batch_set = set(runnable)
                token = self.ex.step(runnable)
                for rid in runnable:
                    self.enqueued[rid] += 1
            if pending is not None:
                self._complete(*pending)
            pending = (token, runnable) if token is not None else None
            if not self.active and pending is None:
                if not self.queue:
                    if until_idle:
                        break
                else:
                    nxt = min(r.arrival for r in self.queue)
                    wait = nxt - (self.clock() - self.t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.05))
        if pending is not None:
            self._complete(*pending)
        self.ex.finish()

    def _complete(self, token, rids):
        t = self.ex.wait(token) - self.t0
        for rid in rids:
            req = self.active[rid]
            req.step_done.append(t)
            if len(req.step_done) == req.n_steps:
                # its last step has completed and no later launch includes it
                req.result = self.ex.remove(req)
                self.used -= footprint_bytes(req.E, req.degree, self.itemsize)
                del self.active[rid]
                self.done.append(req)
                if self.log is not None:
                    self.log("request %d done (%d elements, degree %d, %d steps) at %.2f s; %d finished"
                             % (rid, req.E, req.degree, req.n_steps, t, len(self.done)))

    # -- metrics --------------------------------------------------------------
    def latencies(self):
        lat = []
        for r in self.done:
            if r.rejected or not r.step_done:
                continue
            prev = r.admitted_at
            for t in r.step_done:
                lat.append(t - prev)
                prev = t
        return np.array(lat)

    def summary(self):
        lat = self.latencies()
        served = [r for r in self.done if not r.rejected]
        updates = sum(r.E * len(r.step_done) for r in served)
        span = max((r.step_done[-1] for r in served if r.step_done), default=0.0)
        queue_delay = [r.admitted_at - r.arrival for r in served if r.admitted_at is not None]
        return {"requests": len(served), "rejected": sum(r.rejected for r in self.done),
                "element_updates": updates, "wall_s": span,
                "element_updates_per_s": updates / span if span > 0 else 0.0,
                "p50_step_ms": float(np.percentile(lat, 50) * 1e3) if len(lat) else None,
                "p99_step_ms": float(np.percentile(lat, 99) * 1e3) if len(lat) else None,
                "p50_queue_ms": float(np.percentile(queue_delay, 50) * 1e3) if queue_delay else None}


class GpuExecutor:
    """Device side: resident tensors per request, one dg_batch per active set."""

    def __init__(self, precision, host_workers=4):
        from concurrent.futures import ThreadPoolExecutor

        import torch

        from . import _lib
        self.torch = torch
        self.dg = _lib
        self.precision = precision
        self.meshes = {}
        self.batch = None
        self.stream = torch.cuda.current_stream()
        self.pool = ThreadPoolExecutor(host_workers)
        self.futures = {}
        self.history = []            # the request sets of successive batches

    def prepare(self, req: Request):
        """Start the host-side setup (mesh tables, element data) in a worker
        thread, so that admission only uploads."""
        self.futures[req.rid] = self.pool.submit(req.build)

    def start(self, t0):
        self.t0 = t0

    def add(self, req: Request):
        torch, dg = self.torch, self.dg
        plan = dg.Plan(req.degree, self.precision)
        fut = self.futures.pop(req.rid, None)
        h = fut.result() if fut is not None else req.build()
        dev = torch.device("cuda:0")
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        E = req.E
        self.meshes[req.rid] = dict(
            degree=req.degree, E=E, dt=h["dt"], Q=t(h["Q"]).to(plan.dtype),
            I=torch.empty(plan.dof_shape(E), dtype=plan.dtype, device=dev),
            traces=torch.empty(plan.trace_shape(E), dtype=plan.dtype, device=dev),
            star_packed=plan.pack_star(t(h["star"])), Aplus=t(h["Aplus"]), Aminus=t(h["Aminus"]),
            neigh=t(h["neigh"]), face_rot=t(h["face_rot"]))

    def rebuild(self, rids):
        self.history.append(sorted(rids))
        meshes = [self.meshes[r] for r in rids]
        if self.batch is None:
            self.batch = self.dg.Batch(self.precision, meshes)
        else:
            self.batch.update(meshes)

    def step(self, rids):
        torch = self.torch
        self.batch.step(1)
        ev = torch.cuda.Event()
        ev.record(self.stream)
        return ev

    def wait(self, ev):
        ev.synchronize()
        return time.perf_counter()

    def remove(self, req: Request):
        m = self.meshes.pop(req.rid)
        # stream-ordered after its last step; the batch keeps the request's
        # tensors referenced until no enqueued step can read them
        return m["Q"].double().cpu().numpy()

    def finish(self):
        if self.batch is not None:
            self.torch.cuda.synchronize()
            self.batch.close()
            self.batch = None
        self.torch.cuda.synchronize()
        self.pool.shutdown(wait=False)
