"""Benchmark: degree-5 elastic ADER-DG time steps on one MI355X.

Workload: the 40x40x40 cube grid split into 6 tetrahedra per cube (384000
elements), jittered interior vertices, periodic faces, random materials,
N(0,1) degree-5 DOFs (B = 56, 9 quantities), dt = 0.1 h_min / cp_max; each
step is one full ADER-DG time step (predictor, time integral, volume, local
and neighbour flux) of every element.  All inputs are resident in HBM before
the timed region.

Prints one JSON line: element-updates/s; the roofline of the dominant kernel
(HIP events on the launch stream) on the method's algorithmic bytes and
non-zero flops, with this layout's own bytes beside them; the fraction of the
whole step's roofline; each per-stage entry point timed with its own
roofline fraction; and the FP64 oracle timed on the host cores (all of them
and one) on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PRECISIONS = {"fp64": 0, "fp32": 1, "mixed": 2, "bf16x3": 3}     # dg_precision of include/dg.h
DTYPES = {"fp64": "f64", "fp32": "f32", "mixed": "f32 (f64 time integral and flux solvers)",
          "bf16x3": "f32 storage, 3xbf16 matrix-core contractions (f64 flux solvers)"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=["fp64", "fp32", "mixed", "bf16x3"], default="fp64")
    ap.add_argument("--degree", type=int, default=5)
    ap.add_argument("--n", type=int, default=40, help="cubes per direction")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stages", action="store_true", help="skip the per-stage timing")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--workload", choices=["single", "batched", "serving", "fused", "madness", "lts", "lina",
                                                "visco"],
                    default="single",
                    help="single: one degree-N mesh; batched: 32 independent meshes of mixed degree; "
                         "serving: Poisson arrivals of ensemble requests; fused: 16 simulations per mesh; "
                         "madness: the separable contraction of Sec. 7; lts: local against global time stepping; "
                         "lina: the LinA ADER-DG-SEM scheme on cuboids (Sec. 5.2)")
    ap.add_argument("--grading", type=float, default=64.0, help="lts: cell-width ratio across the graded mesh")
    ap.add_argument("--meshes", type=int, default=32)
    ap.add_argument("--fusion", choices=["auto", "on", "off"], default="auto",
                    help="single: the plan's step schedule (auto), one fused launch per step (on) or two (off)")
    ap.add_argument("--elastic-only", action="store_true", help="batched: no viscoelastic meshes")
    ap.add_argument("--rate", type=float, default=5.0, help="serving: arrivals per second")
    ap.add_argument("--requests", type=int, default=16)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (calibrates HBM byte counters)")
    return ap.parse_args()


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("csrc/dg_kernels.hip", "csrc/dg_launch.hip", "csrc/step_predict_body.inc",
              "csrc/step_correct_body.inc", "csrc/refmat.cpp", "codegen.py"):
        with open(os.path.join(ROOT, "paper_1903_11521_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, degree, precision):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    rec = data.get("%s_deg%d_%s" % (kernel, degree, precision))
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args, mesh, mats, Q, dt):
    """The FP64 oracle (plain loop nests, OpenMP over elements) on the first S
    elements of the same workload, on every host core this process may use
    and on one core; neighbour indices are folded into the sample (same work
    per element)."""
    from oracle import elements as oel
    from oracle import refmat, stages
    rm = refmat.refmats(args.degree)
    cores = len(os.sched_getaffinity(0))

    def run(S, threads):
        X = mesh.X[:S]
        star = oel.star_matrices(X, mats[:S])
        nb = (mesh.neigh[:S] % S).astype(np.int32)
        Ap, Am = oel.flux_matrices(X, mats[:S], nb)
        stages.set_threads(threads)
        t = time.perf_counter()
        stages.step(rm, dt, Q[:S], star, Ap, Am, nb, mesh.nface[:S], mesh.orient[:S])
        return time.perf_counter() - t

    def timed(threads, seconds):
        S0 = 64 * threads
        t0 = run(S0, threads)
        S = int(min(mesh.E, max(S0, S0 * seconds / max(t0, 1e-3))))
        return S, run(S, threads)

    S, t = timed(cores, args.cpu_seconds)
    S1, t1 = timed(1, args.cpu_seconds * 0.6)
    stages.set_threads(cores)
    return {"value": S / t, "unit": "element-updates/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "single_thread": {"value": S1 / t1, "elements": S1, "seconds": t1},
            "sample": "one full time step of the first %d elements (of %d) of the same degree-%d workload, "
                      "FP64 dense loop nests, OpenMP over elements on %d threads (%.1f s); single thread: "
                      "first %d elements (%.1f s)" % (S, mesh.E, args.degree, cores, t, S1, t1)}


def batched(args):
    """32 independent cube-split meshes, E_i ~ log-uniform[10k, 200k] elements
    (n_i = round((E_i/6)^(1/3)) cubes per direction), degree U{2..6}, random
    materials and N(0,1) DOFs per mesh; all stepped together (one predictor and
    one corrector launch per degree and material model, recorded once in a HIP
    graph).  In FP64 every second mesh is viscoelastic (27 quantities, three
    mechanisms with relaxation frequencies f ~ log-uniform[0.1, 10] Hz,
    omega = 2 pi f, memory coefficients Y = (lambda, mu) * U[0.01, 0.05] per
    mechanism); the other precisions have no viscoelastic form, so their
    batches are elastic only."""
    import torch

    import paper_1903_11521_amd as dg
    from workload import cube_mesh, dt_from_mesh, random_dofs, random_materials, seed_for
    prec = {"fp64": dg.DG_FP64, "fp32": dg.DG_FP32, "mixed": dg.DG_MIXED, "bf16x3": dg.DG_BF16X3}[args.precision]
    rng = np.random.Generator(np.random.PCG64(seed_for(2)))
    sizes = np.exp(rng.uniform(np.log(10e3), np.log(200e3), args.meshes))
    degrees = rng.integers(2, 7, args.meshes)
    dev = torch.device("cuda:0")
    from paper_1903_11521_amd import perfmodel as pm
    itemsize = 8 if prec == dg.DG_FP64 else 4
    meshes, flops, nbytes = [], 0.0, 0.0
    visco_on = prec == dg.DG_FP64 and not args.elastic_only
    kinds = []
    for i, (Ei, N) in enumerate(zip(sizes, degrees)):
        n = max(3, int(round((Ei / 6) ** (1 / 3))))
        seed = seed_for(2) + 1000 * (i + 1)
        mesh = cube_mesh(n, seed)
        E = mesh.E
        mats = random_materials(E, seed)
        if visco_on and i % 2 == 1:
            vr = np.random.Generator(np.random.PCG64(seed + 7))
            omega = 2 * np.pi * np.exp(vr.uniform(np.log(0.1), np.log(10.0), 3))
            item = visco_mesh_item(dg, mesh, mats, int(N), omega, vr.uniform(0.01, 0.05, 3), seed, dev)
            item["dt"] = dt_from_mesh(mesh, mats)
            meshes.append(item)
            kinds.append("visco")
            f_, b_ = visco_model(int(N))
            flops += f_ * E
            nbytes += b_ * E
            continue
        kinds.append("elastic")
        plan = dg.Plan(int(N), prec)
        Q = random_dofs(E, 9, plan.B, seed)
        star, Ap, Am = dg.element_data(mesh.X, mats, mesh.neigh)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        meshes.append(dict(degree=int(N), E=E, dt=dt_from_mesh(mesh, mats), Q=t(Q).to(plan.dtype),
                           I=torch.empty(plan.dof_shape(E), dtype=plan.dtype, device=dev),
                           traces=torch.empty(plan.trace_shape(E), dtype=plan.dtype, device=dev),
                           star_packed=plan.pack_star(t(star)), Aplus=t(Ap), Aminus=t(Am),
                           neigh=t(mesh.neigh), face_rot=t(mesh.face_rot)))
        flops += pm.PAPER_NZ_PER_UPDATE[int(N)] * E
        nbytes += pm.method_bytes(int(N), itemsize)["step"] * E
        del star, Ap, Am
    total = sum(m["E"] for m in meshes)
    log("batch of %d meshes, %d elements, degrees %s" % (len(meshes), total, sorted(set(degrees.tolist()))))
    # the viscoelastic launch shapes (waves per workgroup, workgroups per CU)
    # picked by the library's tuner before the batch records its graph
    shapes = {int(m["degree"]): None for m in meshes if m.get("n_quant") == 27}
    for N in sorted(shapes):
        shapes[N] = dg.visco_tune(N, 100000)
        log("viscoelastic degree %d: %d waves per workgroup, %d workgroups per CU" % (N, *shapes[N]))
    batch = dg.Batch(prec, meshes)
    torch.cuda.synchronize()
    batch.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step(args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    dtype = "f64" if prec == dg.DG_FP64 else "f32"
    roof = pm.kernel_roofline(flops, nbytes, el / args.steps, dtype)
    roof["traffic"] = None
    roof["kernel"] = "whole batched step (all launches of one graph replay)"
    out = {"metric": "element-updates/s", "value": total * args.steps / el, "unit": "element-updates/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": DTYPES[args.precision], "data": "synthetic",
           "config": {"workload": "batched: %d independent cube-split meshes (%d viscoelastic with 3 "
                                  "mechanisms, the rest elastic), %d elements in total, log-uniform 10k-200k "
                                  "elements per mesh, degrees uniform in 2..6, one HIP graph replay per step"
                                  % (len(meshes), kinds.count("visco"), total),
                      "elements": total, "degrees": degrees.tolist(), "mesh_elements": [m["E"] for m in meshes],
                      "models": kinds,
                      "visco_shapes": {str(N): {"waves": w, "groups_per_cu": g} for N, (w, g) in shapes.items()}},
           "useful_gflops": flops * args.steps / el / 1e9, "roofline": roof}
    batch.close()
    print(json.dumps(out), flush=True)


def fused(args):
    """Fused simulations: 16 independent simulations on one degree-N mesh
    (the n x n x n cube-split mesh of the single workload, random materials),
    stepped together by dg_fused_step (split-BF16 form, one element and its
    16 simulations per wave).  DOFs N(0,1) drawn on the device from a seeded
    generator.  The metric counts simulation-element updates."""
    import torch

    import paper_1903_11521_amd as dg
    from paper_1903_11521_amd import perfmodel as pm
    from workload import cube_mesh, dt_from_mesh, random_materials, seed_for
    N = args.degree
    plan = dg.Plan(N, dg.DG_BF16X3)
    seed = seed_for(1)
    log("building mesh n=%d degree=%d (16 simulations)" % (args.n, N))
    mesh = cube_mesh(args.n, seed)
    E = mesh.E
    mats = random_materials(E, seed)
    dt = dt_from_mesh(mesh, mats)
    star, Ap, Am = dg.element_data(mesh.X, mats, mesh.neigh)
    dev = torch.device("cuda:0")
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    star_p = plan.pack_star(to(star))
    Apg, Amg = to(Ap), to(Am)
    del star, Ap, Am
    neigh, face_rot = to(mesh.neigh), to(mesh.face_rot)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    Qg = torch.randn(plan.fused_dof_shape(E), generator=g, dtype=torch.float32, device=dev)
    I = torch.empty(plan.fused_dof_shape(E), dtype=torch.float32, device=dev)
    tr = torch.empty(plan.fused_trace_shape(E), dtype=torch.float32, device=dev)
    S = plan.FUSED_SIMS
    torch.cuda.synchronize()
    log("warmup %d steps" % args.warmup)
    plan.fused_step(Qg, I, tr, star_p, Apg, Amg, neigh, face_rot, dt, args.warmup)
    plan.sync()
    log("timed %d steps on %d elements x %d simulations" % (args.steps, E, S))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.fused_step(Qg, I, tr, star_p, Apg, Amg, neigh, face_rot, dt, args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    value = E * S * args.steps / el
    # method bytes per simulation-element update: DOF arrays per simulation,
    # star, flux solvers and tables shared by the 16 simulations
    q = 9 * plan.B * 4
    shared = 81 * 4 + 2 * 4 * 81 * 8 + 4 * 4 + 4
    per_update = 4 * q + shared / S
    roof = pm.kernel_roofline(pm.PAPER_NZ_PER_UPDATE[N] * value * el / args.steps, per_update * E * S,
                              el / args.steps, "bf16x3")
    roof["traffic"] = None
    roof["kernel"] = "whole fused step (predictor and corrector launch)"
    roof["algorithmic_bytes_per_update"] = per_update
    out = {"metric": "element-updates/s", "value": value, "unit": "simulation-element-updates/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": DTYPES["bf16x3"], "data": "synthetic",
           "config": {"workload": "fused simulations: %d simulations of the degree-%d elastic scheme on the "
                                  "%dx%dx%dx6 = %d-element jittered periodic cube-split mesh, one launch pair "
                                  "per step" % (S, N, args.n, args.n, args.n, E),
                      "elements": E, "simulations": S, "degree": N},
           "useful_gflops": pm.PAPER_NZ_PER_UPDATE[N] * value / 1e9, "roofline": roof}
    print(json.dumps(out), flush=True)


def lts(args):
    """Local time stepping (Sec. 6.4, Table tab:loh1): time to solution of the
    degree-N elastic scheme on a graded mesh (the n x n x n cube-split mesh
    with cell widths growing geometrically by --grading along x) in a layered
    medium (a slower layer over a halfspace, the setting of the paper's LTS
    runs), elements in rate-2 clusters of their CFL steps, numbered
    cluster by cluster (interior elements of a cluster before its boundary
    elements).  One timed step is one LTS cycle (2^(C-1) steps of
    the smallest cluster, every element advanced by the same simulated
    time).  Global time stepping over the same simulated time needs 2^(C-1)
    steps of dt0 for every element: timed with dg_step, and with the LTS
    scheduler given a single cluster (its overhead against dg_step)."""
    import torch

    import paper_1903_11521_amd as dg
    from workload import (element_time_steps, graded_cube_mesh, layered_materials, permute_elements,
                          rate2_clusters, seed_for)
    N = args.degree
    prec = PRECISIONS[args.precision]
    plan = dg.Plan(N, prec)
    seed = seed_for(1)
    log("building graded mesh n=%d ratio=%g degree=%d" % (args.n, args.grading, N))
    mesh = graded_cube_mesh(args.n, seed, args.grading)
    mats = layered_materials(mesh, seed)
    cl, dt0 = rate2_clusters(element_time_steps(mesh, mats), mesh.neigh)
    # cluster by cluster: interior elements, other boundary elements, then
    # those with a neighbour one cluster down
    bnd = np.any(cl[mesh.neigh] != cl[:, None], axis=1)
    down = np.any(cl[mesh.neigh] < cl[:, None], axis=1)
    order = np.lexsort((down, bnd, cl))
    mesh = permute_elements(mesh, order)
    mats, cl = mats[order], cl[order]
    E = mesh.E
    star, Ap, Am = dg.element_data(mesh.X, mats, mesh.neigh)
    dev = torch.device("cuda:0")
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    star_p = plan.pack_star(to(star))
    Apg, Amg = to(Ap), to(Am)
    del star, Ap, Am
    neigh, face_rot = to(mesh.neigh), to(mesh.face_rot)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    Qg = torch.randn(plan.dof_shape(E), generator=g, dtype=plan.dtype, device=dev)
    L = dg.Lts(plan, cl, mesh.neigh, dt0)
    C = L.n_clusters
    sizes = np.bincount(cl, minlength=C).tolist()
    log("clusters %s, %d element updates per cycle (global stepping: %d)" % (sizes, L.updates_per_cycle,
                                                                            E << (C - 1)))
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def timed(fn, reps):
        e0, e1 = ev(), ev()
        torch.cuda.synchronize()
        e0.record()
        fn(reps)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3 / reps

    L.advance(args.warmup, Qg, star_p, Apg, Amg, neigh, face_rot)
    t_lts = timed(lambda k: L.advance(k, Qg, star_p, Apg, Amg, neigh, face_rot), args.steps)
    log("LTS: %.3f ms per cycle" % (t_lts * 1e3))
    # global time stepping over one cycle's simulated time
    ticks = 1 << (C - 1)
    I = torch.empty(plan.dof_shape(E), dtype=plan.dtype, device=dev)
    tr = torch.empty(plan.trace_shape(E), dtype=plan.dtype, device=dev)
    trb = torch.empty_like(tr)
    plan.step(Qg, I, tr, star_p, Apg, Amg, neigh, face_rot, dt0, ticks, traces_b=trb)
    t_gts = timed(lambda k: plan.step(Qg, I, tr, star_p, Apg, Amg, neigh, face_rot, dt0, ticks * k,
                                      traces_b=trb), max(1, args.steps // 2))
    log("GTS (fused step kernels): %.3f ms per cycle" % (t_gts * 1e3))
    one = dg.Lts(plan, np.zeros(E, np.int32), mesh.neigh, dt0)
    t_gts_stage = timed(lambda k: one.advance(ticks * k, Qg, star_p, Apg, Amg, neigh, face_rot),
                        max(1, args.steps // 2))
    log("GTS (one-cluster LTS schedule): %.3f ms per cycle" % (t_gts_stage * 1e3))
    value = L.updates_per_cycle / t_lts
    out = {"metric": "time-to-solution speed-up of LTS over GTS", "value": t_gts / t_lts, "unit": "x",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_lts * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": DTYPES[args.precision], "data": "synthetic",
           "config": {"workload": "local time stepping, degree-%d elastic scheme on the %dx%dx%dx6 = %d-element "
                                  "periodic cube-split mesh graded by %g along x, slower top layer over a halfspace, "
                                  "rate-2 clusters of the per-element CFL steps; one step = one cycle"
                                  % (N, args.n, args.n, args.n, E, args.grading),
                      "elements": E, "degree": N, "clusters": sizes},
           "lts_element_updates_per_s": value, "lts_ms_per_cycle": t_lts * 1e3,
           "gts_ms_per_cycle": t_gts * 1e3, "gts_one_cluster_lts_ms_per_cycle": t_gts_stage * 1e3,
           "update_ratio": (E << (C - 1)) / L.updates_per_cycle}
    print(json.dumps(out), flush=True)


def lina(args):
    """The LinA scheme (Sec. 5.2): linear acoustics on a periodic grid of
    cubes with a tensor-product Gauss-Lobatto basis, at the paper's orders 8
    (FP64 and FP32) and 16 (FP32), about 1 GiB of DOFs each (N(0,1) drawn on
    the device), 10 steps timed with HIP events.  Useful flops per element
    update count the derivative recursion and weak derivatives as line
    contractions (12 O^4 per derivative or weak-derivative term set), the
    time integral and the side fluxes (the acoustic flux solvers' non-zeros);
    bytes count Q read and written, the sides written once and read twice
    (own and neighbour), and the boundary nodes of Q updated by the flux."""
    import torch

    import paper_1903_11521_amd as dg
    from paper_1903_11521_amd import perfmodel as pm
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(1903)
    rows = []
    rho0, K0 = 1.2, 1.4e5
    c = (K0 / rho0) ** 0.5
    for dtype, name, order in ((torch.float64, "f64", 8), (torch.float32, "f32", 8), (torch.float32, "f32", 16)):
        elem = 8 if dtype == torch.float64 else 4
        n = max(2, int(round(((1 << 30) / (4 * order ** 3 * elem)) ** (1.0 / 3.0))))
        E = n ** 3
        h = 1.0 / n
        dt = 0.3 * h / (c * (2 * order - 1))
        idx = np.arange(E)
        ix, iy, iz = idx % n, (idx // n) % n, idx // (n * n)
        at = lambda a, b, cc: ((cc % n) * n + (b % n)) * n + (a % n)
        neigh = np.stack([at(ix - 1, iy, iz), at(ix + 1, iy, iz), at(ix, iy - 1, iz), at(ix, iy + 1, iz),
                          at(ix, iy, iz - 1), at(ix, iy, iz + 1)], axis=1).astype(np.int32)
        coef = torch.from_numpy(dg.lina_coefficients(order, rho0, K0, h)["blob"]).to(dtype).to(dev)
        Q = torch.randn((E, 4, order, order, order), generator=g, dtype=dtype, device=dev)
        sides = torch.empty((E, 6, 4, order, order), dtype=dtype, device=dev)
        nb = torch.from_numpy(neigh).to(dev)
        dg.lina_step(Q, sides, coef, nb, dt, 1)
        torch.cuda.synchronize()
        steps = 10
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dg.lina_step(Q, sides, coef, nb, dt, steps)
        e1.record()
        torch.cuda.synchronize()
        el = e0.elapsed_time(e1) / 1e3 / steps
        O3, O2, N = order ** 3, order ** 2, order - 1
        flops = 12.0 * order ** 4 * (N + 1) + 8.0 * O3 * (N + 1) + 96.0 * O2
        nbytes = (2 * 4 * O3 + 3 * 6 * 4 * O2 + 2 * 6 * 4 * O2) * elem
        roof = pm.kernel_roofline(flops * E, nbytes * E, el, name)
        rows.append({"dtype": name, "order": order, "elements": E, "ms_per_step": el * 1e3,
                     "element_updates_per_s": E / el, "useful_gflops": flops * E / el / 1e9,
                     "bound": roof["bound"], "frac": roof["frac"]})
        log("lina %s order %d, %d elements: %.3f ms/step, %.1f M element-updates/s, %.0f GFLOP/s (%s, %.2f)"
            % (name, order, E, el * 1e3, E / el / 1e6, flops * E / el / 1e9, roof["bound"], roof["frac"]))
        del Q, sides, coef
    best = max(r["useful_gflops"] for r in rows if r["dtype"] == "f64")
    out = {"metric": "useful GFLOP/s", "value": best, "unit": "GFLOP/s", "n_gpus": 1, "steps": 10, "warmup": 1,
           "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64 and f32", "data": "synthetic",
           "config": {"workload": "LinA ADER-DG-SEM (Sec. 5.2): linear acoustics on a periodic grid of cubes, "
                                  "Gauss-Lobatto tensor basis of order 8 (FP64, FP32) and 16 (FP32), about 1 GiB "
                                  "of DOFs"},
           "lina": rows}
    print(json.dumps(out), flush=True)


def visco_model(N):
    """Useful flops and algorithmic bytes per viscoelastic element update at
    degree N: the executed contractions over the 9 elastic columns the
    Jacobians read (predictor recursion, traces, volume, the four faces' f^h,
    flux-solver and lift products) and the source terms; Q read twice and
    written, the time integral written and read, the traces written and read
    (own and neighbour), the star matrices read twice, the flux solvers read
    once, the neighbour table."""
    from math import comb
    B, Bf = comb(N + 3, 3), comb(N + 2, 2)
    star_fl = 3 * (2 * B * B * 9 + 2 * B * 9 * 27)
    flops = (N + 1) * star_fl + 4 * 2 * B * Bf * 9 + 4 * (2 * Bf * Bf * 9 + 4 * Bf * 27 * 9 + 2 * B * Bf * 27) \
        + (N + 1) * (36 + 2 * 27) * B
    nbytes = 8 * (3 * 27 * B + 2 * 27 * B + 3 * 4 * 9 * Bf + 2 * 3 * 27 * 9 + 2 * 4 * 27 * 9) + 4 * 5
    return flops, nbytes


def visco_mesh_item(dg, mesh, mats, N, omega, yfac, seed, dev):
    """Device arrays of one viscoelastic mesh (batch item): memory
    coefficients Y = (lambda, mu) * yfac per mechanism, N(0,1) DOFs."""
    import torch
    from math import comb
    mu = mats[:, 0] * mats[:, 2] ** 2                    # rho cs^2
    lam = mats[:, 0] * mats[:, 1] ** 2 - 2.0 * mu        # rho cp^2 - 2 mu
    Ylam, Ymu = lam[:, None] * yfac[None, :], mu[:, None] * yfac[None, :]
    star, Ap, Am = dg.visco_element_data(mesh.X, mats, omega, Ylam, Ymu, mesh.neigh)
    E, B, Bf = mesh.E, comb(N + 3, 3), comb(N + 2, 2)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    from workload import random_dofs
    return dict(degree=N, E=E, n_quant=27, omega=omega, Q=t(random_dofs(E, 27, B, seed)),
                I=torch.empty((E, 27, B), dtype=torch.float64, device=dev),
                traces=torch.empty((E, 4, 9, Bf), dtype=torch.float64, device=dev), star=t(star), Aplus=t(Ap),
                Aminus=t(Am), neigh=t(mesh.neigh.astype(np.int32)), face_rot=t(mesh.face_rot))


def visco(args):
    """Viscoelastic elements (27 quantities, three mechanisms) on the
    n x n x n cube-split mesh with random materials, degrees 3 and the
    --degree one, DOFs N(0,1) drawn on the device, relaxation frequencies
    with omega dt = 0.02, 0.1, 0.3, 10 steps timed with HIP events on the
    launch stream.  Useful flops per element update count the executed
    contractions over the 9 elastic columns the Jacobians read (predictor
    recursion, traces, volume, the four faces' f^h, flux-solver and lift
    products) and the source terms; bytes count Q (read twice, written
    once), the time integral (written, read), the traces (written, read own
    and neighbour), the star matrices (read twice) and the flux solvers."""
    from math import comb

    import torch

    import paper_1903_11521_amd as dg
    from paper_1903_11521_amd import perfmodel as pm
    from workload import cube_mesh, dt_from_mesh, random_materials, seed_for
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(1903)
    mesh = cube_mesh(args.n, seed_for(0), relabel=True)
    mats = random_materials(mesh.E, seed_for(0))
    dt = dt_from_mesh(mesh, mats)
    omega = np.array([0.02, 0.1, 0.3]) / dt
    mu = mats[:, 0] * mats[:, 2] ** 2                    # rho cs^2
    lam = mats[:, 0] * mats[:, 1] ** 2 - 2.0 * mu        # rho cp^2 - 2 mu
    Ylam = lam[:, None] * np.array([0.02, 0.01, 0.04])[None, :]
    Ymu = mu[:, None] * np.array([0.03, 0.015, 0.005])[None, :]
    star, Ap, Am = dg.visco_element_data(mesh.X, mats, omega, Ylam, Ymu, mesh.neigh)
    E = mesh.E
    star_d, Ap_d, Am_d = (torch.from_numpy(a).to(dev) for a in (star, Ap, Am))
    del star, Ap, Am
    nb = torch.from_numpy(np.ascontiguousarray(mesh.neigh, dtype=np.int32)).to(dev)
    fr = torch.from_numpy(mesh.face_rot).to(dev)
    rows = []
    for N in sorted({3, args.degree}):
        B, Bf = comb(N + 3, 3), comb(N + 2, 2)
        waves, per_cu = dg.visco_tune(N, 100000)
        ref = torch.from_numpy(dg.reference_blob(N)).to(dev)
        Q = torch.randn((E, 27, B), generator=g, dtype=torch.float64, device=dev)
        I = torch.empty_like(Q)
        tr = torch.empty((E, 4, 9, Bf), dtype=torch.float64, device=dev)
        dg.visco_step(N, Q, I, tr, star_d, Ap_d, Am_d, omega, ref, nb, fr, dt, 1)
        torch.cuda.synchronize()
        steps = 10
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dg.visco_step(N, Q, I, tr, star_d, Ap_d, Am_d, omega, ref, nb, fr, dt, steps)
        e1.record()
        torch.cuda.synchronize()
        el = e0.elapsed_time(e1) / 1e3 / steps
        flops, nbytes = visco_model(N)
        roof = pm.kernel_roofline(flops * E, nbytes * E, el, "f64")
        rows.append({"degree": N, "elements": E, "waves_per_workgroup": waves, "workgroups_per_cu": per_cu,
                     "ms_per_step": el * 1e3, "element_updates_per_s": E / el,
                     "useful_gflops": flops * E / el / 1e9, "flops_per_element": flops,
                     "bytes_per_element": nbytes, "bound": roof["bound"], "frac": roof["frac"]})
        log("visco degree %d, %d elements: %.3f ms/step, %.2f M element-updates/s, %.0f GFLOP/s (%s, %.3f)"
            % (N, E, el * 1e3, E / el / 1e6, flops * E / el / 1e9, roof["bound"], roof["frac"]))
        del Q, I, tr, ref
    top = rows[-1]
    out = {"metric": "element updates per second", "value": top["element_updates_per_s"], "unit": "1/s",
           "n_gpus": 1, "steps": 10, "warmup": 1, "ms_per_step": top["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "viscoelastic ADER-DG (27 quantities, 3 mechanisms), degree %d, %dx%dx%dx6 = "
                                  "%d-element jittered periodic cube-split mesh, random materials"
                                  % (top["degree"], args.n, args.n, args.n, E)},
           "visco": rows}
    print(json.dumps(out), flush=True)


def madness(args):
    """The separable contraction of Sec. 7 (Eq. stock_mra): batches of random
    p x p x p tensors (1 GiB of inputs, resident in HBM) and operator pairs of
    rank q, FP64 and FP32, through dg_mra_apply, timed with HIP events over 10
    launches on the launch stream; useful GFLOP/s counts the 12 p^3 q non-zero
    flops of the six-step chain per tensor (the paper's counting), GB/s the
    tensors read and written once."""
    import torch

    import paper_1903_11521_amd as dg
    from paper_1903_11521_amd import perfmodel as pm
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(1903)
    rows = []
    for dtype, name, sizes in ((torch.float64, "f64", (8, 16, 20)), (torch.float32, "f32", (8, 16, 24))):
        elem = 8 if dtype == torch.float64 else 4
        for p in sizes:
            for q in sorted({1, max(1, p // 2), p}):
                nb = max(1, (1 << 30) // (p ** 3 * elem))          # 1 GiB of input tensors
                S = torch.randn((nb, p, p, p), generator=g, dtype=dtype, device=dev)
                ops = [torch.randn(sh, generator=g, dtype=dtype, device=dev) for sh in ((p, q), (q, p)) * 3]
                R = torch.empty_like(S)
                dg.mra_apply(S, *ops, R=R)
                torch.cuda.synchronize()
                reps = 10
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    dg.mra_apply(S, *ops, R=R)
                e1.record()
                torch.cuda.synchronize()
                el = e0.elapsed_time(e1) / 1e3 / reps
                fl = 12.0 * p ** 3 * q * nb
                nbytes = 2.0 * p ** 3 * nb * elem
                roof = pm.kernel_roofline(fl, nbytes, el, name)
                rows.append({"dtype": name, "p": p, "q": q, "tensors": nb, "ms": el * 1e3,
                             "gflops": fl / el / 1e9, "gbs": nbytes / el / 1e9, "bound": roof["bound"],
                             "frac": roof["frac"]})
                log("mra %s p=%d q=%d: %.3f ms, %.1f GFLOP/s, %.0f GB/s (%s bound, %.2f of peak)"
                    % (name, p, q, el * 1e3, fl / el / 1e9, nbytes / el / 1e9, roof["bound"], roof["frac"]))
                del S, R, ops
    best = max(r["gflops"] for r in rows if r["dtype"] == "f64")
    out = {"metric": "useful GFLOP/s", "value": best, "unit": "GFLOP/s", "n_gpus": 1, "steps": 10, "warmup": 1,
           "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64 and f32", "data": "synthetic",
           "config": {"workload": "separable contraction of Sec. 7 (Eq. stock_mra): batches of p^3 tensors, "
                                  "rank-q operator pairs, p in 8..24, q in {1, p/2, p}"},
           "madness": rows}
    print(json.dumps(out), flush=True)


def serving(args):
    """Poisson arrivals of independent simulations: E ~ log-uniform[5k, 500k]
    elements (cube-split meshes), degree U{3..6}, U{50..500} steps, random
    materials; admitted by HBM footprint (80 % of free HBM), DOFs resident,
    steps of all admitted requests batched per launch (mixed precision by
    default)."""
    import torch

    import paper_1903_11521_amd as dg
    from paper_1903_11521_amd.serving import GpuExecutor, Request, Server
    from workload import cube_mesh, dt_from_mesh, random_dofs, random_materials, seed_for
    from math import comb
    prec = {"fp64": dg.DG_FP64, "fp32": dg.DG_FP32, "mixed": dg.DG_MIXED, "bf16x3": dg.DG_BF16X3}[args.precision]
    rng = np.random.Generator(np.random.PCG64(seed_for(4)))
    arrivals = np.cumsum(rng.exponential(1.0 / args.rate, args.requests))
    arrivals -= arrivals[0]
    sizes = np.exp(rng.uniform(np.log(5e3), np.log(500e3), args.requests))
    degrees = rng.integers(3, 7, args.requests)
    steps = rng.integers(50, 501, args.requests)

    def make(i):
        n = max(3, int(round((sizes[i] / 6) ** (1 / 3))))
        N = int(degrees[i])
        seed = seed_for(4) + 1000 * (i + 1)

        def build():
            mesh = cube_mesh(n, seed)
            mats = random_materials(mesh.E, seed)
            star, Ap, Am = dg.element_data(mesh.X, mats, mesh.neigh)
            return dict(dt=dt_from_mesh(mesh, mats), Q=random_dofs(mesh.E, 9, comb(N + 3, 3), seed), star=star,
                        Aplus=Ap, Aminus=Am, neigh=mesh.neigh, face_rot=mesh.face_rot)
        return Request(rid=i, degree=N, E=6 * n ** 3, n_steps=int(steps[i]), arrival=float(arrivals[i]),
                       build=build)

    free, _ = torch.cuda.mem_get_info()
    itemsize = 8 if prec == dg.DG_FP64 else 4
    srv = Server(GpuExecutor(prec), int(0.8 * free), itemsize, log=log)
    for i in range(args.requests):
        srv.submit(make(i))
    log("serving %d requests at %.1f req/s" % (args.requests, args.rate))
    srv.run()
    s = srv.summary()
    out = {"metric": "element-updates/s", "value": s["element_updates_per_s"], "unit": "element-updates/s",
           "n_gpus": 1, "steps": int(steps.sum()), "warmup": 0,
           "ms_per_step": s["p50_step_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": DTYPES[args.precision], "data": "synthetic",
           "config": {"workload": "serving: %d Poisson arrivals at %.1f req/s, cube-split meshes 5k-500k elements "
                                  "(log-uniform), degree 3..6, 50-500 steps each, continuous batching"
                                  % (args.requests, args.rate), "rate": args.rate},
           "serving": s}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: the multi-GPU sharding of the step is described in the "
                          "design notes but not implemented", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")      # 1 GiB
        c = torch.empty_like(a)
        for _ in range(3):
            c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": a.numel() * 8}), flush=True)
        return
    if args.workload == "batched":
        return batched(args)
    if args.workload == "fused":
        return fused(args)
    if args.workload == "madness":
        return madness(args)
    if args.workload == "lts":
        return lts(args)
    if args.workload == "lina":
        return lina(args)
    if args.workload == "visco":
        return visco(args)
    if args.workload == "serving":
        if args.precision == "fp64" and "--precision" not in sys.argv:
            args.precision = "mixed"
        return serving(args)
    import torch

    import paper_1903_11521_amd as dg
    from paper_1903_11521_amd import perfmodel as pm
    from workload import cube_mesh, dt_from_mesh, random_dofs, random_materials, seed_for

    N = args.degree
    prec = {"fp64": dg.DG_FP64, "fp32": dg.DG_FP32, "mixed": dg.DG_MIXED, "bf16x3": dg.DG_BF16X3}[args.precision]
    plan = dg.Plan(N, prec)
    if args.fusion != "auto":
        plan.set_fusion(args.fusion == "on")
    seed = seed_for(1)
    log("building mesh n=%d degree=%d" % (args.n, N))
    mesh = cube_mesh(args.n, seed)
    E = mesh.E
    mats = random_materials(E, seed)
    Q = random_dofs(E, 9, plan.B, seed)
    dt = dt_from_mesh(mesh, mats)
    star, Ap, Am = dg.element_data(mesh.X, mats, mesh.neigh)
    dev = torch.device("cuda:0")
    to = lambda a, dt_=None: (torch.from_numpy(np.ascontiguousarray(a)).to(dt_) if dt_ else
                              torch.from_numpy(np.ascontiguousarray(a))).to(dev)
    Qg = to(Q, plan.dtype)
    star_p = plan.pack_star(to(star))
    del star
    Apg, Amg = to(Ap), to(Am)
    del Ap, Am
    neigh, face_rot = to(mesh.neigh), to(mesh.face_rot)
    I = torch.empty(plan.dof_shape(E), dtype=plan.dtype, device=dev)
    tr = torch.empty(plan.trace_shape(E), dtype=plan.dtype, device=dev)
    tr2 = torch.empty_like(tr)      # second trace array: one launch per step
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    log("warmup %d steps" % args.warmup)
    plan.step(Qg, I, tr, star_p, Apg, Amg, neigh, face_rot, dt, args.warmup, traces_b=tr2)
    plan.sync()
    log("timed %d steps on %d elements" % (args.steps, E))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.step(Qg, I, tr, star_p, Apg, Amg, neigh, face_rot, dt, args.steps, traces_b=tr2)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    value = E * args.steps / elapsed

    # per-kernel launch durations with HIP events on the launch stream (the
    # timed region is one predictor, steps-1 fused-step calls, one corrector)
    log("per-kernel event timing")
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    for k in range(args.steps):
        ev[k][0].record(stream)
        plan.step_predict(Qg, star_p, dt, I, tr)
        ev[k][1].record(stream)
        plan.step_fused(Qg, I, tr, tr2, star_p, Apg, Amg, neigh, face_rot, dt)
        ev[k][2].record(stream)
        plan.step_correct(I, tr2, star_p, Apg, Amg, neigh, face_rot, Qg)
        ev[k][3].record(stream)
    torch.cuda.synchronize()
    mean_s = lambda a, b: float(np.mean([ev[k][a].elapsed_time(ev[k][b]) for k in range(args.steps)])) * 1e-3
    t_pred, t_fused, t_corr = mean_s(0, 1), mean_s(1, 2), mean_s(2, 3)
    itemsize = 8 if prec == dg.DG_FP64 else 4
    dtype = {dg.DG_FP64: "f64", dg.DG_BF16X3: "bf16x3"}.get(prec, "f32")
    counts = np.bincount(mesh.orient.ravel(), minlength=3) / mesh.orient.size
    sf = pm.stage_flops(N, counts)
    mb = pm.method_bytes(N, itemsize)
    lb = pm.layout_bytes(N, itemsize)
    # the dominant kernel: the fused launch where the plan fuses, else the
    # slower of corrector and predictor
    if plan.fuses_steps and args.steps > 1:
        kern, tk = "step_fused", t_fused
        kflops, kbytes, klayout = sf["step"], mb["step"], lb["step_fused"]
    else:
        kern, tk = max((("step_correct", t_corr), ("step_predict", t_pred)), key=lambda kt: kt[1])
        kflops, kbytes, klayout = sf[kern], mb[kern], lb[kern]
    roof = pm.kernel_roofline(kflops * E, kbytes * E, tk, dtype)
    roof["traffic"] = measured_traffic(kern, N, args.precision)
    roof["kernel"] = kern
    roof["kernel_ms"] = tk * 1e3
    roof["algorithmic_bytes_per_launch"] = kbytes * E
    roof["algorithmic_bytes_per_element"] = kbytes
    roof["algorithmic_flops_per_launch"] = kflops * E
    roof["layout_bytes_per_launch"] = klayout * E
    roof["layout_hbm_gbs"] = klayout * E / tk / 1e9
    step_rate = pm.step_roofline_rate(N, itemsize, dtype)
    out = {
        "metric": "element-updates/s", "value": value, "unit": "element-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPES[args.precision], "data": "synthetic",
        "config": {"workload": "elastic ADER-DG, degree %d (B=%d), %dx%dx%dx6 = %d-element jittered periodic "
                               "cube-split mesh, random materials, %d time steps, %s" % (
                                   N, plan.B, args.n, args.n, args.n, E, args.steps,
                                   "one launch per step (corrector fused with the next predictor)"
                                   if plan.fuses_steps else "predictor and corrector launch per step"),
                   "elements": E, "degree": N, "dt": dt},
        "useful_gflops": pm.PAPER_NZ_PER_UPDATE[N] * value / 1e9,
        "kernel_ms": dict({"step_predict": t_pred * 1e3, "step_correct": t_corr * 1e3},
                          **({"step_fused": t_fused * 1e3} if plan.fuses_steps else {})),
        "roofline": roof,
        "step_roofline": {"element_updates_per_s": step_rate, "frac": value / step_rate,
                          "flops_per_update": pm.PAPER_NZ_PER_UPDATE[N], "bytes_per_update": mb["step"],
                          "bound": pm.roofline(pm.PAPER_NZ_PER_UPDATE[N], mb["step"], dtype)["bound"]},
        "paper_context": "paper's best single-simulation O6 DP CPU figure: 1244 MDoF/s on 2x Xeon 8174 "
                         "(about 2.47 M element-updates/s, 15.3 % of NZ peak); context, not the target",
    }
    if not args.no_stages and prec != dg.DG_BF16X3:
        log("per-stage timing")
        out["stages"] = time_stages(plan, E, Qg, star_p, Apg, Amg, neigh, face_rot, dt, sf, mb, dtype, stream)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(args, mesh, mats, Q, dt)
    print(json.dumps(out), flush=True)


def time_stages(plan, E, Q, star_p, Ap, Am, neigh, face_rot, dt, sf, mb, dtype, stream, reps=5):
    """Each per-stage entry point (dg_predictor ... dg_neighbour_flux) on the
    same workload, HIP events on the launch stream, mean over `reps` calls
    after one warm-up; per stage its roofline fraction on the method bytes,
    and the element-updates/s of the step done stage by stage."""
    import torch
    from paper_1903_11521_amd import perfmodel as pm
    T = torch.empty(plan.deriv_shape(E), dtype=plan.dtype, device=Q.device)
    I = torch.empty(plan.dof_shape(E), dtype=plan.dtype, device=Q.device)
    Qs = Q.clone()
    calls = {
        "predictor": lambda: plan.predictor(Qs, star_p, dt, T),
        "time_integral": lambda: plan.time_integral(T, dt, I),
        "volume": lambda: plan.volume(I, star_p, Qs),
        "local_flux": lambda: plan.local_flux(I, Ap, Qs),
        "neighbour_flux": lambda: plan.neighbour_flux(I, neigh, face_rot, Am, Qs),
    }
    out, total = {}, 0.0
    for name, fn in calls.items():
        fn()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in evs:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        t = float(np.mean([a.elapsed_time(b) for a, b in evs])) * 1e-3
        total += t
        r = pm.kernel_roofline(sf[name] * E, mb[name] * E, t, dtype)
        out[name] = {"ms": t * 1e3, "bound": r["bound"], "achieved": r["achieved"], "unit": r["unit"],
                     "frac": r["frac"], "bytes_per_element": mb[name], "flops_per_element": sf[name]}
    out["per_stage_step_element_updates_per_s"] = E / total
    del T, I, Qs
    return out


if __name__ == "__main__":
    main()
