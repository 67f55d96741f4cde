"""Work and traffic model of the element kernels, for rooflines.

Two kinds of byte counts per element:
  * method bytes: the arrays the scheme itself needs (Q, I, the Taylor
    derivatives where a stage writes them out, packed star, A+/A-, the
    neighbour tables), each read or written once, the neighbours' I with
    ideal reuse.  These are the roofline's algorithmic bytes; they do not
    depend on how a kernel lays out its work arrays.
  * layout bytes: what this library's step kernels move by design, which adds
    the face traces (written by the predictor, read by the own and the
    neighbour corrector).  Reported beside the method bytes, never as them.

Flops are non-zero flops (one multiply and one add per structural non-zero
product of the reference matrices, the paper's counting, Sec. 4.3) of the
paper's formulation of each stage (Sec. 5.1.1): the local and the neighbour
flux each project I onto the face and each end in a lift.  For a whole
element-update the paper's own implied figure per order is used (its appendix
tables give MDoF/s and NZ GFLOPS for the same runs).
"""
from __future__ import annotations

from math import comb

PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3,   # vector FP64 and FP32 (MI355X datasheet)
               "bf16x3": 2500.0 / 3}       # dense BF16 matrix cores, three products per useful one

# Non-zero flops per element-update implied by the paper's SeisSol runs
# (NZ GFLOPS / (MDoF/s / (9 B))), orders 3..7 = degrees 2..6.
PAPER_NZ_PER_UPDATE = {2: 19.4e3, 3: 50.7e3, 4: 118e3, 5: 253.5e3, 6: 506e3}


def sizes(N):
    B, Bf = comb(N + 3, 3), comb(N + 2, 2)
    bd = [comb(N - d + 3, 3) for d in range(N + 1)]   # non-zero rows of D^d (staircase)
    return B, Bf, bd, comb(N + 2, 3)


def method_bytes(N, itemsize=8, P=9):
    """Algorithmic bytes per element of each stage and of the step.  DOF-like
    arrays and the star matrices have `itemsize` bytes per value, A+/A- are
    FP64 in every form."""
    B, Bf, bd, Bv = sizes(N)
    q = P * B * itemsize                     # Q or I of one element
    star = 81 * itemsize                     # packed star, 3 x 27 values (elastic)
    apm = 4 * 81 * 8                         # A+ or A- of one element
    tables = 4 * 4 + 4                       # neigh int32 + face_rot uint8
    tstair = sum(bd) * P * itemsize          # derivatives, staircase rows only
    out = {
        "predictor": q + star + tstair,                       # CK with derivative write-out
        "time_integral": tstair + q,
        "volume": Bv * P * itemsize + star + 2 * q,           # only Bv rows of I contribute
        "local_flux": q + apm + 2 * q,
        "neighbour_flux": q + apm + tables + 2 * q,           # neighbours' I with ideal reuse
        "neighbour_flux_noreuse": 4 * q + apm + tables + 2 * q,
        "step_predict": q + star + q,                         # CK + TI fused, writes I only
        "step_correct": q + star + 2 * apm + tables + 2 * q,  # I, star, A+-, tables, Q read+write
    }
    # one whole step: Q read and written, I written and read back (by the
    # element and its neighbours, ideal reuse), star, A+-, tables
    out["step"] = 2 * q + 2 * q + star + 2 * apm + tables
    return out


def layout_bytes(N, itemsize=8, P=9):
    """Bytes per element the step kernels move by design (face traces
    included), each array once, neighbour traces with ideal reuse."""
    B, Bf, _, _ = sizes(N)
    q = P * B * itemsize
    tr = 4 * P * Bf * itemsize
    star = 81 * itemsize
    apm = 4 * 81 * 8
    tables = 4 * 4 + 4
    predict = q + star + q + tr
    correct = q + tr + tr + star + 2 * apm + tables + 2 * q
    return {"step_predict": predict, "step_correct": correct, "step": predict + correct,
            "step_fused": correct + q + tr}


def stage_flops(N, orient_counts=None):
    """Non-zero flops per element of each stage in the paper's formulation,
    and of the library's step kernels as they run (traces computed once per
    element in the predictor, one lift per face in the corrector counted as
    two, like the paper)."""
    from ._lib import flop_model
    f = flop_model(N, orient_counts)
    tr = f["traces"]
    return {
        "predictor": f["ck"],
        "time_integral": f["ti"],
        "volume": f["volume"],
        "local_flux": tr + f["local"],
        "neighbour_flux": tr + f["neighbour"],
        "step_predict": f["step_predict"],
        "step_correct": f["step_correct"],
        "step": f["step"],
    }


def roofline(flops, nbytes, dtype="f64"):
    """Roofline of one kernel or step: the bound, its time (s) per unit of
    (flops, bytes) and the peak it is measured against."""
    peak_f = PEAK_TFLOPS[dtype] * 1e12
    t_f = flops / peak_f
    t_b = nbytes / (PEAK_HBM_GBS * 1e9)
    if t_b >= t_f:
        return {"bound": "hbm", "t_roof": t_b, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    return {"bound": "alu", "t_roof": t_f, "peak": PEAK_TFLOPS[dtype], "unit": "TFLOP/s"}


def kernel_roofline(flops, nbytes, seconds, dtype="f64"):
    """Roofline entry of a measured kernel: achieved algorithmic rate of the
    bounding resource, its peak and the fraction."""
    r = roofline(flops, nbytes, dtype)
    if r["bound"] == "hbm":
        achieved = nbytes / seconds / 1e9
    else:
        achieved = flops / seconds / 1e12
    return {"bound": r["bound"], "achieved": achieved, "peak": r["peak"], "unit": r["unit"],
            "frac": achieved / r["peak"], "t_roof_s": r["t_roof"]}


def step_roofline_rate(N, itemsize=8, dtype="f64"):
    """Roofline element-updates/s of the whole step: the paper-implied NZ
    flops per element-update against the vector peak, and the method bytes of
    a step against HBM."""
    f = PAPER_NZ_PER_UPDATE[N]
    b = method_bytes(N, itemsize)["step"]
    return 1.0 / roofline(f, b, dtype)["t_roof"]


def mixed_method_bytes(N, P=9):
    """Method bytes of a step of the mixed forms (FP32 DOFs and star, FP64
    A+/A-)."""
    return method_bytes(N, 4, P)
