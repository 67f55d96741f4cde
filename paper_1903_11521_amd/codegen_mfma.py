"""Build-time generator of the matrix-core operand tables.

The matrix-core (MFMA) forms of the element kernels multiply the reference
matrices (K-tilde, K-hat, R^T, R-hat; Sec. 5.1.1) with tiles of 16 elements'
degrees of freedom.  A reference matrix is the A operand of
v_mfma_f32_16x16x4_f32 (FP32 form) or of three v_mfma_f32_16x16x32_bf16
products (3xBF16 form: A = A_hi + A_lo, each rounded to bfloat16 to nearest
even).  This script writes, for every degree, the A-operand fragments of every
non-zero 16-row block, in the order in which a lane reads them, plus a table
of block indices (-1 for an all-zero block, which the kernels skip at compile
time).

Row mapping.  A lane (group G = lane / 16, element e = lane % 16) owns the
rows 4 o + G (o = 0, 1, ...) of every quantity column of its element: the
rows of an MFMA output tile m land in the lane as o = 4 m + r, which is what
the next contraction reads as its input, so a chain of contractions (the
derivative recursion) never moves data between lanes.  Output row i of tile m
(i = 4 G + r in the hardware layout) is basis row 16 m + 4 r + G; input
(K) index k of K-step s is basis row 4 s + k for the FP32 form and
4 (8 s + k % 8) + k // 8 for the 3xBF16 form (a lane supplies 8 of its own
rows per step).
"""
from __future__ import annotations

import numpy as np

from codegen import DEGREES, matrices

KINDS = {1: "f32", 2: "bf16x3"}
FAMS = ("kt", "kh", "rt", "rh")   # K-tilde^d, K-hat^d, R^s transposed, R-hat^s


def bf16_rne(x):
    """Round float64 values to bfloat16 (8 significant bits), to nearest even;
    returns float64 values exactly representable in bfloat16."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                    # x = m 2^e, 0.5 <= |m| < 1
    q = m * 256.0                         # 8 significant bits before the point
    r = np.round(q)                       # numpy rounds half to even
    return np.ldexp(r / 256.0, e)


def bf16_bits(v):
    """Bit patterns (uint16) of float64 values that are exact bfloat16."""
    f = np.asarray(v, dtype=np.float32)
    assert np.array_equal(f.astype(np.float64), np.asarray(v, dtype=np.float64))
    return (f.view(np.uint32) >> 16).astype(np.uint16)


def family(M, N, fam):
    """(list of matrices [rows_out][rows_in], rows_out, rows_in)."""
    B, Bf = M["B"], M["Bf"]
    Bv = N * (N + 1) * (N + 2) // 6
    if fam == "kt":
        return [M["Kt"][d][:Bv, :] for d in range(3)], Bv, B
    if fam == "kh":
        return [M["Kh"][d][:, :Bv] for d in range(3)], B, Bv
    if fam == "rt":
        return [M["R"][s].T for s in range(4)], Bf, B
    return [M["Rh"][s] for s in range(4)], B, Bf


def out_row(mo, i):
    return 16 * mo + 4 * (i % 4) + i // 4


def in_rows(kind, ks, G):
    if kind == 1:
        return [4 * ks + G]
    return [4 * (8 * ks + v) + G for v in range(8)]


def fragments(mats, rows_out, rows_in, kind):
    rpl = 1 if kind == 1 else 8
    MT = (rows_out + 15) // 16
    own_in = (rows_in + 3) // 4
    NKS = (own_in + rpl - 1) // rpl
    idx = -np.ones((len(mats), MT, NKS), dtype=np.int64)
    blocks = []
    for a, A in enumerate(mats):
        for mo in range(MT):
            for ks in range(NKS):
                frag = np.zeros((64, rpl))
                for lane in range(64):
                    i, G = lane % 16, lane // 16
                    r = out_row(mo, i)
                    for v, c in enumerate(in_rows(kind, ks, G)):
                        if r < rows_out and c < rows_in:
                            frag[lane, v] = A[r, c]
                if np.any(frag != 0.0):
                    idx[a, mo, ks] = len(blocks)
                    blocks.append(frag)
    return idx, blocks, MT, NKS


def _ints(a):
    if a.ndim == 1:
        return "{" + ", ".join(str(int(v)) for v in a) + "}"
    return "{" + ", ".join(_ints(x) for x in a) + "}"


def emit(em, N, M, kind):
    for f, fam in enumerate(FAMS):
        mats, ro, ri = family(M, N, fam)
        idx, blocks, MT, NKS = fragments(mats, ro, ri, kind)
        name = "mfa_%s_%d_%d" % (fam, N, kind)
        data = np.concatenate([b.ravel() for b in blocks]) if blocks else np.zeros(1)
        if kind == 1:
            vals = ", ".join("%.9ef" % float(np.float32(v)) for v in data)
            em("__device__ const float %s[] __attribute__((aligned(16))) = {%s};" % (name, vals))
        else:
            hi = bf16_rne(data)
            lo = bf16_rne(data - hi)
            em("__device__ const unsigned short %s_hi[] __attribute__((aligned(16))) = {%s};"
               % (name, ", ".join(str(int(v)) for v in bf16_bits(hi))))
            em("__device__ const unsigned short %s_lo[] __attribute__((aligned(16))) = {%s};"
               % (name, ", ".join(str(int(v)) for v in bf16_bits(lo))))
        em("template <> struct MTab<%d, %d, %d> {" % (N, kind, f))
        em("  static constexpr int NMAT = %d, MT = %d, NKS = %d, ROWS_OUT = %d, ROWS_IN = %d;" % (len(mats), MT, NKS, ro, ri))
        em("  static constexpr int idx[%d][%d][%d] = %s;" % (len(mats), MT, NKS, _ints(idx)))
        if kind == 1:
            em("  __device__ static const float *data() { return %s; }" % name)
        else:
            em("  __device__ static const unsigned short *hi() { return %s_hi; }" % name)
            em("  __device__ static const unsigned short *lo() { return %s_lo; }" % name)
        em("};")


def generate(host_lib_path, out_path):
    from codegen import Emitter, load_host
    import os
    lib = load_host(host_lib_path)
    em = Emitter()
    em("// GENERATED by codegen_mfma.py from the library's reference-matrix generator. Do not edit.")
    em("#pragma once")
    em("namespace mft {")
    em("template <int N, int KIND, int FAM> struct MTab;")
    for N in DEGREES:
        M = matrices(lib, N)
        for kind in KINDS:
            emit(em, N, M, kind)
    em("}  // namespace mft")
    with open(out_path + ".tmp", "w") as fh:
        fh.write("\n".join(em.lines) + "\n")
    os.replace(out_path + ".tmp", out_path)


if __name__ == "__main__":
    import sys
    generate(sys.argv[1], sys.argv[2])
