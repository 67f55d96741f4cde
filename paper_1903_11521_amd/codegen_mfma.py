"""Build-time generator of the matrix-core operand tables of the split-BF16
form.

In that form the reference-matrix contractions (K-tilde, K-hat, R^T, R-hat,
f^h; Sec. 5.1.1) run on v_mfma_f32_16x16x32_bf16 with three products per
contraction, A_hi B_hi + A_hi B_lo + A_lo B_hi, where x_hi = bf16(x) and
x_lo = bf16(x - x_hi), both rounded to nearest even.  A reference matrix is
the A operand; the B operand holds one quantity column of 16 elements (one
element per MFMA column).  This script writes, for every degree and matrix
family, the A-operand fragments of every 16 x 32 block that has a non-zero
entry, in the order in which the 64 lanes read them, and a table of fragment
numbers per (matrix, row tile, K step) with -1 for an all-zero block (the
kernels skip those at compile time).

Row mapping.  A lane (G = lane / 16, element e = lane % 16) owns, in row tile
m of a column, the four consecutive basis rows 16 m + 4 G + r (r = 0..3):
exactly the rows an MFMA output tile leaves in that lane, and four
consecutive values in memory.  In K step s the lane supplies its rows of
tiles 2 s and 2 s + 1: MFMA K index k = 8 G + v is basis row
32 s + 16 (v / 4) + 4 G + v % 4.  A chain of contractions (the derivative
recursion) therefore never moves data between lanes.

Fragment layout (per fragment, 2 KB): hi part, lane-major, 8 bf16 per lane
(the A operand: row i = lane % 16 of the tile, K indices 8 (lane / 16) ..
+7), then the lo part in the same order.
"""
from __future__ import annotations

import os

import numpy as np

from codegen import DEGREES, Emitter, load_host, matrices

# family index -> (name, description)
FAMS = ("kt", "kh", "rt", "rh", "fh")


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


def split(a):
    """hi = bf16(a), lo = bf16(a - hi) of the FP64 matrix entries (the
    difference is exact in FP64); |a - hi - lo| <= 2^-16 |a|."""
    a = np.asarray(a, dtype=np.float64)
    hi = bf16_rne(a)
    return hi, bf16_rne(a - hi)


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
    if fam == "rh":
        return [M["Rh"][s] for s in range(4)], B, Bf
    return [M["f"][h] for h in range(3)], Bf, Bf


def in_row(s, G, v):
    """Basis row of MFMA K index 8 G + v in K step s."""
    return 32 * s + 16 * (v // 4) + 4 * G + v % 4


def fragments(mats, rows_out, rows_in):
    MT = (rows_out + 15) // 16
    NKS = (rows_in + 31) // 32
    idx = -np.ones((len(mats), MT, NKS), dtype=np.int64)
    blocks = []
    for a, A in enumerate(mats):
        for mo in range(MT):
            for ks in range(NKS):
                frag = np.zeros((64, 8))
                for lane in range(64):
                    r = 16 * mo + lane % 16
                    G = lane // 16
                    for v in range(8):
                        c = in_row(ks, G, v)
                        if r < rows_out and c < rows_in:
                            frag[lane, v] = A[r, c]
                if np.any(frag != 0.0):
                    idx[a, mo, ks] = len(blocks)
                    blocks.append(frag)
    return idx, blocks, MT, NKS


def dense_from_fragments(blocks, idx, rows_out, rows_in, part):
    """Inverse map (for tests): the matrices a fragment table encodes,
    part = 0 (hi), 1 (lo) or None (hi + lo)."""
    nm, MT, NKS = idx.shape
    out = np.zeros((nm, rows_out, rows_in))
    for a in range(nm):
        for mo in range(MT):
            for ks in range(NKS):
                f = idx[a, mo, ks]
                if f < 0:
                    continue
                hi, lo = split(blocks[f])
                val = hi if part == 0 else lo if part == 1 else hi + lo
                for lane in range(64):
                    r = 16 * mo + lane % 16
                    for v in range(8):
                        c = in_row(ks, lane // 16, v)
                        if r < rows_out and c < rows_in:
                            out[a, r, c] = val[lane, v]
    return out


def _ints(a):
    if a.ndim == 1:
        return "{" + ", ".join(str(int(v)) for v in a) + "}"
    return "{" + ", ".join(_ints(x) for x in a) + "}"


def emit(em, N, M):
    for f, fam in enumerate(FAMS):
        mats, ro, ri = family(M, N, fam)
        idx, blocks, MT, NKS = fragments(mats, ro, ri)
        name = "mfr_%s_%d" % (fam, N)
        words = []
        for b in blocks:
            hi, lo = split(b)
            for part in (hi, lo):
                bits = bf16_bits(part).reshape(64, 8).astype(np.uint32)
                # two bf16 per 32-bit word, lower K index in the low half
                w = bits[:, 0::2] | (bits[:, 1::2] << 16)
                words.extend(int(x) for x in w.ravel())
        if not words:
            words = [0]
        em("__device__ const unsigned int %s[] __attribute__((aligned(16))) = {%s};"
           % (name, ", ".join("0x%08x" % x for x in words)))
        em("template <> struct Frag<%d, %d> {" % (N, f))
        em("  static constexpr int NMAT = %d, MT = %d, NKS = %d, ROWS_OUT = %d, ROWS_IN = %d, NFRAG = %d;"
           % (len(mats), MT, NKS, ro, ri, len(blocks)))
        em("  static constexpr int idx[%d][%d][%d] = %s;" % (len(mats), MT, NKS, _ints(idx)))
        em("  __device__ static const unsigned int *data() { return %s; }" % name)
        em("};")


def generate(host_lib_path, out_path):
    lib = load_host(host_lib_path)
    em = Emitter()
    em("// GENERATED by codegen_mfma.py from the library's reference-matrix generator. Do not edit.")
    em("#pragma once")
    em("namespace mft {")
    em("template <int N, int FAM> struct Frag;")
    em("enum { KT = 0, KH = 1, RT = 2, RH = 3, FH = 4 };")
    for N in DEGREES:
        emit(em, N, matrices(lib, N))
    em("}  // namespace mft")
    with open(out_path + ".tmp", "w") as fh:
        fh.write("\n".join(em.lines) + "\n")
    os.replace(out_path + ".tmp", out_path)


if __name__ == "__main__":
    import sys
    generate(sys.argv[1], sys.argv[2])
