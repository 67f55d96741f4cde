"""Build-time generator of the sparse element-kernel code.

The reference matrices are element independent, so their sparsity pattern and
values are compile-time constants (the paper stores such matrices inside the
generated code, Sec. 4.9).  This script asks the library's own host generator
(csrc/refmat.cpp, loaded through a small host-only shared object) for the
matrices of every supported degree and writes `dg_generated.h`:

  * per-column functors that apply one column of a matrix to register arrays
    with fully unrolled FMAs, one FMA per non-zero.  FP32 kernels take the
    matrix entry as a literal, which the compiler folds into the FMA.  FP64
    kernels read it from a per-degree constant table in consumption order:
    an FP64 literal costs two scalar moves of 12 bytes each, while table
    entries arrive eight at a time through one scalar load, which shrinks
    the code and its scalar issue.

Column order conventions (matching the consumption order of the kernels):
  KtCol<N,L>    acc[k] += Kt^d[k][L] * x_d           (predictor, d = 0..2)
  KhCol<N,L>    acc[k] += Kh^d[k][L] * x_d           (volume)
  RCol<N,S,L>   tr[m]  += R^S[L][m]  * v             (face trace of row L)
  RhCol<N,S,M>  acc[k] += Rh^S[k][M] * g             (lift of face row M)
  FApply<N,H>   out[m]  = sum_n f^H[m][n] in[n]      (orientation change)
"""
from __future__ import annotations

import ctypes
import os
import sys

import numpy as np

DEGREES = (2, 3, 4, 5, 6)


def load_host(lib_path):
    lib = ctypes.CDLL(lib_path)
    lib.dg_reference_blob_size.restype = ctypes.c_int64
    lib.dg_reference_blob_size.argtypes = [ctypes.c_int]
    lib.dg_reference_matrices.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    return lib


def matrices(lib, N):
    n = lib.dg_reference_blob_size(N)
    buf = np.zeros(n)
    rc = lib.dg_reference_matrices(N, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise RuntimeError("reference matrix generation failed")
    B = (N + 1) * (N + 2) * (N + 3) // 6
    Bf = (N + 1) * (N + 2) // 2
    o = 0

    def take(shape):
        nonlocal o
        sz = int(np.prod(shape))
        a = buf[o:o + sz].reshape(shape)
        o += sz
        return a

    return dict(B=B, Bf=Bf, Kh=take((3, B, B)), Kt=take((3, B, B)), R=take((4, B, Bf)),
                Rh=take((4, B, Bf)), f=take((3, Bf, Bf)))


class Consts:
    """The FP64 entries of one degree in the order the code consumes them."""

    def __init__(self, N):
        self.N = N
        self.values = []

    def __call__(self, v):
        """A matrix entry: the table entry in FP64 kernels, a literal of the
        kernel's precision (rounded once, at compile time) otherwise."""
        self.values.append(float(v))
        return "dg_kv<real>(dg_kc_%d[%d], %r)" % (self.N, len(self.values) - 1, float(v))


class Emitter:
    def __init__(self):
        self.lines = []

    def __call__(self, s=""):
        self.lines.append(s)


# A scheduling fence after every FENCE FMAs of a functor, in FP32 code only.
# The fences date from FP64 literals, each materialised by two scalar moves:
# without them the scheduler hoisted the moves of a whole row block,
# overflowed the SGPRs and spilled them into VGPR lanes.  With the FP64 table
# the loads may run ahead freely (1-3 % faster at degrees 5 and 6 without
# fences); the FP32 kernels keep the schedule they were tuned with.
FENCE = 16


def fenced(stms):
    out = []
    for i, s in enumerate(stms):
        out.append(s)
        if (i + 1) % FENCE == 0 and i + 1 < len(stms):
            out.append("if constexpr (sizeof(real) == 4) __builtin_amdgcn_sched_barrier(0);")
    return out


def _degrees(N):
    return [i + j + k for dd in range(N + 1) for k in range(dd + 1) for j in range(dd - k + 1)
            for i in (dd - j - k,)]


def check_structure(N, M):
    """Properties the kernels rely on: Kt^d[k][l] != 0 only for deg(k) <
    deg(l) (derivative staircase), Kh non-zero only in the first
    C(N+2,3) columns, f^h block diagonal by face-basis degree."""
    fdeg = np.array([dd for dd in range(N + 1) for _ in range(dd + 1)])
    for h in range(3):
        m, n = np.nonzero(M["f"][h])
        if not np.all(fdeg[m] == fdeg[n]):
            raise RuntimeError("f is not block diagonal by degree")
    deg = np.array(_degrees(N))
    for d in range(3):
        k, l = np.nonzero(M["Kt"][d])
        if not np.all(deg[k] < deg[l]):
            raise RuntimeError("Ktilde breaks the staircase structure")
        k, l = np.nonzero(M["Kh"][d])
        if len(l) and l.max() >= N * (N + 1) * (N + 2) // 6:
            raise RuntimeError("Khat has non-zeros beyond the degree N-1 columns")


def gen_degree(out, N, M):
    check_structure(N, M)
    B, Bf = M["B"], M["Bf"]
    em = Emitter()
    _lit = Consts(N)
    # K-tilde, column(L)-major, then d, then k
    for key, nm in (("Kt", "KtCol"), ("Kh", "KhCol")):
        A = M[key]
        bodies = []
        for L in range(B):
            stm = []
            for d in range(3):
                for k in range(B):
                    v = A[d, k, L]
                    if v != 0.0:
                        stm.append(f"acc[{k}] = fma({_lit(v)}, x{d}, acc[{k}]);")
            bodies.append(stm)
        for L in range(B):
            em(f"template <> struct {nm}<{N}, {L}> {{ template <typename real> __device__ __forceinline__ static void apply(real x0, real x1, real x2, real* __restrict__ acc) {{")
            for s in fenced(bodies[L]):
                em("  " + s)
            em("} };")
    # R: trace, row(L)-major per face S, then m
    for S in range(4):
        for L in range(B):
            stm = []
            for m in range(Bf):
                v = M["R"][S, L, m]
                if v != 0.0:
                    stm.append(f"tr[{m}] = fma({_lit(v)}, v, tr[{m}]);")
            em(f"template <> struct RCol<{N}, {S}, {L}> {{ template <typename real> __device__ __forceinline__ static void apply(real v, real* __restrict__ tr) {{")
            for s in fenced(stm):
                em("  " + s)
            em("} };")
    # R-hat: lift, column(M)-major per face, then k
    for S in range(4):
        for Mi in range(Bf):
            stm = []
            for k in range(B):
                v = M["Rh"][S, k, Mi]
                if v != 0.0:
                    stm.append(f"acc[{k}] = fma({_lit(v)}, g, acc[{k}]);")
            em(f"template <> struct RhCol<{N}, {S}, {Mi}> {{ template <typename real> __device__ __forceinline__ static void apply(real g, real* __restrict__ acc) {{")
            for s in fenced(stm):
                em("  " + s)
            em("} };")
    # f^h: full apply
    for H in range(3):
        em(f"template <> struct FApply<{N}, {H}> {{ template <typename real> __device__ __forceinline__ static void apply(const real* __restrict__ in, real* __restrict__ out) {{")
        for m in range(Bf):
            terms = [(n, M["f"][H, m, n]) for n in range(Bf) if M["f"][H, m, n] != 0.0]
            if not terms:
                em(f"  out[{m}] = real(0);")
                continue
            n0, v0 = terms[0]
            em(f"  out[{m}] = {_lit(v0)} * in[{n0}];")
            for n, v in terms[1:]:
                em(f"  out[{m}] = fma({_lit(v)}, in[{n}], out[{m}]);")
        em("} };")
    # f^h one degree block at a time (f^h is block diagonal by degree: the
    # orientation maps are measure-preserving affine symmetries of the
    # reference triangle, which keep each degree's orthogonal subspace)
    for H in range(3):
        for d in range(N + 1):
            off = d * (d + 1) // 2
            em(f"template <> struct FBlock<{N}, {H}, {d}> {{ template <typename real> __device__ __forceinline__ static void apply(const real* __restrict__ in, real* __restrict__ out) {{")
            for i in range(d + 1):
                terms = [(j, M["f"][H, off + i, off + j]) for j in range(d + 1) if M["f"][H, off + i, off + j] != 0.0]
                if not terms:
                    em(f"  out[{i}] = real(0);")
                    continue
                j0, v0 = terms[0]
                em(f"  out[{i}] = {_lit(v0)} * in[{j0}];")
                for j, v in terms[1:]:
                    em(f"  out[{i}] = fma({_lit(v)}, in[{j}], out[{i}]);")
            em("} };")
    # the degree's FP64 table first, then its functors
    out(f"static __constant__ double dg_kc_{N}[{len(_lit.values)}] = {{")
    for i in range(0, len(_lit.values), 4):
        out("  " + ", ".join("%r" % v for v in _lit.values[i:i + 4]) + ",")
    out("};")
    out.lines.extend(em.lines)


def flop_counts(M, N):
    """Non-zero multiply-add pairs per element-column of the generated code."""
    B, Bf = M["B"], M["Bf"]
    bd = [(N - d + 1) * (N - d + 2) * (N - d + 3) // 6 for d in range(N + 1)]
    ck = sum(int(np.count_nonzero(M["Kt"][:, :, :bd[d]])) for d in range(N))
    vol = int(np.count_nonzero(M["Kh"]))
    r = [int(np.count_nonzero(M["R"][s])) for s in range(4)]
    rh = [int(np.count_nonzero(M["Rh"][s])) for s in range(4)]
    f = [int(np.count_nonzero(M["f"][h])) for h in range(3)]
    return dict(ck=ck, vol=vol, R=r, Rh=rh, f=f, bd=bd)


def generate(host_lib_path, out_path):
    lib = load_host(host_lib_path)
    em = Emitter()
    em("// GENERATED by codegen.py from the library's reference-matrix generator. Do not edit.")
    em("#pragma once")
    em("template <int N, int L> struct KtCol;")
    em("template <int N, int L> struct KhCol;")
    em("template <int N, int S, int L> struct RCol;")
    em("template <int N, int S, int M> struct RhCol;")
    em("template <int N, int H> struct FApply;")
    em("template <int N, int H, int D> struct FBlock;")
    em("// a matrix entry: from the constant table in FP64, as the literal otherwise")
    em("template <typename real> __device__ __forceinline__ real dg_kv(const double &table, double lit)")
    em("{ if constexpr (sizeof(real) == 8) return table; else return real(lit); }")
    stats = {}
    for N in DEGREES:
        M = matrices(lib, N)
        gen_degree(em, N, M)
        stats[N] = flop_counts(M, N)
    with open(out_path + ".tmp", "w") as fh:
        fh.write("\n".join(em.lines) + "\n")
    os.replace(out_path + ".tmp", out_path)
    return stats


if __name__ == "__main__":
    generate(sys.argv[1], sys.argv[2])
