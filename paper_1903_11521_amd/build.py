"""Build the gfx950 element-kernel library in-tree.

Steps: (1) host-only build of the reference-matrix generator, (2) code
generation of the sparse contraction code from those matrices, (3) hipcc of
one translation unit per polynomial degree plus the host C ABI, (4) link
into paper_1903_11521_amd/libdg_mi355x.so.
"""
from __future__ import annotations

import hashlib
import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
GEN = os.path.join(BUILD, "gen")
LIB = os.path.join(PKG, "libdg_mi355x.so")
DEGREES = (2, 3, 4, 5, 6)

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
HIP_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-I" + GEN]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed: %s\n%s" % (" ".join(cmd), r.stdout[-6000:]))
    return r.stdout


def kernel_usage(text):
    """Per-kernel VGPR/AGPR/scratch/occupancy from the compiler's resource remarks."""
    usage, cur = {}, None
    for line in text.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            usage[cur] = {}
            continue
        m = re.search(r"(VGPRs|AGPRs|ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]): (\d+)", line)
        if m and cur:
            usage[cur][m.group(1).split(" ")[0]] = int(m.group(2))
    return usage


def _stamp(cmd, inputs):
    """Hash of a compile command and the contents of its inputs."""
    h = hashlib.sha256(" ".join(cmd).encode())
    for f in inputs:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _compile(cmd, inputs, incremental):
    """Run one compile step; with `incremental`, skip it when the object's
    stamp matches (its remarks are then read back from the stamp file)."""
    out = cmd[cmd.index("-o") + 1]
    st = out + ".stamp"
    key = _stamp(cmd, inputs)
    if incremental and os.path.exists(out) and os.path.exists(st):
        with open(st) as fh:
            old = fh.read()
        if old.startswith(key + "\n"):
            return old[len(key) + 1:]
    text = _run(cmd)
    with open(st, "w") as fh:
        fh.write(key + "\n" + text)
    return text


def build(verbose: bool = False, jobs: int | None = None, incremental: bool = False) -> str:
    os.makedirs(GEN, exist_ok=True)
    host = os.path.join(BUILD, "librefmat_host.so")
    _run(["g++", "-O2", "-shared", "-fPIC", "-DDG_REFMAT_STANDALONE", os.path.join(CSRC, "refmat.cpp"),
          "-o", host])
    sys.path.insert(0, PKG)
    try:
        import codegen  # noqa: E402  (build-time helper beside this file)
    finally:
        sys.path.pop(0)
    codegen.generate(host, os.path.join(GEN, "dg_generated.h"))
    sys.path.insert(0, PKG)
    try:
        import codegen_mfma  # noqa: E402
    finally:
        sys.path.pop(0)
    codegen_mfma.generate(host, os.path.join(GEN, "mfma_tables.h"))
    objs = []
    cmds = []
    deps = {}    # object -> the sources and headers it is built from
    c = lambda *names: [os.path.join(CSRC, n) for n in names]
    gen_sparse = [os.path.join(GEN, "dg_generated.h")]
    gen_mfma = [os.path.join(GEN, "mfma_tables.h")]
    pub = [os.path.join(ROOT, "include", "dg.h")]
    for n in DEGREES:
        o = os.path.join(BUILD, "dg_launch_%d.o" % n)
        cmds.append([HIPCC] + HIP_FLAGS + ["-DDG_DEGREE=%d" % n, "-Rpass-analysis=kernel-resource-usage",
                                           "-c", os.path.join(CSRC, "dg_launch.hip"), "-o", o])
        deps[o] = c("dg_launch.hip", "dg_kernels.hip", "dg_common.h", "dg_tables.h", "step_predict_body.inc",
                    "step_correct_body.inc") + gen_sparse
        objs.append(o)
    for n in DEGREES:
        o = os.path.join(BUILD, "mfma_launch_%d.o" % n)
        cmds.append([HIPCC] + HIP_FLAGS + ["-DDG_DEGREE=%d" % n, "-Rpass-analysis=kernel-resource-usage",
                                           "-c", os.path.join(CSRC, "mfma_launch.hip"), "-o", o])
        deps[o] = c("mfma_launch.hip", "mfma_kernels.hip", "dg_common.h", "dg_tables.h") + gen_mfma
        objs.append(o)
    for src in ("dg_api.cpp", "refmat.cpp", "elements.cpp", "dg_noalloc.hip", "mra_kernels.hip", "lts.cpp",
                "lts_kernels.hip", "lina.cpp", "lina_kernels.hip", "visco.cpp", "visco_kernels.hip"):
        o = os.path.join(BUILD, src.replace(".cpp", ".o").replace(".hip", ".o"))
        cmds.append([HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, src), "-o", o])
        deps[o] = c(src, "dg_internal.h", "dg_tables.h", "refmat.h", "lts_internal.h", "lina_internal.h",
                    "visco_internal.h", "dg_common.h") + pub
        objs.append(o)
    jobs = jobs or min(8, os.cpu_count() or 4)
    with ThreadPoolExecutor(jobs) as ex:
        outs = list(ex.map(lambda cmd: _compile(cmd, deps[cmd[cmd.index("-o") + 1]], incremental), cmds))
    usage = kernel_usage("\n".join(outs))
    spills = {k: v for k, v in usage.items() if v.get("ScratchSize", 0) > 0}
    # the sparse-FMA family must not spill; the matrix-core family's spills
    # are reported in kernel_usage.txt
    hard = sorted(k for k in spills if not k.startswith("_ZN3dgm"))
    if hard:
        raise RuntimeError("kernels spill to scratch memory: %s" % hard)
    with open(os.path.join(BUILD, "kernel_usage.txt"), "w") as fh:
        for name, v in sorted(usage.items()):
            fh.write("%s %s\n" % (name, " ".join("%s=%s" % kv for kv in sorted(v.items()))))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))
