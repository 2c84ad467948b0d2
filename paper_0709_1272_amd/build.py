"""Compile the HIP library ``libtileqr.so`` in-tree for gfx950.

Every source is built with ``-Xclang -target-feature -Xclang -packed-fp32-ops``
(packed FP32 instructions disabled; the host pass warns that it does not know
that target feature, which is harmless) and ``-ffp-contract=on``: a multiply
and an add are fused only inside one source expression, so every kernel that
inlines the same tile routine performs the same roundings (the serial driver
and the persistent scheduler then agree bit for bit).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtileqr.so")
# (source, extra defines, object name): the split-precision kernels are one
# source compiled once per arithmetic.
UNITS = [("tileqr_kernels.hip", [], "tileqr_kernels"),
         ("tileqr_mixed.hip", ["-DTQ_PREC=1"], "tileqr_mixed_bf16x2"),
         ("tileqr_mixed.hip", ["-DTQ_PREC=2"], "tileqr_mixed_fp16x2"),
         ("tileqr_mixed.hip", ["-DTQ_PREC=3"], "tileqr_mixed_bf16x3"),
         ("tileqr_solve.hip", [], "tileqr_solve"),
         ("tileqr_peak.hip", [], "tileqr_peak"),
         ("tileqr_noalloc.hip", [], "tileqr_noalloc"),
         ("tileqr_lsbatch.hip", [], "tileqr_lsbatch"),
         ("tileqr_tree.hip", [], "tileqr_tree"),
         ("tilechol.hip", [], "tilechol"),
         ("tilelu.hip", [], "tilelu"),
         ("tileqr_api.cpp", [], "tileqr_api"),
         ("tileqr_batched.cpp", [], "tileqr_batched")]
SOURCES = sorted({u[0] for u in UNITS})
ARCH = os.environ.get("TILEQR_ARCH", "gfx950")


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def build(verbose=False, jobs=None):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    procs = []
    for name, defs, oname in UNITS:
        src = os.path.join(CSRC, name)
        obj = os.path.join(CSRC, oname + ".o")
        cmd = [hipcc, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-ffp-contract=on",
               "-I", os.path.join(ROOT, "include")] + defs + ["-c", src, "-o", obj]
        if src.endswith(".cpp"):
            cmd[1:1] = ["-x", "hip"]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
        objs.append(obj)
    failed = False
    for pr, (src, _, _) in zip(procs, UNITS):
        out, _ = pr.communicate()
        text = out.decode(errors="replace")
        lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if pr.returncode != 0:
            failed = True
            sys.stderr.write(text)
        elif verbose and lines:
            sys.stderr.write("\n".join(lines) + "\n")
    if failed:
        raise RuntimeError("hipcc failed")
    tmp = LIB + ".tmp"
    subprocess.run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
