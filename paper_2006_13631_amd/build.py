"""Build ``libhlbm.so`` (gfx950) in-tree with hipcc.

Host code and the forward kernels are built without contraction of a*b+c
(the FP64 scalars that decide node classes and donor cells must follow their
written formulas, and a forward expression must round identically in every
kernel that inlines it); the adjoint kernels may use FMA. Packed FP32
instructions are disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhlbm.so")
SOURCES = ["api.hip", "kernels.hip", "adjoint.hip", "grid_host.cpp"]
ARCH = os.environ.get("HLBM_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for p in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if p and (os.path.isabs(p) and os.path.exists(p) or not os.path.isabs(p)):
            return p
    return "hipcc"


def build(verbose: bool = False) -> str:
    objs = []
    common = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wshadow",
              "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    procs = []
    for src in SOURCES:  # the sources compile independently, in parallel
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        # forward kernels: no contraction of a*b+c, so an expression rounds the
        # same wherever it is inlined (single-case and case-batched kernels
        # compute identical bits); the adjoint kernels may contract
        contract = "-ffp-contract=fast" if src == "adjoint.hip" else "-ffp-contract=off"
        cmd = [hipcc(), "-x", "hip", f"--offload-arch={ARCH}",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               *common, contract, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    failed = [cmd for p, cmd in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
