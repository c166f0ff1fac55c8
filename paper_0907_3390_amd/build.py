"""Build ``libtvd.so`` for gfx950 with hipcc, in-tree.

``python -m paper_0907_3390_amd.build`` (or ``build()``) compiles the HIP
kernels and the C ABI into ``paper_0907_3390_amd/_lib/libtvd.so``.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "_lib", "libtvd.so")
SOURCES = ["tvd_kernels.hip", "tvd_capi.hip"]
ARCH = "gfx950"

# packed FP32 instructions are turned off for every HIP translation unit;
# FMA contraction is off too: the kernels write every fused multiply-add
# explicitly, so the same expression rounds the same way everywhere
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=" + ARCH,
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-ffp-contract=off",
         "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False, extra=(), out: str = LIB) -> str:
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp%d" % os.getpid()
    cmd = (["hipcc"] + FLAGS + list(extra) + ["-I", INCLUDE, "-I", CSRC, "-o", tmp]
           + [os.path.join(CSRC, s) for s in SOURCES])
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libtvd.so")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
