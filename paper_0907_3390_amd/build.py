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
SOURCES = ["tvd_k_stream_f32.hip", "tvd_k_batched_f32_e16.hip", "tvd_k_stream_f64.hip",
           "tvd_kernels.hip", "tvd_k_batched_f32_e8.hip", "tvd_k_batched_f64_e8.hip",
           "tvd_k_fused.hip", "tvd_pipeline.hip", "tvd_capi.hip"]
OBJDIR = os.path.join(HERE, "_build")
ARCH = "gfx950"

# packed FP32 instructions are turned off for every HIP translation unit;
# FMA contraction is off too: the kernels write every fused multiply-add
# explicitly, so the same expression rounds the same way everywhere
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-ffp-contract=off",
         "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False, extra=(), out: str = LIB, jobs: int | None = None) -> str:
    """Compile every translation unit (in parallel, one hipcc each) and link
    them into ``out``."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    objdir = os.path.join(OBJDIR, "%d" % os.getpid())
    os.makedirs(objdir, exist_ok=True)
    try:
        return _build(objdir, verbose, extra, out, jobs)
    finally:
        # the objects of this build only: removed whether it succeeded or not
        for f in os.listdir(objdir):
            os.remove(os.path.join(objdir, f))
        os.rmdir(objdir)


def _build(objdir: str, verbose: bool, extra, out: str, jobs: int | None) -> str:
    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 1)))
    base = ["hipcc"] + FLAGS + list(extra) + ["-I", INCLUDE, "-I", CSRC]
    cmds = [(src, base + ["-c", os.path.join(CSRC, src), "-o",
                          os.path.join(objdir, src.replace(".hip", ".o"))]) for src in SOURCES]
    pending, running, failed = list(cmds), [], []
    while pending or running:
        while pending and len(running) < jobs:
            src, cmd = pending.pop(0)
            if verbose:
                print(" ".join(cmd), flush=True)
            running.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                  stderr=subprocess.STDOUT, text=True)))
        src, p = running.pop(0)
        text, _ = p.communicate()
        if p.returncode != 0:
            failed.append((src, text))
        elif text.strip() and verbose:
            sys.stderr.write(text)
    if failed:
        for src, text in failed:
            sys.stderr.write(f"--- {src}\n{text}")
        raise RuntimeError("hipcc failed building libtvd.so")
    tmp = out + ".tmp%d" % os.getpid()
    link = (["hipcc"] + FLAGS + ["-shared"] + list(extra) + ["-o", tmp]
            + [os.path.join(objdir, s.replace(".hip", ".o")) for s in SOURCES])
    if verbose:
        print(" ".join(link), flush=True)
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        if os.path.exists(tmp):
            os.remove(tmp)
        raise RuntimeError("hipcc failed linking libtvd.so")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
