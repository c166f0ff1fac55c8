"""Resource usage of the streamed advance's kernels, read from the gfx950
code object metadata of a device-only compile (no GPU needed).

The streamed advance is bound by the issue rate of its vector instructions,
so two silent compiler decisions cost it a lot: spilling registers to
scratch memory (the FP64 kernels with the half-pencil second sweep, and the
FP32 kernels with flux records in half pencils, spilled hundreds of
registers per lane), and moving a register array of a thread into LDS (the
AMDGPU alloca promotion, which once took the backward order's output runs
into a 32-byte-per-thread LDS array with 8-way bank conflicts).  Every
instantiation the library launches by default must have no spills and
exactly the slab's LDS (no promoted arrays).
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_0907_3390_amd import build

# shared memory of one workgroup: 5 variables x 8 planes x 368 words of the
# slab, 64 chain offsets, 9 neighbour offsets, the 4 x 10 reduction values
# and a counter (StreamLds<T, 8>), rounded up to 16 bytes
SLAB_LDS = {"f": 5 * 8 * 368 * 4 + 64 * 8 + 9 * 8 + 4 * 10 * 8 + 8,
            "d": 5 * 8 * 368 * 8 + 64 * 8 + 9 * 8 + 4 * 10 * 8 + 8}


def kernels(tu):
    """name -> (vgpr spills, private segment bytes, LDS bytes) of every
    kernel in a device-only compile of csrc/<tu>."""
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    out = os.path.join(build.OBJDIR, f"resources_{os.getpid()}_{tu}.s")
    os.makedirs(build.OBJDIR, exist_ok=True)
    try:
        subprocess.run(["hipcc"] + build.FLAGS + ["--cuda-device-only", "-S", "-o", out,
                                                  "-I", build.INCLUDE, "-I", build.CSRC,
                                                  os.path.join(build.CSRC, tu)],
                       check=True, capture_output=True)
        text = open(out).read()
    finally:
        if os.path.exists(out):
            os.remove(out)
    res = {}
    # the metadata block lists, per kernel, its fields in alphabetical order
    for block in text.split("  - .agpr_count:")[1:]:
        name = re.search(r"\.name:\s+(\S+)", block).group(1)
        spill = int(re.search(r"\.vgpr_spill_count:\s+(\d+)", block).group(1))
        priv = int(re.search(r"\.private_segment_fixed_size:\s+(\d+)", block).group(1))
        lds = int(re.search(r"\.group_segment_fixed_size:\s+(\d+)", block).group(1))
        res[name] = (spill, priv, lds)
    return res


def stream_args(name):
    """(T, E, ORDER, P, SPLITB, FLUX) of a mangled k_stream instantiation."""
    m = re.match(r"_ZN3tvd8k_streamI([fd])Li(\d+)ELi(\d)ELi(\d+)ELb(\d)ELi(\d)EE", name)
    return None if m is None else (m.group(1), int(m.group(2)), int(m.group(3)), int(m.group(4)),
                                   bool(int(m.group(5))), int(m.group(6)))


@pytest.mark.parametrize("tu", ["tvd_k_stream_f32.hip", "tvd_k_stream_f64.hip"])
def test_streamed_kernels_do_not_spill_or_promote(tu):
    ks = {n: v for n, v in kernels(tu).items() if stream_args(n)}
    assert ks, "no k_stream instantiation found"
    checked = 0
    for name, (spill, priv, lds) in ks.items():
        t, e, order, p, splitb, flux = stream_args(name)
        # the layouts launched by default: FP32 without records in half
        # pencils (and whole, a tuner candidate), FP32 with records and FP64
        # in whole pencils; FP64 in half pencils is kept only on request
        if t == "d" and splitb:
            continue
        assert lds == SLAB_LDS[t], (name, lds)
        assert spill == 0 and priv == 0, (name, spill, priv)
        checked += 1
    assert checked >= 4
