"""GPU parity of the host-resident advance (tvd_patch_advance_host).

A level whose blocks live in host memory passes through the GPU in launches
of N_s x N_g blocks on N_s streams (Sec. 3.1), with the host's preparation
and closing steps overlapped with the GPU's work or not (Sec. 3.5).  The
host's steps only copy data and the advance is the batched kernel, so the
results must equal, bit for bit, the device path (sibling ghost fill on the
device, then tvd_patch_advance) for every stream count, launch size
(including ragged last launches and streams left idle) and both modes; FP64
is also held to the oracle at 1e-12 (relative L1 and Linf).
"""
import numpy as np
import pytest
import torch

from gpu_helpers import GAMMA, norms, note, worst
from paper_0907_3390_amd import layout, tvd, workloads as wl

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    c = tvd.Context(0)
    yield c
    c.close()


def make_pipe(dtype_code, edge, ns, ng, threads, concurrent):
    streams = [torch.cuda.Stream() for _ in range(ns)]
    pipe = tvd.HostPipeline(streams, ng, threads, concurrent)
    hb, db = pipe.stage_bytes(dtype_code, edge)
    h = torch.empty(hb, dtype=torch.uint8, pin_memory=True)
    d = torch.empty(db, dtype=torch.uint8, device="cuda")
    pipe.attach(h, d)
    return pipe


def level(N, n, seed, dtype):
    bs = layout.periodic_grid_blockset(N, n, curve="morton")
    g = wl.lognormal(N, seed=seed, sigma_ln=0.6)
    if dtype == torch.float32:
        g = g.astype(np.float32).astype(np.float64)
    npdt = np.float32 if dtype == torch.float32 else np.float64
    u = bs.pack_interior(layout.grid_to_blocks(g, n, bs.perm)).astype(npdt)
    return bs, g, u


def device_step(ctx, bs, u, n, dtype, order, dt, dh):
    """Sibling ghost fill and the batched advance on the device."""
    code = tvd.dtype_code(dtype)
    batch = tvd.Batch(code, bs.n_blocks, n, dt=dt, dh=dh)
    d_int = torch.from_numpy(u).cuda()
    d_gh = torch.zeros(bs.in_total, dtype=dtype, device="cuda")
    d_out = torch.zeros(bs.out_total, dtype=dtype, device="cuda")
    ctx.tvd_fill_ghosts(batch, torch.from_numpy(bs.nbr).cuda(), d_int, d_gh)
    ctx.tvd_patch_advance(batch, d_gh, d_out, order, GAMMA, 0.0, tvd.TVD_KERNEL_BATCHED)
    torch.cuda.synchronize()
    return d_out.cpu().numpy()


def host_step(ctx, bs, u, n, dtype, order, dt, dh, ns, ng, concurrent, threads=4):
    code = tvd.dtype_code(dtype)
    batch = tvd.Batch(code, bs.n_blocks, n, dt=dt, dh=dh)
    pipe = make_pipe(code, n, ns, ng, threads, concurrent)
    out = np.full_like(u, np.nan)
    _, times = ctx.tvd_patch_advance_host(batch, bs.nbr, u, out, pipe, order, GAMMA, 0.0,
                                          times=True)
    return out, times


@pytest.mark.parametrize("ns,ng,concurrent", [(1, 64, False), (1, 7, True), (2, 5, True),
                                              (4, 3, False), (4, 3, True), (3, 40, True)])
def test_host_pipeline_equals_device_path_fp32(ctx, ns, ng, concurrent):
    """FP32, 64^3 as 64 blocks of 16^3 (and 512 of 8^3), both sweep orders:
    bit-identical to the device path.  The launch sizes leave ragged last
    launches (64 = 3 x 20 + 4 for N_s = 4, N_g = 5) and idle streams
    (N_s = 3, N_g = 40)."""
    for n in (16, 8):
        bs, g, u = level(64, n, 41, torch.float32)
        for order in (tvd.TVD_XYZ, tvd.TVD_ZYX):
            note(f"host pipeline fp32 edge {n} ns {ns} ng {ng} concurrent {concurrent} "
                 f"order {order}")
            want = device_step(ctx, bs, u, n, torch.float32, order, 0.3 / 64, 1.0 / 64)
            got, times = host_step(ctx, bs, u, n, torch.float32, order, 0.3 / 64, 1.0 / 64,
                                   ns, ng, concurrent)
            assert np.array_equal(got, want)
            assert times["wall"] > 0 and min(times.values()) >= 0
            assert times["advance"] > 0 and times["copy_down"] > 0 and times["copy_up"] > 0
    st, fl, bad = ctx.tvd_read_flags()
    assert bad == 0


def test_host_pipeline_fp64_against_oracle(ctx):
    """FP64 edge 8 on a 32^3 grid: bit-identical to the device path and
    within 1e-12 (relative L1 and Linf per variable) of the oracle's step."""
    note("host pipeline fp64 vs oracle")
    N, n = 32, 8
    bs, g, u = level(N, n, 42, torch.float64)
    dt, dh = 0.3 / N, 1.0 / N
    got, _ = host_step(ctx, bs, u, n, torch.float64, tvd.TVD_XYZ, dt, dh, 4, 5, True)
    want_dev = device_step(ctx, bs, u, n, torch.float64, tvd.TVD_XYZ, dt, dh)
    assert np.array_equal(got, want_dev)
    ref = oracle.step_periodic(g, n, tvd.TVD_XYZ, dt, dh, GAMMA)
    out = layout.blocks_to_grid(np.stack(bs.unpack_interior(got)), g.shape, bs.perm)
    nrm = norms(out, ref)
    note(str({k: (f"{v['relL1']:.1e}", f"{v['relLinf']:.1e}") for k, v in nrm.items()}))
    assert worst(nrm) <= 1e-12
    assert worst(nrm, "relLinf") <= 1e-12


def test_host_pipeline_argument_errors(ctx):
    """Host-side checks, before anything is launched."""
    bs, g, u = level(32, 16, 43, torch.float32)
    batch = tvd.Batch(tvd.TVD_F32, bs.n_blocks, 16, dt=1e-3, dh=1.0 / 32)
    pipe = make_pipe(tvd.TVD_F32, 16, 2, 2, 2, True)
    out = np.zeros_like(u)
    bad = bs.nbr.copy()
    bad[3, 5] = bs.n_blocks
    st, _ = ctx.tvd_patch_advance_host(batch, bad, u, out, pipe, 0, GAMMA, check=False)
    assert st == tvd.TVD_ERR_INVALID_ARG and "h_nbr" in ctx.last_error()
    st, _ = ctx.tvd_patch_advance_host(batch, bs.nbr, u, u, pipe, 0, GAMMA, check=False)
    assert st == tvd.TVD_ERR_ALIAS
    b64 = tvd.Batch(tvd.TVD_F64, bs.n_blocks, 16, dt=1e-3, dh=1.0 / 32)
    st, _ = ctx.tvd_patch_advance_host(b64, bs.nbr, u, out, pipe, 0, GAMMA, check=False)
    assert st == tvd.TVD_ERR_UNSUPPORTED
    dtd = torch.zeros(bs.n_blocks, dtype=torch.float64, device="cuda")
    bdev = tvd.Batch(tvd.TVD_F32, bs.n_blocks, 16, d_dt=dtd, dh=1.0 / 32)
    st, _ = ctx.tvd_patch_advance_host(bdev, bs.nbr, u, out, pipe, 0, GAMMA, check=False)
    assert st == tvd.TVD_ERR_UNSUPPORTED
    zero = tvd.HostPipeline([torch.cuda.Stream()], 0, 1, False)
    st, _ = ctx.tvd_patch_advance_host(batch, bs.nbr, u, out, zero, 0, GAMMA, check=False)
    assert st == tvd.TVD_ERR_INVALID_ARG
    assert not np.any(out)
