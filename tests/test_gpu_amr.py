"""GPU parity of the coarse-fine ghost fill (Sec. 2.2: sibling copy, else
Min-Mod limited linear interpolation from one level coarser) through the C
ABI, against the oracle's two-level ghosted blocks; then one step of the fine
blocks from those ghost zones against the oracle's step.

The fill is the same arithmetic in the same order on both sides (differences,
the limiter's choice, exact quarter offsets, three additions in x, y, z
order), so FP64 and FP32 fills are compared bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import ghosts
from gpu_helpers import FP64, check, GAMMA, norms, note, worst
from paper_0907_3390_amd import layout, tvd, workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    c = tvd.Context(0)
    yield c
    c.close()


def _case(Nc, origin, shape, n, seed):
    coarse_grid = wl.lognormal(Nc, seed=seed, sigma_ln=0.6)
    # fine data: an independent smooth field at twice the resolution
    fine_full = wl.smooth_random(2 * Nc, seed=seed + 1, amplitude=0.3)
    oz, oy, ox = origin
    Lz, Ly, Lx = shape
    box = np.ascontiguousarray(fine_full[:, oz:oz + Lz, oy:oy + Ly, ox:ox + Lx])
    return coarse_grid, box


def _gpu_fill(ctx, coarse_grid, box, origin, n, dtype):
    Nc = coarse_grid.shape[1]
    coarse_bs, fine_bs, cnbr, corigin = layout.two_level(Nc, origin, box.shape[1:], n)
    code = tvd.dtype_code(dtype)
    dev = "cuda"
    c_in = torch.from_numpy(layout.grid_to_blocks(coarse_grid, 8)).to(dtype).to(dev).reshape(-1)
    f_in = torch.from_numpy(layout.grid_to_blocks(box, n)).to(dtype).to(dev).reshape(-1)
    m = n + 6
    f_gh = torch.full((fine_bs.n_blocks * 5 * m ** 3,), -7.0, dtype=dtype, device=dev)
    nbr = torch.from_numpy(fine_bs.nbr).to(dev)
    cn = torch.from_numpy(cnbr).to(dev)
    co = torch.from_numpy(corigin).to(dev)
    fb = tvd.Batch(code, fine_bs.n_blocks, n, dt=1e-3, dh=0.5 / Nc)
    cb = tvd.Batch(code, coarse_bs.n_blocks, 8, dt=1e-3, dh=1.0 / Nc)
    ctx.tvd_read_flags()
    ctx.tvd_fill_ghosts_amr(fb, nbr, f_in, f_gh, cb, c_in, cn, co)
    torch.cuda.synchronize()
    st, fl, bad = ctx.tvd_read_flags()
    assert bad == 0
    return fine_bs, f_gh, (fb, cb, nbr, f_in, c_in, cn, co)


@pytest.mark.parametrize("dtype,n", [(torch.float64, 8), (torch.float64, 16), (torch.float32, 8),
                                     (torch.float32, 16)])
def test_fill_matches_oracle_bitwise(ctx, dtype, n):
    note(f"coarse-fine ghost fill dtype={dtype} n={n}")
    origin, shape = (16, 32, 16), (32, 16, 32)
    coarse_grid, box = _case(32, origin, shape, n, seed=40)
    npd = np.float32 if dtype == torch.float32 else np.float64
    fine_bs, f_gh, _ = _gpu_fill(ctx, coarse_grid.astype(npd), box.astype(npd), origin, n, dtype)
    want = ghosts.two_level_ghosted_blocks(coarse_grid.astype(npd), box.astype(npd), origin, n)
    m = n + 6
    got = f_gh.cpu().numpy().reshape(fine_bs.n_blocks, 5, m, m, m)
    # both sides in the same precision and order: identical bits
    assert np.array_equal(got, want)
    # and some ghost cells really were interpolated (the box has a coarse-fine boundary)
    assert not np.array_equal(got[0][:, 0, 3:-3, 3:-3], box.astype(npd)[:, 0, 0:n, 0:n])


def test_fill_then_step_fp64(ctx):
    """One forward step of the fine blocks of a coarse-fine box from the device
    ghost fill, against the oracle's step on the oracle's ghosted blocks."""
    note("coarse-fine ghost fill, then one step, fp64")
    n, origin, shape = 8, (8, 8, 16), (32, 24, 16)
    coarse_grid, box = _case(32, origin, shape, n, seed=41)
    fine_bs, f_gh, _ = _gpu_fill(ctx, coarse_grid, box, origin, n, torch.float64)
    want_gh = ghosts.two_level_ghosted_blocks(coarse_grid, box, origin, n)
    dh = 0.5 / 32
    dt = 0.5 * dh / oracle.max_signal_speed(box, GAMMA)
    want = np.stack(oracle.advance_ragged(list(want_gh), 0, dt, dh, GAMMA))
    out = torch.zeros(fine_bs.n_blocks * 5 * n ** 3, dtype=torch.float64, device="cuda")
    ctx.tvd_patch_advance(tvd.Batch(tvd.TVD_F64, fine_bs.n_blocks, n, dt=dt, dh=dh), f_gh, out, 0,
                          GAMMA, flags=tvd.TVD_KERNEL_BATCHED)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(fine_bs.n_blocks, 5, n, n, n)
    nrm = norms(got.transpose(1, 0, 2, 3, 4).reshape(5, -1), want.transpose(1, 0, 2, 3, 4).reshape(5, -1))
    note(str({k: f"{v['relL1']:.2e}" for k, v in nrm.items()}))
    check(nrm, FP64)


def test_fill_flags_a_missing_coarse_patch(ctx):
    """A coarse-neighbour entry that names no coarse patch leaves the cells
    that need it untouched and counts them; everything else is filled."""
    note("coarse-fine ghost fill with a missing coarse patch")
    n, origin, shape = 8, (16, 16, 16), (16, 16, 16)
    coarse_grid, box = _case(32, origin, shape, n, seed=42)
    fine_bs, f_gh, (fb, cb, nbr, f_in, c_in, cn, co) = _gpu_fill(ctx, coarse_grid, box, origin, n,
                                                                torch.float64)
    good = f_gh.clone()
    cn[0, 4] = -1                     # the coarse patch below block 0's parent in z (r = 4)
    f_gh.fill_(-7.0)
    ctx.tvd_read_flags()
    ctx.tvd_fill_ghosts_amr(fb, nbr, f_in, f_gh, cb, c_in, cn, co)
    torch.cuda.synchronize()
    st, fl, bad = ctx.tvd_read_flags()
    assert st == tvd.TVD_ERR_NONPHYSICAL and bad > 0
    changed = (f_gh != good).cpu().numpy()
    assert changed.sum() == 5 * bad and np.all(f_gh.cpu().numpy()[changed] == -7.0)
