"""GPU parity of the coarse-fine fill into stand-in blocks (tvd_fill_coarse_fine).

A ghost cell whose sibling is missing is interpolated from the level one
coarser (Sec. 2.2).  With stand-ins, those cells are written into source-only
blocks that the gathering advance reads as if they were siblings.  For every
real block and every ghost region whose neighbour entry names a stand-in, the
stand-in's cells must equal, bit for bit, the ghost cells that the
ghosted-copy fill (tvd_fill_ghosts_amr, itself bitwise equal to the oracle's
interpolation in test_gpu_amr.py) writes for the coarse level
old + w (new - old) (tvd_lerp, the same expression).  Cells of a stand-in
that no ghost region covers are left untouched.  Patches (8^3 fine under 8^3
coarse) and 2^3 patch groups (16^3 under 16^3), FP32 and FP64, w = 0 and 1/2.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import note
from paper_0907_3390_amd import layout, tvd

pytestmark = pytest.mark.gpu
NC = 32
KG = 3


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    c = tvd.Context(0)
    yield c
    c.close()


def _refined():
    r0 = np.zeros((4, 4, 4), dtype=bool)
    r0[1:3, 1:3, 1:3] = True
    r0[0, 3, 1] = True  # a refined patch whose region wraps around the box
    return [r0]


def _slab(r, n):
    """Per axis (x, y, z) the ghosted range [lo, hi) of ghost region r."""
    ra = (r % 3 - 1, (r // 3) % 3 - 1, r // 9 - 1)
    lo = [0 if a < 0 else (KG if a == 0 else n + KG) for a in ra]
    hi = [KG if a < 0 else (n + KG if a == 0 else n + 2 * KG) for a in ra]
    return ra, lo, hi


@pytest.mark.parametrize("n,dtype", [(8, torch.float32), (8, torch.float64),
                                     (16, torch.float32), (16, torch.float64)])
@pytest.mark.parametrize("w", [0.0, 0.5])
def test_standin_fill_equals_ghosted_fill(ctx, n, dtype, w):
    L = layout.NestedLevels(NC, _refined(), n)
    code = tvd.dtype_code(dtype)
    nb, nc = L.blocks[1].n_blocks, L.blocks[0].n_blocks
    vnbr, nsrc = L.stand_ins(1)
    note(f"stand-in fill n {n} {dtype} w {w}: {nb} fine blocks, {nsrc - nb} stand-ins, "
         f"{int((vnbr >= nb).sum())} stand-in regions")
    assert nsrc > nb
    rng = np.random.default_rng(5 + n)
    cells = n ** 3

    def state(k):
        a = rng.uniform(0.5, 2.0, size=(k, 5, n, n, n))
        a[:, 1:4] -= 1.25  # momenta of both signs, so that the limiter takes every branch
        return torch.from_numpy(a).to(dtype).cuda()

    c_old, c_new, f_int = state(nc), state(nc), state(nb)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    cnbr, corig = dev(L.cnbr[1]), dev(L.corigin[1])
    fb = tvd.Batch(code, nb, n, dt=0.0, dh=0.5 / NC)
    cb = tvd.Batch(code, nc, n, dt=0.0, dh=1.0 / NC)
    buf = torch.full((nsrc, 5, n, n, n), float("nan"), dtype=dtype, device="cuda")
    buf[:nb] = f_int
    ctx.tvd_fill_coarse_fine(fb, dev(vnbr), nsrc, buf, cb, c_old, c_new if w else None, w,
                             cnbr, corig)
    c_mid = torch.empty_like(c_old)
    ctx.tvd_lerp(code, nc * 5 * cells, c_old, c_new, c_mid, w)
    gh = torch.zeros((nb, 5, n + 2 * KG, n + 2 * KG, n + 2 * KG), dtype=dtype, device="cuda")
    ctx.tvd_fill_ghosts_amr(fb, dev(L.blocks[1].nbr), f_int, gh, cb, c_mid, cnbr, corig)
    torch.cuda.synchronize()
    got, want = buf.cpu().numpy(), gh.cpu().numpy()
    assert np.array_equal(got[:nb], f_int.cpu().numpy()), "real blocks were written"
    covered = np.zeros((nsrc, n, n, n), dtype=bool)
    for b in range(nb):
        for r in np.nonzero(vnbr[b] >= nb)[0]:
            s = int(vnbr[b, r])
            ra, lo, hi = _slab(int(r), n)
            sl_g = (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
            sl_s = tuple(slice(lo[a] - KG - ra[a] * n, hi[a] - KG - ra[a] * n) for a in (2, 1, 0))
            assert np.array_equal(got[s][(slice(None),) + sl_s], want[b][(slice(None),) + sl_g]), \
                (b, int(r), s)
            covered[s][sl_s] = True
    assert covered[nb:].any()
    standins = got[nb:].transpose(1, 0, 2, 3, 4)  # (5, stand-ins, n, n, n)
    assert np.isnan(standins[:, ~covered[nb:]]).all(), "cells outside every slab were written"
    st, fl, bad = ctx.tvd_read_flags()
    assert bad == 0


def test_standin_fill_argument_errors(ctx):
    L = layout.NestedLevels(NC, _refined(), 8)
    nb, nc = L.blocks[1].n_blocks, L.blocks[0].n_blocks
    vnbr, nsrc = L.stand_ins(1)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    f = torch.zeros(nsrc * 5 * 512, dtype=torch.float32, device="cuda")
    c = torch.zeros(nc * 5 * 512, dtype=torch.float32, device="cuda")
    args = (dev(vnbr), nsrc, f)
    cnbr, corig = dev(L.cnbr[1]), dev(L.corigin[1])
    fb = tvd.Batch(tvd.TVD_F32, nb, 8, dh=0.5 / NC)
    cb = tvd.Batch(tvd.TVD_F32, nc, 8, dh=1.0 / NC)
    call = lambda fb_, cb_, nbr, ns, fi, co, cn, w: ctx.tvd_fill_coarse_fine(
        fb_, nbr, ns, fi, cb_, co, cn, w, cnbr, corig, check=False)
    assert call(fb, cb, *args, c, None, 0.0) == tvd.TVD_OK
    assert call(fb, cb, args[0], nb - 1, f, c, None, 0.0) == tvd.TVD_ERR_INVALID_ARG
    assert call(fb, cb, *args, c, c, 1.5) == tvd.TVD_ERR_INVALID_ARG
    assert call(fb, cb, *args, c, None, 0.5) == tvd.TVD_ERR_INVALID_ARG  # new state missing
    assert call(fb, cb, *args, f, None, 0.0) == tvd.TVD_ERR_ALIAS
    c64 = tvd.Batch(tvd.TVD_F64, nc, 8, dh=1.0 / NC)
    assert call(fb, c64, *args, c, None, 0.0) == tvd.TVD_ERR_INVALID_ARG
    big = tvd.Batch(tvd.TVD_F32, 1290556, 8, dh=0.5 / NC)
    assert call(big, cb, args[0], 1290557, f, c, None, 0.0) == tvd.TVD_ERR_UNSUPPORTED
    st, fl, bad = ctx.tvd_read_flags()
    assert bad == 0
