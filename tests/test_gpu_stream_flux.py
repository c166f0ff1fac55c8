"""GPU parity of the streamed advance with flux records
(tvd_patch_advance_stream_flux).

The streamed schedule does the per-block advance's arithmetic cell by cell,
and the flux through every interface is the same value in both (Sec. 3.1,
step 8: the closing step's fluxes across patch boundaries), so the state and
every record entry must equal, bit for bit, those of the per-block gathering
advance with records (tvd_patch_advance_flux_gather), which the closing
tests hold to the oracle's records: on a periodic grid (chains of whole
columns, and cut into shorter chains), in both sweep orders, writing and
adding with a weight; and on a refined level whose missing siblings are
stand-ins (chains ending at them), after the coarse-fine fill.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import GAMMA, note
from paper_0907_3390_amd import layout, tvd, workloads as wl

pytestmark = pytest.mark.gpu
REC = layout.flux_record_size(16)


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    c = tvd.Context(0)
    yield c
    c.close()


def chains(nbr, order, chain_len, members=None):
    st, bl = layout.stream_chains(nbr, 2 if order == tvd.TVD_XYZ else 0, chain_len, members)
    return tvd.Chains(torch.from_numpy(st).cuda(), torch.from_numpy(bl).cuda())


def both(ctx, batch, nbr, nsrc, u, order, chain_len, rec0, w, acc, members=None):
    nb = batch.c.n_blocks
    n3 = 5 * 16 ** 3
    dnbr = torch.from_numpy(np.ascontiguousarray(nbr)).cuda()
    out_a = torch.full((nb * n3,), float("nan"), dtype=torch.float32, device="cuda")
    out_b = out_a.clone()
    rec_a = rec0.clone()
    rec_b = rec0.clone()
    ctx.tvd_patch_advance_flux_gather(batch, dnbr, nsrc, u, out_a, rec_a, None, order, GAMMA,
                                      flux_weight=w, accumulate=acc)
    ch = chains(nbr[:nb], order, chain_len, members)
    ctx.tvd_patch_advance_stream_flux(batch, dnbr, nsrc, ch, u, out_b, rec_b, None, order, GAMMA,
                                      flux_weight=w, accumulate=acc)
    torch.cuda.synchronize()
    return out_a.cpu().numpy(), out_b.cpu().numpy(), rec_a.cpu().numpy(), rec_b.cpu().numpy()


@pytest.mark.parametrize("order", [tvd.TVD_XYZ, tvd.TVD_ZYX])
@pytest.mark.parametrize("chain_len,w,acc", [(4, 1.0, 0), (3, 0.5, 1), (1, 1.0, 0)])
def test_stream_flux_equals_per_block_periodic(ctx, order, chain_len, w, acc):
    """64^3 rough lognormal state as 64 Morton-numbered 16^3 groups (columns
    of 4 blocks: whole cycles, cut 3 + 1, or single blocks), records starting
    from random values: state and records bit-identical."""
    N = 64
    note(f"stream flux periodic order {order} chain {chain_len} w {w} acc {acc}")
    bs = layout.periodic_grid_blockset(N, 16, curve="morton")
    g = wl.lognormal(N, seed=71, sigma_ln=0.8).astype(np.float32)
    u = torch.from_numpy(bs.pack_interior(layout.grid_to_blocks(g, 16, bs.perm))).cuda()
    batch = tvd.Batch(tvd.TVD_F32, bs.n_blocks, 16, dt=0.2 / N, dh=1.0 / N)
    rec0 = torch.from_numpy(wl.rng(72).standard_normal(bs.n_blocks * REC).astype(np.float32)).cuda()
    oa, ob, ra, rb = both(ctx, batch, bs.nbr, bs.n_blocks, u, order, chain_len, rec0, w, acc)
    assert not np.isnan(oa).any()
    assert np.array_equal(oa, ob)
    assert np.array_equal(ra, rb)
    assert not np.array_equal(ra, rec0.cpu().numpy())
    st, fl, bad = ctx.tvd_read_flags()
    assert bad == 0


def _refined():
    r0 = np.zeros((4, 4, 4), dtype=bool)
    r0[1:3, 1:3, 1:3] = True
    r0[0, 3, 1] = True
    return [r0]


@pytest.mark.parametrize("order", [tvd.TVD_XYZ, tvd.TVD_ZYX])
def test_stream_flux_with_standins(ctx, order):
    """A refined level of 16^3 groups (two levels, 32^3 base): stand-ins
    filled from the coarse level (tvd_fill_coarse_fine), chains over the
    real blocks that end where a stand-in follows; state and records
    bit-identical to the per-block gathering advance."""
    note(f"stream flux with stand-ins order {order}")
    L = layout.NestedLevels(32, _refined(), 16)
    nb, nc = L.blocks[1].n_blocks, L.blocks[0].n_blocks
    vnbr, nsrc = L.stand_ins(1)
    rng = wl.rng(73)
    c = rng.uniform(0.5, 2.0, size=(nc, 5, 16, 16, 16))
    c[:, 1:4] -= 1.25
    c[:, 4] += 3.0
    f = rng.uniform(0.5, 2.0, size=(nb, 5, 16, 16, 16))
    f[:, 1:4] -= 1.25
    f[:, 4] += 3.0
    cdev = torch.from_numpy(c.astype(np.float32)).cuda()
    buf = torch.zeros((nsrc, 5, 16, 16, 16), dtype=torch.float32, device="cuda")
    buf[:nb] = torch.from_numpy(f.astype(np.float32)).cuda()
    fb = tvd.Batch(tvd.TVD_F32, nb, 16, dt=0.1 / 64, dh=1.0 / 64)
    cb = tvd.Batch(tvd.TVD_F32, nc, 16, dt=0.1 / 64, dh=1.0 / 32)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    ctx.tvd_fill_coarse_fine(fb, dev(vnbr), nsrc, buf, cb, cdev, None, 0.0, dev(L.cnbr[1]),
                             dev(L.corigin[1]))
    rec0 = torch.zeros(nb * REC, dtype=torch.float32, device="cuda")
    oa, ob, ra, rb = both(ctx, fb, vnbr, nsrc, buf, order, 8, rec0, 1.0, 0)
    assert not np.isnan(oa).any()
    assert np.array_equal(oa, ob)
    assert np.array_equal(ra, rb)
    st, fl, bad = ctx.tvd_read_flags()
    assert bad == 0


def test_stream_flux_argument_errors(ctx):
    bs = layout.periodic_grid_blockset(32, 16)
    u = torch.zeros((bs.n_blocks, 5, 4096), dtype=torch.float32, device="cuda")
    u[:, 0] = 1.0   # gas at rest, rho 1, e 1.5
    u[:, 4] = 1.5
    u = u.reshape(-1)
    out = torch.zeros_like(u)
    rec = torch.zeros(bs.n_blocks * REC, dtype=torch.float32, device="cuda")
    nbr = torch.from_numpy(bs.nbr).cuda()
    ch = chains(bs.nbr, 0, 2)
    b = tvd.Batch(tvd.TVD_F32, bs.n_blocks, 16, dt=1e-3, dh=1.0 / 32)
    call = lambda *a, **k: ctx.tvd_patch_advance_stream_flux(*a, check=False, **k)
    assert call(b, nbr, bs.n_blocks, ch, u, out, rec, None, 0, GAMMA) == tvd.TVD_OK
    assert call(b, nbr, bs.n_blocks - 1, ch, u, out, rec, None, 0, GAMMA) == tvd.TVD_ERR_INVALID_ARG
    assert call(b, nbr, bs.n_blocks, ch, u, out, None, None, 0, GAMMA) == tvd.TVD_ERR_INVALID_ARG
    assert call(b, nbr, bs.n_blocks, ch, u, out, rec, None, 0, GAMMA,
                accumulate=2) == tvd.TVD_ERR_INVALID_ARG
    assert call(b, nbr, bs.n_blocks, ch, u, out, u, None, 0, GAMMA) == tvd.TVD_ERR_ALIAS
    assert call(b, nbr, bs.n_blocks, ch, u, u, rec, None, 0, GAMMA) == tvd.TVD_ERR_ALIAS
    b64 = tvd.Batch(tvd.TVD_F64, bs.n_blocks, 16, dt=1e-3, dh=1.0 / 32)
    assert call(b64, nbr, bs.n_blocks, ch, u, out, rec, None, 0, GAMMA) == tvd.TVD_ERR_UNSUPPORTED
    b8 = tvd.Batch(tvd.TVD_F32, 64, 8, dt=1e-3, dh=1.0 / 32)
    assert call(b8, nbr, 64, ch, u, out, rec, None, 0, GAMMA) == tvd.TVD_ERR_UNSUPPORTED
    torch.cuda.synchronize()
    st, fl, bad = ctx.tvd_read_flags()
    assert bad == 0
