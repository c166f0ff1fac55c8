"""GPU parity of the streamed advance (tvd_patch_advance_stream).

The streamed advance carries the third sweep of every step along a chain of
blocks and runs the first two on slabs of planes; the arithmetic of every
cell is the per-block advance's, and the region rule is exact, so its
results are compared bit for bit with the gathering per-block advance (and
across block edges, chain lengths and launch variants), and with the FP64
oracle to the stated tolerances: FP64 relative L1 and relative Linf (against
each variable's largest magnitude) <= 1e-12; FP32 relative L1 <= 1e-5 and
relative Linf <= 1e-4 on smooth data.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import GAMMA, norms, note, oracle_boxes, oracle_periodic, worst
from paper_0907_3390_amd import layout, tvd, workloads as wl
from paper_0907_3390_amd.driver import DeviceBlocks

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    c = tvd.Context(0)
    yield c
    c.close()


def run(ctx, grid, steps, n, dtype, stream, chain_len=None, kernel=tvd.TVD_KERNEL_AUTO,
        sums=False, curve="morton", p_floor=0.0, gamma=GAMMA):
    N = grid.shape[3]
    bs = layout.periodic_grid_blockset(N, n, curve=curve)
    dev = DeviceBlocks(ctx, bs, dtype=dtype, gather=True, stream=stream, chain_len=chain_len,
                       kernel=kernel, p_floor=p_floor, gamma=gamma)
    dev.upload(layout.grid_to_blocks(grid, n, bs.perm))
    rec = dev.run(steps, sums_each_step=sums)
    torch.cuda.synchronize()
    out = layout.blocks_to_grid(np.stack(dev.download()), grid.shape, bs.perm)
    return out, (rec.cpu().numpy() if rec is not None else None), dev


@pytest.mark.parametrize("n", [16, 32])
def test_stream_equals_per_block_fp32(ctx, n):
    """FP32: the streamed advance (edge 16 or 32) over 4 steps equals the
    gathering per-block advance on 16^3 blocks bit for bit, fused speed and
    dt included."""
    note(f"stream vs per-block fp32, edge {n}")
    g = wl.lognormal(64, seed=21, sigma_ln=0.7).astype(np.float32).astype(np.float64)
    ref, _, dref = run(ctx, g, 4, 16, torch.float32, stream=False)
    got, _, dgot = run(ctx, g, 4, n, torch.float32, stream=True)
    assert np.array_equal(got, ref)
    assert torch.equal(dgot.dt[:1], dref.dt[:1])
    st, fl, bad = ctx.tvd_read_flags()
    assert bad == 0


@pytest.mark.parametrize("n", [16, 32])
def test_stream_fp64_against_oracle_and_edge8(ctx, n):
    """FP64 at edges 16 and 32 (the per-block kernel holds FP64 blocks of
    edge 8 only): equal bit for bit to the per-block advance on 8^3 blocks,
    and within 1e-12 of the oracle (relative L1 and Linf) after 6 steps."""
    note(f"stream fp64 edge {n}")
    g = wl.smooth_random(64, seed=22, amplitude=0.3)
    ref8, _, _ = run(ctx, g, 6, 8, torch.float64, stream=False)
    got, _, _ = run(ctx, g, 6, n, torch.float64, stream=True)
    assert np.array_equal(got, ref8)
    want, _ = oracle_periodic(g, 6)
    nrm = norms(got, want)
    note(str({k: (f"{v['relL1']:.1e}", f"{v['relLinf']:.1e}") for k, v in nrm.items()}))
    assert worst(nrm) <= 1e-12
    assert worst(nrm, "relLinf") <= 1e-12


def test_stream_fp32_against_oracle_smooth(ctx):
    """FP32 on smooth data, 10 steps, edge 32: relative L1 <= 1e-5 and
    relative Linf <= 1e-4 per variable against the FP64 oracle run from the
    same FP32-rounded state."""
    note("stream fp32 vs oracle, smooth, edge 32")
    g = wl.smooth_random(64, seed=23, amplitude=0.2).astype(np.float32).astype(np.float64)
    got, _, _ = run(ctx, g, 10, 32, torch.float32, stream=True)
    want, _ = oracle_periodic(g, 10)
    nrm = norms(got, want)
    note(str({k: (f"{v['relL1']:.1e}", f"{v['relLinf']:.1e}") for k, v in nrm.items()}))
    assert worst(nrm) <= 1e-5
    assert worst(nrm, "relLinf") <= 1e-4


@pytest.mark.parametrize("chain_len", [1, 2, 3, 8])
def test_chain_length_is_invisible(ctx, chain_len):
    """Chains of 1, 2, 3 and 8 blocks (a whole periodic line) give the same
    bits: the chain's ends only repeat the first two sweeps on ghost planes."""
    note(f"chain length {chain_len}")
    g = wl.lognormal(128, seed=24, sigma_ln=0.5).astype(np.float32).astype(np.float64)
    ref, _, _ = run(ctx, g, 2, 16, torch.float32, stream=True, chain_len=4)
    got, _, _ = run(ctx, g, 2, 16, torch.float32, stream=True, chain_len=chain_len)
    assert np.array_equal(got, ref)


def test_whole_pencil_variant_and_fused_sums(ctx):
    """The whole-pencil second sweep gives the same bits as the half-pencil
    one; the fused FP64 sums of every step equal the per-block advance's
    (the same cells, reduced in another fixed order) to 1e-15 relative."""
    note("stream whole-pencil variant, fused sums")
    g = wl.lognormal(64, seed=25, sigma_ln=0.7).astype(np.float32).astype(np.float64)
    a, sa, _ = run(ctx, g, 4, 16, torch.float32, stream=True, sums=True)
    b, sb, _ = run(ctx, g, 4, 16, torch.float32, stream=True, sums=True,
                   kernel=tvd.TVD_STREAM_WHOLE_B)
    c, sc, _ = run(ctx, g, 4, 16, torch.float32, stream=False, sums=True)
    assert np.array_equal(a, b) and np.array_equal(a, c)
    assert np.array_equal(sa, sb)
    scale = np.abs(sc).max(axis=0) + np.abs(sc[:, 0:1]).max()
    assert np.all(np.abs(sa - sc) <= 1e-15 * scale)


@pytest.mark.parametrize("n", [16, 32])
def test_whole_pencil_variant_fp64(ctx, n):
    """FP64: the whole-pencil second sweep (the default in FP64: no registers
    held across a barrier) gives the bits of the half-pencil one and of the
    per-block advance on 8^3 patches (the region rule is exact), on edge-16
    and edge-32 blocks."""
    note(f"stream whole-pencil variant fp64 edge {n}")
    g = wl.lognormal(64, seed=27, sigma_ln=0.7)
    a, _, _ = run(ctx, g, 4, n, torch.float64, stream=True)  # default: whole in FP64
    h, _, _ = run(ctx, g, 4, n, torch.float64, stream=True, kernel=tvd.TVD_STREAM_HALF_B)
    w, _, _ = run(ctx, g, 4, n, torch.float64, stream=True, kernel=tvd.TVD_STREAM_WHOLE_B)
    c, _, _ = run(ctx, g, 4, 8, torch.float64, stream=False)
    assert not np.isnan(a).any()
    assert np.array_equal(a, h) and np.array_equal(a, w) and np.array_equal(a, c)


def test_stream_graph_replay_matches_eager(ctx):
    """A captured pair of streamed steps replays to the eager steps' bits."""
    note("stream graph replay")
    g = wl.lognormal(64, seed=26, sigma_ln=0.7).astype(np.float32).astype(np.float64)
    eager, _, _ = run(ctx, g, 6, 16, torch.float32, stream=True)
    bs = layout.periodic_grid_blockset(64, 16, curve="morton")
    dev = DeviceBlocks(ctx, bs, dtype=torch.float32, stream=True)
    dev.upload(layout.grid_to_blocks(g, 16, bs.perm))
    dev.run(2)
    s = torch.cuda.Stream()
    gr = dev.capture(2, stream=s, sums=True)
    for _ in range(2):
        dev.replay(gr, stream=s)
        torch.cuda.synchronize()
    gr.close()
    got = layout.blocks_to_grid(np.stack(dev.download()), g.shape, bs.perm)
    assert np.array_equal(got, eager)


def test_uneven_32cube_boxes_as_edge32_blocks(ctx):
    """The 32^3 boxes of the uneven batch (sound waves of amplitude 1e-3,
    each box periodic on itself), every box one edge-32 block whose chains
    are the box itself along the streamed axis: ten steps with dt from the
    device, bit-identical to the same boxes cut into 16^3 groups and advanced
    by the per-block gathering kernel, and against the oracle run over the
    boxes (relative L1 <= 1e-5 and Linf <= 1e-4 per variable)."""
    boxes = wl.sound_wave_boxes(seed=4)
    pick = [i for i, g in enumerate(boxes.grids) if g.shape[1] == 32][:48]
    grids = [boxes.grids[i].astype(np.float32).astype(np.float64) for i in pick]
    dhs = [boxes.dh[i] for i in pick]
    note(f"uneven batch: {len(pick)} boxes of 32^3 as edge-32 streamed blocks")
    outs = {}
    for e, stream in ((32, True), (16, False)):
        bs = layout.boxes_blockset([32] * len(grids), lambda L: e, dhs)
        dev = DeviceBlocks(ctx, bs, dtype=torch.float32, gather=True, stream=stream)
        dev.upload(layout.boxes_to_blocks(grids, lambda L: e))
        ctx.tvd_read_flags()
        dev.run(10)
        torch.cuda.synchronize()
        st, fl, bad = ctx.tvd_read_flags()
        assert st == tvd.TVD_OK and fl == 0 and bad == 0
        outs[e] = layout.blocks_to_boxes(dev.download(), [32] * len(grids), lambda L: e)
        del dev
    for a, b in zip(outs[32], outs[16]):
        assert np.array_equal(a, b)
    want = oracle_boxes(grids, dhs, 10)
    nrm = norms(np.concatenate([x.reshape(5, -1) for x in outs[32]], axis=1),
                np.concatenate([x.reshape(5, -1) for x in want], axis=1))
    note(str({k: (f"{v['relL1']:.1e}", f"{v['relLinf']:.1e}") for k, v in nrm.items()}))
    assert worst(nrm) <= 1e-5
    assert worst(nrm, "relLinf") <= 1e-4


def test_bad_chains_are_flagged_not_advanced(ctx):
    """A chain whose blocks are not consecutive along the streamed axis, or
    that names a block out of range, is not advanced (output untouched) and
    its cells are counted as non-physical; the other chains still run."""
    note("stream bad chains")
    g = wl.lognormal(32, seed=27, sigma_ln=0.5).astype(np.float32).astype(np.float64)
    bs = layout.periodic_grid_blockset(32, 16)
    dev = DeviceBlocks(ctx, bs, dtype=torch.float32, stream=True, chain_len=2)
    dev.upload(layout.grid_to_blocks(g, 16))
    dev.dt.fill_(0.2 / 32)
    st, bl = layout.stream_chains(bs.nbr, 2, 2)
    bl_bad = bl.copy()
    # chain 0: swap its two blocks (no longer consecutive along +z in this order? both
    # orders are consecutive on a periodic line of two, so swap with another chain)
    bl_bad[0], bl_bad[2] = bl[2], bl[0]
    bad = tvd.Chains(torch.from_numpy(st).cuda(), torch.from_numpy(bl_bad).cuda())
    out = torch.full_like(dev.interior, 7.0)
    ctx.tvd_read_flags()
    ctx.tvd_patch_advance_stream(dev.batch, dev.nbr, bad, dev.interior, out, 0, GAMMA)
    torch.cuda.synchronize()
    stt, fl, nonphys = ctx.tvd_read_flags()
    assert nonphys > 0
    o = out.cpu().numpy().reshape(bs.n_blocks, -1)
    touched = [not np.all(o[b] == 7.0) for b in range(bs.n_blocks)]
    good = tvd.Chains(torch.from_numpy(st).cuda(), torch.from_numpy(bl).cuda())
    ref = torch.zeros_like(dev.interior)
    ctx.tvd_patch_advance_stream(dev.batch, dev.nbr, good, dev.interior, ref, 0, GAMMA)
    torch.cuda.synchronize()
    r = ref.cpu().numpy().reshape(bs.n_blocks, -1)
    for c in range(len(st) - 1):
        members = bl_bad[st[c]:st[c + 1]]
        ok = all(bs.nbr[a, layout.PLUS_REGION[2]] == b for a, b in zip(members[:-1], members[1:]))
        for b in members:
            assert touched[b] == ok
            if ok:
                assert np.array_equal(o[b], r[b])
    # a block number out of range in a chain
    bl_oob = bl.copy()
    bl_oob[-1] = bs.n_blocks + 5
    oob = tvd.Chains(torch.from_numpy(st).cuda(), torch.from_numpy(bl_oob).cuda())
    out.fill_(7.0)
    ctx.tvd_patch_advance_stream(dev.batch, dev.nbr, oob, dev.interior, out, 0, GAMMA)
    torch.cuda.synchronize()
    stt, fl, nonphys = ctx.tvd_read_flags()
    assert nonphys > 0


def test_stream_argument_errors(ctx):
    """Host-side checks: edges other than 16/32, mixed edges, bad flags,
    aliasing, misaligned state pointers, a too-small workspace."""
    note("stream argument errors")
    bs = layout.periodic_grid_blockset(32, 16)
    dev = DeviceBlocks(ctx, bs, dtype=torch.float32, stream=True)
    ch = dev.chains[0]
    u, o = dev.interior, dev.spare
    with pytest.raises(tvd.TvdError) as e:
        ctx.tvd_patch_advance_stream(tvd.Batch(tvd.TVD_F32, bs.n_blocks, 8, dt=1e-3, dh=1.0),
                                     dev.nbr, ch, u, o, 0, GAMMA)
    assert e.value.status == tvd.TVD_ERR_UNSUPPORTED
    with pytest.raises(tvd.TvdError) as e:
        ctx.tvd_patch_advance_stream(dev.batch, dev.nbr, ch, u, o, 0, GAMMA, flags=5)
    assert e.value.status == tvd.TVD_ERR_INVALID_ARG
    with pytest.raises(tvd.TvdError) as e:   # both layouts at once
        ctx.tvd_patch_advance_stream(dev.batch, dev.nbr, ch, u, o, 0, GAMMA,
                                     flags=tvd.TVD_STREAM_WHOLE_B | tvd.TVD_STREAM_HALF_B)
    assert e.value.status == tvd.TVD_ERR_INVALID_ARG
    with pytest.raises(tvd.TvdError) as e:
        ctx.tvd_patch_advance_stream(dev.batch, dev.nbr, ch, u, u, 0, GAMMA)
    assert e.value.status == tvd.TVD_ERR_ALIAS
    # rows are read and written 16 bytes at a time: a state pointer off by one
    # element is refused before any launch
    shifted = torch.zeros(bs.out_total + 4, dtype=torch.float32, device="cuda")[1:1 + bs.out_total]
    with pytest.raises(tvd.TvdError) as e:
        ctx.tvd_patch_advance_stream(dev.batch, dev.nbr, ch, shifted, o, 0, GAMMA)
    assert e.value.status == tvd.TVD_ERR_INVALID_ARG and "aligned" in str(e.value)
    # 4096 blocks in 2048 chains: more partials (one per chain) than the
    # 1024 a fresh context reserves
    big = layout.periodic_grid_blockset(256, 16)
    c2 = tvd.Context(0)
    try:
        b2 = tvd.Batch(tvd.TVD_F32, big.n_blocks, 16, dt=1e-4, dh=1.0 / 256)
        st, bl = layout.stream_chains(big.nbr, 2, 2)
        chb = tvd.Chains(torch.from_numpy(st).cuda(), torch.from_numpy(bl).cuda())
        assert len(st) - 1 > 1024
        nb = torch.from_numpy(big.nbr).cuda()
        uu = torch.ones(big.out_total, dtype=torch.float32, device="cuda")
        oo = torch.zeros_like(uu)
        sm = torch.zeros(1, dtype=torch.float64, device="cuda")
        with pytest.raises(tvd.TvdError) as e:
            c2.tvd_patch_advance_stream(b2, nb, chb, uu, oo, 0, GAMMA, smax=sm)
        assert e.value.status == tvd.TVD_ERR_STATE
    finally:
        c2.close()
