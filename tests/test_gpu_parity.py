"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (per variable, norms defined in gpu_helpers.norms):
* FP64 GPU (plain and batched kernels): relative L1 <= 1e-12 against the
  oracle after the stated number of steps (round-off of the same FP64
  arithmetic in a different order; the scheme is Lipschitz, so differences
  stay near 1e-15).
* FP32 GPU on smooth data: relative L1 <= 1e-5 after 10 steps against the
  oracle run from the same FP32-rounded initial state.
* Pure copies (ghost fill) and exact invariants (uniform state) are
  bit-exact; sums of dyadic data are exact.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import (FP32_ROUGH, FP32_SMOOTH, FP64, GAMMA, check, norms, note, oracle_boxes,
                         oracle_periodic, worst)
from paper_0907_3390_amd import layout, tvd, workloads as wl
from paper_0907_3390_amd.driver import DeviceBlocks

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    c = tvd.Context(0)
    yield c
    c.close()


def run_gpu_periodic(ctx, grid, steps, n, dtype, kernel=tvd.TVD_KERNEL_AUTO, fused=True,
                     p_floor=0.0, gamma=GAMMA, curve="linear", gather=False):
    N = grid.shape[3]
    bs = layout.periodic_grid_blockset(N, n, curve=curve)
    dev = DeviceBlocks(ctx, bs, dtype=dtype, gamma=gamma, p_floor=p_floor, kernel=kernel,
                       gather=gather)
    dev.upload(layout.grid_to_blocks(grid, n, bs.perm))
    dev.run(steps, fused=fused)
    torch.cuda.synchronize()
    out = layout.blocks_to_grid(np.stack(dev.download()), grid.shape, bs.perm)
    return out, dev


# ---------------------------------------------------------------------------
# exact invariants
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype,kernel,n", [
    (torch.float32, tvd.TVD_KERNEL_BATCHED, 8), (torch.float32, tvd.TVD_KERNEL_BATCHED, 16),
    (torch.float64, tvd.TVD_KERNEL_BATCHED, 8), (torch.float64, tvd.TVD_KERNEL_PLAIN, 8)])
def test_uniform_state_bitwise(ctx, dtype, kernel, n):
    note(f"uniform state dtype={dtype} kernel={kernel} n={n}")
    g = wl.uniform(32, rho=1.3, v=(0.2, -0.4, 0.1), P=0.8)
    g = g.astype(np.float32).astype(np.float64) if dtype == torch.float32 else g
    out, dev = run_gpu_periodic(ctx, g, 4, n, dtype, kernel)
    assert np.array_equal(out, g)
    st, fl, bad = ctx.tvd_read_flags()
    assert st == tvd.TVD_OK and fl == 0 and bad == 0


def _rotate_state(g, perm):
    arr_axes = [0] + [3 - perm[2 - i] for i in range(3)]
    out = np.transpose(g, arr_axes).copy()
    for a in range(3):
        out[1 + a] = np.transpose(g[1 + perm[a]], [x - 1 for x in arr_axes[1:]])
    return out


@pytest.mark.parametrize("dtype,n", [(torch.float32, 16), (torch.float64, 8)])
def test_mirror_and_transpose_bitwise(ctx, dtype, n):
    """The GPU update commutes bit for bit with reflecting an axis (momentum
    negated) and swapping x with z also swaps the sweep order (explicit FMAs,
    symmetric transverse terms)."""
    note(f"mirror/transpose dtype={dtype} n={n}")
    g = wl.smooth_random(32, seed=15, amplitude=0.3)
    if dtype == torch.float32:
        g = g.astype(np.float32).astype(np.float64)
    base, _ = run_gpu_periodic(ctx, g, 2, n, dtype)
    for axis in range(3):
        gm = np.flip(g, axis=3 - axis).copy()
        gm[1 + axis] *= -1
        outm, _ = run_gpu_periodic(ctx, gm, 2, n, dtype)
        back = np.flip(outm, axis=3 - axis).copy()
        back[1 + axis] *= -1
        assert np.array_equal(back, base), axis
    # one forward step on the transposed state == transpose of one backward step
    bs = layout.periodic_grid_blockset(32, n)
    res = []
    for state, order in [(_rotate_state(g, [2, 1, 0]), 0), (g, 1)]:
        dev = DeviceBlocks(ctx, bs, dtype=dtype)
        dev.upload(layout.grid_to_blocks(state, n))
        dev.dt.fill_(0.3 / 32)
        dev.fill_ghosts()
        dev.advance(order)
        torch.cuda.synchronize()
        res.append(layout.blocks_to_grid(np.stack(dev.download()), g.shape))
    assert np.array_equal(res[0], _rotate_state(res[1], [2, 1, 0]))


def test_edge8_equals_edge16_fp32(ctx):
    """Decomposition invariance on the GPU: the same periodic grid advanced as
    8^3 blocks and as 16^3 blocks gives identical FP32 results."""
    note("edge 8 vs edge 16 fp32")
    g = wl.lognormal(32, seed=16, sigma_ln=0.7).astype(np.float32).astype(np.float64)
    a, _ = run_gpu_periodic(ctx, g, 4, 8, torch.float32)
    b, _ = run_gpu_periodic(ctx, g, 4, 16, torch.float32)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("gather", [False, True])
def test_morton_numbering_is_invisible(ctx, gather):
    """Blocks numbered along the Morton curve instead of x fastest (only the
    neighbour table and the placement change) give identical results."""
    note(f"Morton vs linear block numbering, gather={gather}")
    g = wl.lognormal(64, seed=19, sigma_ln=0.7).astype(np.float32).astype(np.float64)
    a, _ = run_gpu_periodic(ctx, g, 4, 16, torch.float32, gather=gather)
    b, _ = run_gpu_periodic(ctx, g, 4, 16, torch.float32, gather=gather, curve="morton")
    assert np.array_equal(a, b)


@pytest.mark.parametrize("dtype,n", [(torch.float32, 16), (torch.float32, 8), (torch.float64, 8)])
def test_gather_equals_fill_then_advance(ctx, dtype, n):
    """Gathering ghost cells inside the advance gives bit for bit the result
    of filling a ghosted copy first (same arithmetic, same inputs)."""
    note(f"gather vs fill+advance dtype={dtype} n={n}")
    g = wl.lognormal(32, seed=17, sigma_ln=0.8)
    if dtype == torch.float32:
        g = g.astype(np.float32).astype(np.float64)
    bs = layout.periodic_grid_blockset(32, n)
    outs = []
    for gather in (False, True):
        dev = DeviceBlocks(ctx, bs, dtype=dtype, gather=gather)
        dev.upload(layout.grid_to_blocks(g, n))
        rec = dev.run(6, sums_each_step=True)
        torch.cuda.synchronize()
        outs.append((np.stack(dev.download()), dev.dt.cpu().numpy(), rec.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    np.testing.assert_allclose(outs[0][2], outs[1][2], rtol=1e-15)


def test_gather_mixed_edges_fp32(ctx):
    note("gather with mixed edges (boxes)")
    boxes = wl.sound_wave_boxes(counts=(4, 2, 1), seed=6)
    grids = [b.astype(np.float32).astype(np.float64) for b in boxes.grids]
    edges = [g.shape[1] for g in grids]
    efor = lambda L: 8 if L == 8 else 16
    bs = layout.boxes_blockset(edges, efor, boxes.dh)
    outs = []
    for gather in (False, True):
        dev = DeviceBlocks(ctx, bs, dtype=torch.float32, gather=gather)
        dev.upload(layout.boxes_to_blocks(grids, efor))
        dev.run(4)
        torch.cuda.synchronize()
        outs.append(dev.interior.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("gather", [False, True])
def test_persistent_equals_per_edge_launches(ctx, gather):
    """Mixed edges in one persistent launch (workgroups drawing edge-16 blocks
    and quads of edge-8 blocks from per-XCD queues, more blocks than
    workgroups, a ragged last quad) give bit for bit the result of one launch
    per edge, fused signal speed, dt and sums included."""
    note(f"persistent vs per-edge launches gather={gather}")
    boxes = wl.sound_wave_boxes(counts=(301, 40, 30), seed=9)
    grids = [b.astype(np.float32).astype(np.float64) for b in boxes.grids]
    edges = [g.shape[1] for g in grids]
    efor = lambda L: 8 if L == 8 else 16
    bs = layout.boxes_blockset(edges, efor, boxes.dh)
    assert bs.n_blocks > 256 and (bs.edges == 8).sum() % 4 == 1
    outs = []
    for kernel in (tvd.TVD_KERNEL_BATCHED, tvd.TVD_KERNEL_PERSISTENT, tvd.TVD_KERNEL_AUTO):
        dev = DeviceBlocks(ctx, bs, dtype=torch.float32, gather=gather, kernel=kernel)
        dev.upload(layout.boxes_to_blocks(grids, efor))
        rec = dev.run(6, sums_each_step=True)
        torch.cuda.synchronize()
        outs.append((dev.interior.cpu().numpy(), dev.dt.cpu().numpy(), rec.cpu().numpy(),
                     dev.smax.cpu().numpy()))
    for o in outs[1:]:
        assert np.array_equal(outs[0][0], o[0])   # state
        assert np.array_equal(outs[0][1], o[1])   # dt
        assert np.array_equal(outs[0][3], o[3])   # signal speed (a max: exact)
        # compensated sums: the variants visit a block's cells in different
        # orders, so the last bit may differ
        np.testing.assert_allclose(outs[0][2], o[2], rtol=1e-15, atol=0)


@pytest.mark.parametrize("n", [8, 16])
def test_persistent_uniform_edge(ctx, n):
    """The persistent kernel also takes a uniform-edge batch (no d_edge):
    same bits as the one-workgroup-per-block launch."""
    note(f"persistent uniform edge {n}")
    g = wl.lognormal(64, seed=31, sigma_ln=0.6).astype(np.float32).astype(np.float64)
    a, _ = run_gpu_periodic(ctx, g, 4, n, torch.float32, kernel=tvd.TVD_KERNEL_BATCHED)
    b, _ = run_gpu_periodic(ctx, g, 4, n, torch.float32, kernel=tvd.TVD_KERNEL_PERSISTENT)
    assert np.array_equal(a, b)


def test_persistent_skips_unknown_edge(ctx):
    """A block whose edge entry is neither 8 nor 16 is left out of the
    persistent launch's plan: not advanced, counted once as non-physical; the
    other blocks are advanced as usual."""
    note("persistent launch with an unknown edge entry")
    boxes = wl.sound_wave_boxes(counts=(6, 2, 1), seed=10)
    grids = [b.astype(np.float32).astype(np.float64) for b in boxes.grids]
    edges = [g.shape[1] for g in grids]
    efor = lambda L: 8 if L == 8 else 16
    bs = layout.boxes_blockset(edges, efor, boxes.dh)
    dev = DeviceBlocks(ctx, bs, dtype=torch.float32, kernel=tvd.TVD_KERNEL_PERSISTENT)
    dev.upload(layout.boxes_to_blocks(grids, efor))
    dev.fill_ghosts()
    dev.dt.fill_(1e-3)
    dev.advance(0)
    ref = dev.interior.cpu().numpy()
    victim = int(np.nonzero(bs.edges == 16)[0][1])
    dev.edges[victim] = 12
    dev.interior.fill_(7.0)
    ctx.tvd_read_flags()
    dev.advance(0)
    st, fl, bad = ctx.tvd_read_flags()
    assert st == tvd.TVD_ERR_NONPHYSICAL and bad == 1 and fl == 0
    got = dev.interior.cpu().numpy()
    lo, hi = int(bs.out_off[victim]), int(bs.out_off[victim]) + 5 * 16 ** 3
    assert np.all(got[lo:hi] == 7.0)
    keep = np.ones(got.size, dtype=bool)
    keep[lo:hi] = False
    assert np.array_equal(got[keep], ref[keep])


def test_gather_missing_neighbour_is_flagged(ctx):
    note("gather with a missing neighbour")
    g = wl.uniform(16, rho=1.0, P=1.0)
    bs = layout.periodic_grid_blockset(16, 8)
    bs.nbr[3, 4] = -1
    dev = DeviceBlocks(ctx, bs, dtype=torch.float32, gather=True)
    dev.upload(layout.grid_to_blocks(g, 8))
    dev.spare.fill_(7.0)
    ctx.tvd_read_flags()
    dev.dt.fill_(1e-3)
    dev.advance(0)
    st, fl, bad = ctx.tvd_read_flags()
    assert st == tvd.TVD_ERR_NONPHYSICAL and bad == 8 ** 3
    out = dev.interior.cpu().numpy().reshape(8, 5, 8, 8, 8)
    assert np.all(out[3] == 7.0)                      # block 3 untouched
    assert np.array_equal(out[0], layout.grid_to_blocks(g, 8)[0].astype(np.float32))


def test_fill_ghosts_bitwise(ctx):
    note("ghost fill vs periodic copy, n=8 and 16, FP64")
    g = wl.lognormal(32, seed=21)
    for n in (8, 16):
        bs = layout.periodic_grid_blockset(32, n)
        dev = DeviceBlocks(ctx, bs, dtype=torch.float64)
        dev.upload(layout.grid_to_blocks(g, n))
        dev.fill_ghosts()
        torch.cuda.synchronize()
        m = n + 6
        got = dev.ghosted.cpu().numpy().reshape(bs.n_blocks, 5, m, m, m)
        want = oracle.periodic_ghosted_blocks(g, n)
        assert np.array_equal(got, want)


# ---------------------------------------------------------------------------
# FP64 parity (<= 1e-12)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kernel", [tvd.TVD_KERNEL_PLAIN, tvd.TVD_KERNEL_BATCHED])
def test_sod_32cube_fp64(ctx, kernel):
    """Sod tube along x on a periodic 32^3 grid as 64 patches of 8^3, 10 steps
    at CFL 0.5 (the paper's Sec. 4.2 states)."""
    note(f"sod 32^3 fp64 kernel={kernel}")
    g = wl.sod_x(32)
    ref, dts = oracle_periodic(g, 10, n=8)
    out, dev = run_gpu_periodic(ctx, g, 10, 8, torch.float64, kernel)
    nrm = norms(out, ref)
    note(str({k: (v["relL1"], v["relLinf"]) for k, v in nrm.items()}))
    check(nrm, FP64)
    np.testing.assert_allclose(dev.dt.cpu().numpy(), dts[-1], rtol=1e-14)


@pytest.mark.parametrize("kernel", [tvd.TVD_KERNEL_PLAIN, tvd.TVD_KERNEL_BATCHED])
def test_lognormal_fp64(ctx, kernel):
    """Rough lognormal density (sigma_ln = 1) with Gaussian velocities, 32^3,
    6 steps: the shape of the 256^3 throughput workload at a size the oracle
    runs in seconds."""
    note(f"lognormal 32^3 fp64 kernel={kernel}")
    g = wl.lognormal(32, seed=7)
    ref, _ = oracle_periodic(g, 6, n=8)
    out, _ = run_gpu_periodic(ctx, g, 6, 8, torch.float64, kernel)
    nrm = norms(out, ref)
    note(str({k: (v["relL1"], v["relLinf"]) for k, v in nrm.items()}))
    check(nrm, FP64)


def test_plain_equals_batched_fp64(ctx):
    note("plain vs batched fp64 (both against the oracle, and each other)")
    g = wl.smooth_random(16, seed=3, amplitude=0.4)
    a, _ = run_gpu_periodic(ctx, g, 4, 8, torch.float64, tvd.TVD_KERNEL_PLAIN)
    b, _ = run_gpu_periodic(ctx, g, 4, 8, torch.float64, tvd.TVD_KERNEL_BATCHED)
    check(norms(a, b), (1e-13, 1e-13))


# ---------------------------------------------------------------------------
# FP32 parity (<= 1e-5 on smooth data after 10 steps)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [8, 16])
def test_smooth_fp32(ctx, n):
    note(f"smooth 32^3 fp32 n={n}")
    g = wl.smooth_random(32, seed=9, amplitude=0.1, vel=0.1)
    g = g.astype(np.float32).astype(np.float64)
    ref, _ = oracle_periodic(g, 10, n=8)
    out, _ = run_gpu_periodic(ctx, g, 10, n, torch.float32)
    nrm = norms(out, ref)
    note(str({k: (v["relL1"], v["relL1_own"], v["relLinf"]) for k, v in nrm.items()}))
    check(nrm, FP32_SMOOTH)


def test_uneven_boxes_fp32(ctx):
    """Independent periodic boxes of 8^3, 16^3 and 32^3 (4:2:1) with sound
    waves of amplitude 1e-3, one mixed-edge batch (8^3 boxes as edge-8
    blocks, the others as edge-16 blocks), per-block dh, 10 steps."""
    note("uneven boxes fp32 mixed edges")
    boxes = wl.sound_wave_boxes(counts=(8, 4, 2), seed=4)
    grids = [b.astype(np.float32).astype(np.float64) for b in boxes.grids]
    edges = [g.shape[1] for g in grids]
    efor = lambda L: 8 if L == 8 else 16
    bs = layout.boxes_blockset(edges, efor, boxes.dh)
    dev = DeviceBlocks(ctx, bs, dtype=torch.float32)
    dev.upload(layout.boxes_to_blocks(grids, efor))
    dev.run(10)
    torch.cuda.synchronize()
    got = layout.blocks_to_boxes(dev.download(), edges, efor)
    # oracle: every box on its own, with the global dt rule dt_b = C dh_b / S
    # (S over all boxes), evaluated before even steps
    state = [g.copy() for g in grids]
    for s in range(10):
        if s % 2 == 0:
            S = max(oracle.max_signal_speed(g, GAMMA) for g in state)
        state = [oracle.step_periodic(g, 8, s % 2, 0.5 * h / S, h, GAMMA)
                 for g, h in zip(state, boxes.dh)]
    a = np.concatenate([x.reshape(5, -1) for x in got], axis=1)
    b = np.concatenate([x.reshape(5, -1) for x in state], axis=1)
    nrm = norms(a, b)
    note(str({k: (v["relL1"], v["relL1_own"], v["relLinf"]) for k, v in nrm.items()}))
    check(nrm, FP32_SMOOTH)


# ---------------------------------------------------------------------------
# CFL speed, dt and sums
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_signal_speed_and_dt(ctx, dtype):
    note(f"signal speed dtype={dtype}")
    g = wl.lognormal(32, seed=5)
    g = g.astype(np.float32).astype(np.float64) if dtype == torch.float32 else g
    bs = layout.periodic_grid_blockset(32, 8)
    dev = DeviceBlocks(ctx, bs, dtype=dtype)
    dev.upload(layout.grid_to_blocks(g, 8))
    dev.signal_speed()
    dev.set_dt_from_speed()
    torch.cuda.synchronize()
    S = oracle.max_signal_speed(g, GAMMA)
    assert dev.smax.item() == pytest.approx(S, rel=2e-15)
    np.testing.assert_allclose(dev.dt.cpu().numpy(), 0.5 / 32 / S, rtol=4e-15)


def test_conservation_sums_exact_on_dyadic_data(ctx):
    note("conservation sums on dyadic data")
    r = wl.rng(8)
    g = r.integers(-2 ** 16, 2 ** 16, size=(5, 32, 32, 32)).astype(np.float64) * 2.0 ** -10
    g[0] = np.abs(g[0]) + 1.0
    bs = layout.periodic_grid_blockset(32, 8)
    dev = DeviceBlocks(ctx, bs, dtype=torch.float64)
    dev.upload(layout.grid_to_blocks(g, 8))
    sums = dev.conservation_sums().cpu().numpy()
    w = (1.0 / 32) ** 3
    for k in range(5):
        assert sums[k] == math.fsum((g[k] * w).ravel())


def test_fused_diagnostics_match_standalone(ctx):
    note("fused speed/sums vs standalone kernels")
    g = wl.lognormal(32, seed=12, sigma_ln=0.5)
    for dtype, n in [(torch.float32, 16), (torch.float32, 8), (torch.float64, 8)]:
        bs = layout.periodic_grid_blockset(32, n)
        dev = DeviceBlocks(ctx, bs, dtype=dtype)
        dev.upload(layout.grid_to_blocks(g, n))
        dev.signal_speed()
        dev.set_dt_from_speed()
        dev.fill_ghosts()
        dev.advance(0, fuse_speed=True, fuse_sums=True)
        torch.cuda.synchronize()
        s_fused, sums_fused = dev.smax.item(), dev.sums.cpu().numpy().copy()
        dev.signal_speed()
        sums = dev.conservation_sums().cpu().numpy()
        assert dev.smax.item() == s_fused
        np.testing.assert_allclose(sums_fused, sums, rtol=1e-14, atol=1e-300)
        # and the sums equal the exactly rounded sums of the stored state
        out = np.stack(dev.download()).astype(np.float64)
        w = (1.0 / 32) ** 3
        for k in range(5):
            exact = math.fsum(out[:, k].ravel()) * w
            assert abs(sums[k] - exact) <= 1e-14 * abs(exact) + 1e-300


def test_conservation_over_steps_fp64(ctx):
    note("conservation over 10 steps, fp64 batched")
    g = wl.lognormal(32, seed=13)
    bs = layout.periodic_grid_blockset(32, 8)
    dev = DeviceBlocks(ctx, bs, dtype=torch.float64)
    dev.upload(layout.grid_to_blocks(g, 8))
    rec = dev.run(10, sums_each_step=True).cpu().numpy()
    w = (1.0 / 32) ** 3
    s0 = np.array([math.fsum((g[k] * w).ravel()) for k in range(5)])
    scale = np.array([np.abs(g[k]).sum() * w for k in range(5)])
    assert np.all(np.abs(rec - s0) <= 1e-13 * scale)


# ---------------------------------------------------------------------------
# graph capture, flags, argument errors, empty batch
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("gather", [False, True])
def test_graph_replay_matches_eager(ctx, gather):
    """A two-step sequence recorded into a HIP graph by the library's native
    capture and replayed three times, with eager work in between, equals the
    eager sequence bit for bit after every replay."""
    note(f"native graph capture of a 2-step sequence, gather={gather}")
    g = wl.smooth_random(32, seed=14, amplitude=0.2).astype(np.float32).astype(np.float64)
    bs = layout.periodic_grid_blockset(32, 16)
    eager = DeviceBlocks(ctx, bs, dtype=torch.float32, gather=gather)
    graph = DeviceBlocks(ctx, bs, dtype=torch.float32, gather=gather)
    eager.upload(layout.grid_to_blocks(g, 16))
    graph.upload(layout.grid_to_blocks(g, 16))
    for d in (eager, graph):
        d.run(2)   # the first pair seeds the fused signal speed
    torch.cuda.synchronize()
    gr = graph.capture(2)
    torch.cuda.synchronize()
    for rep in range(3):
        eager.run(2)
        torch.cuda.synchronize()
        x = eager.interior.sum()  # eager work between replays
        graph.replay(gr)
        torch.cuda.synchronize()
        assert torch.equal(eager.interior, graph.interior), rep
        assert torch.equal(eager.dt, graph.dt), rep
        del x
    gr.close()


def test_graph_replay_persistent_mixed_edges(ctx):
    """A four-step sequence of persistent mixed-edge launches (each with its
    planning kernel, which clears the work counters) recorded into a HIP graph
    and replayed three times, with eager work in between, equals the eager
    sequence bit for bit after every replay; then the block-edge tuner runs on
    the same boxes."""
    note("graph capture of persistent mixed-edge steps; block-edge tuner")
    from paper_0907_3390_amd import tuning
    boxes = wl.sound_wave_boxes(counts=(61, 10, 6), seed=12)
    grids = [b.astype(np.float32).astype(np.float64) for b in boxes.grids]
    efor = lambda L: 8 if L == 8 else 16
    eager = tuning.boxes_device(ctx, grids, boxes.dh, efor)
    graph = tuning.boxes_device(ctx, grids, boxes.dh, efor)
    for d in (eager, graph):
        d.run(2)
    torch.cuda.synchronize()
    gr = graph.capture(4)
    torch.cuda.synchronize()
    for rep in range(3):
        eager.run(4)
        torch.cuda.synchronize()
        x = eager.interior.sum()
        graph.replay(gr)
        torch.cuda.synchronize()
        assert torch.equal(eager.interior, graph.interior), rep
        assert torch.equal(eager.dt, graph.dt), rep
        del x
    gr.close()
    best, times = tuning.tune_block_edge(
        ctx, grids, boxes.dh, {"8": lambda L: 8, "8/16": efor}, pairs=2)
    assert best in ("8", "8/16") and all(t > 0 for t in times.values())


def test_torch_graph_capture_also_works(ctx):
    """The entry points are capture-safe under torch's graph wrapper too."""
    note("torch graph capture")
    g = wl.smooth_random(32, seed=18, amplitude=0.2).astype(np.float32).astype(np.float64)
    bs = layout.periodic_grid_blockset(32, 16)
    eager = DeviceBlocks(ctx, bs, dtype=torch.float32, gather=True)
    graph = DeviceBlocks(ctx, bs, dtype=torch.float32, gather=True)
    for d in (eager, graph):
        d.upload(layout.grid_to_blocks(g, 16))
        d.run(2)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    cg = torch.cuda.CUDAGraph()
    with torch.cuda.graph(cg, stream=s):
        graph.step()
        graph.step()
    graph.step_index -= 2
    for rep in range(2):
        eager.run(2)
        cg.replay()
        graph.step_index += 2
        torch.cuda.synchronize()
        assert torch.equal(eager.interior, graph.interior), rep


@pytest.mark.parametrize("dtype,edge", [(torch.float32, 16), (torch.float32, 8), (torch.float64, 8)])
def test_all_variants_bitwise_equal_and_autotune(ctx, dtype, edge):
    """Every compiled launch variant (workgroup size, LDS padding, pencils per
    thread) computes the same arithmetic per cell: results are bit-identical.
    The tuner then picks one of them."""
    note(f"variants and autotune dtype={dtype} edge={edge}")
    code = tvd.dtype_code(dtype)
    g = wl.lognormal(32, seed=19, sigma_ln=0.6)
    if dtype == torch.float32:
        g = g.astype(np.float32).astype(np.float64)
    bs = layout.periodic_grid_blockset(32, edge)
    ref = None
    cands = [v for v in tvd.variants() if v[1] == edge]
    assert cands
    for v in cands:
        ctx.tvd_set_variant(code, edge, v[0])
        dev = DeviceBlocks(ctx, bs, dtype=dtype, gather=True)
        dev.upload(layout.grid_to_blocks(g, edge))
        dev.run(2)
        torch.cuda.synchronize()
        out = dev.interior.cpu().numpy()
        if ref is None:
            ref = out
        assert np.array_equal(out, ref), v
    ctx.tvd_set_variant(code, edge, -1)
    dev = DeviceBlocks(ctx, bs, dtype=dtype, gather=True)
    dev.upload(layout.grid_to_blocks(g, edge))
    dev.dt.fill_(1e-3)
    idx, ms = ctx.tvd_autotune(dev.batch, dev.nbr, dev.interior, dev.spare, GAMMA, reps=2)
    assert idx in [v[0] for v in cands] and ms > 0
    ctx.tvd_set_variant(code, edge, -1)


def test_health_flags(ctx):
    note("health counters")
    g = wl.uniform(16, rho=1.0, P=1.0)
    g[0, 4, 4, 4] = -1.0  # one cell with negative density
    bs = layout.periodic_grid_blockset(16, 8)
    dev = DeviceBlocks(ctx, bs, dtype=torch.float64)
    dev.upload(layout.grid_to_blocks(g, 8))
    ctx.tvd_read_flags()
    dev.dt.fill_(1e-3)
    dev.fill_ghosts()
    dev.advance(0)
    st, fl, bad = ctx.tvd_read_flags()
    assert st == tvd.TVD_ERR_NONPHYSICAL and bad > 0
    st, fl, bad = ctx.tvd_read_flags()
    assert st == tvd.TVD_OK and bad == 0 and fl == 0  # reset after read
    # pressure floor: cold cells below the floor are counted, not changed
    g = wl.uniform(16, rho=1.0, P=1e-12)
    dev.upload(layout.grid_to_blocks(g, 8))
    dev.p_floor = 1e-10
    dev.fill_ghosts()
    dev.advance(0)
    st, fl, bad = ctx.tvd_read_flags()
    assert st == tvd.TVD_WARN_FLOORED and fl == 16 ** 3 and bad == 0


def test_argument_errors(ctx):
    note("argument validation")
    dev_in = torch.zeros(5 * 14 ** 3, dtype=torch.float64, device="cuda")
    dev_out = torch.zeros(5 * 8 ** 3, dtype=torch.float64, device="cuda")
    ok = tvd.Batch(tvd.TVD_F64, 1, 8, dt=1e-3, dh=1.0)
    E = tvd.TvdError
    with pytest.raises(E) as e:
        ctx.tvd_patch_advance(tvd.Batch(tvd.TVD_F64, 1, 12, dt=1e-3, dh=1.0), dev_in, dev_out, 0, GAMMA)
    assert e.value.status == tvd.TVD_ERR_INVALID_ARG
    with pytest.raises(E) as e:
        ctx.tvd_patch_advance(ok, dev_in, dev_in, 0, GAMMA)
    assert e.value.status == tvd.TVD_ERR_ALIAS
    big_in = torch.zeros(5 * 22 ** 3, dtype=torch.float64, device="cuda")
    big_out = torch.zeros(5 * 16 ** 3, dtype=torch.float64, device="cuda")
    with pytest.raises(E) as e:
        ctx.tvd_patch_advance(tvd.Batch(tvd.TVD_F64, 1, 16, dt=1e-3, dh=1.0), big_in, big_out, 0, GAMMA)
    assert e.value.status == tvd.TVD_ERR_UNSUPPORTED
    with pytest.raises(E) as e:
        ctx.tvd_patch_advance(tvd.Batch(tvd.TVD_F32, 1, 8, dt=1e-3, dh=1.0), dev_in, dev_out, 0,
                              GAMMA, flags=tvd.TVD_KERNEL_PLAIN)
    assert e.value.status == tvd.TVD_ERR_UNSUPPORTED
    for bad_gamma in (0.5, float("nan")):
        with pytest.raises(E) as e:
            ctx.tvd_patch_advance(ok, dev_in, dev_out, 0, bad_gamma)
        assert e.value.status == tvd.TVD_ERR_INVALID_ARG
    with pytest.raises(E) as e:
        ctx.tvd_patch_advance(ok, dev_in, dev_out, 2, GAMMA)
    assert e.value.status == tvd.TVD_ERR_INVALID_ARG
    with pytest.raises(E) as e:
        ctx.tvd_dt_from_speed(ok, dev_out, 1.5, dev_out)
    assert e.value.status == tvd.TVD_ERR_INVALID_ARG
    # empty batch: nothing to do, nothing launched
    assert ctx.tvd_patch_advance(tvd.Batch(tvd.TVD_F64, 0, 8, dt=1e-3, dh=1.0), dev_in, dev_out, 0,
                                 GAMMA) == tvd.TVD_OK
    torch.cuda.synchronize()


# ---------------------------------------------------------------------------
# full-size workloads, sampled outputs from each block's dependency cone
# ---------------------------------------------------------------------------

def _full_size_sampled(ctx, grid, n, dtype, steps, dt, picks, p_floor=0.0, bounds=FP32_ROUGH,
                       curve="morton", stream=False):
    """picks are x-fastest (linear) block indices; the device numbers the
    blocks along `curve`, as the bench does (and, with `stream`, advances
    them with the streamed kernel over its default chains)."""
    N = grid.shape[3]
    bs = layout.periodic_grid_blockset(N, n, curve=curve)
    dev = DeviceBlocks(ctx, bs, dtype=dtype, gather=True, p_floor=p_floor, stream=stream)
    dev.upload(layout.grid_to_blocks(grid, n, bs.perm))
    slot = np.argsort(bs.perm) if bs.perm is not None else np.arange(bs.n_blocks)
    dev.dt.fill_(dt)
    ctx.tvd_read_flags()
    for s in range(steps):
        dev.advance(s % 2, fuse_sums=True)
    torch.cuda.synchronize()
    st, fl, bad = ctx.tvd_read_flags()
    assert bad == 0
    sums = dev.sums.cpu().numpy()
    out = dev.interior.cpu().numpy()
    from gpu_helpers import cone_blocks
    ref = cone_blocks(grid, n, picks, steps, dt, 1.0 / N, p_floor=p_floor)
    m3 = 5 * n ** 3
    got = np.stack([out[slot[p] * m3:(slot[p] + 1) * m3].reshape(5, -1) for p in picks],
                   1).reshape(5, -1)
    want = np.stack([ref[p].reshape(5, -1) for p in picks], 1).reshape(5, -1)
    nrm = norms(got, want)
    note(str({k: (f"{v['relL1']:.2e}", f"{v['relLinf']:.2e}") for k, v in nrm.items()}))
    check(nrm, bounds)
    # conservation: the fused FP64 sums of the output against the input's exact
    # sums, on each variable's own scale (momentum: sum of rho c_s)
    w = (1.0 / N) ** 3
    rho = grid[0]
    kin = 0.5 * (grid[1] ** 2 + grid[2] ** 2 + grid[3] ** 2) / rho
    P = np.maximum((GAMMA - 1.0) * (grid[4] - kin), p_floor)
    mscale = np.sum(rho * np.sqrt(GAMMA * P / rho)) * w
    for k in range(5):
        s0 = math.fsum((grid[k].ravel() * w).tolist())
        scale = np.abs(grid[k]).sum() * w if k in (0, 4) else mscale
        assert abs(sums[k] - s0) <= (1e-6 if dtype == torch.float32 else 1e-13) * scale, k
    return nrm


@pytest.mark.parametrize("stream", [False, True])
def test_full_size_256cube_bench_config_fp32(ctx, stream):
    """The 256^3 rough lognormal workload at full size (4096 patch groups of
    16^3 numbered along the Morton curve, FP32, gathering advance, per-block
    or streamed): two steps (xyz, zyx), 24 sampled blocks against the
    oracle's dependency-cone result."""
    note(f"full size 256^3 lognormal fp32, sampled blocks, stream={stream}")
    g = wl.lognormal(256, seed=2024).astype(np.float32).astype(np.float64)
    S = oracle.max_signal_speed(g, GAMMA)
    dt = 0.5 / 256 / S
    picks = sorted(set(int(x) for x in wl.rng(1).integers(0, 4096, size=24)) | {0, 4095})
    _full_size_sampled(ctx, g, 16, torch.float32, 2, dt, picks, bounds=FP32_ROUGH, stream=stream)


@pytest.mark.parametrize("n,stream", [(16, True), (8, False)])
def test_full_size_256cube_fp64(ctx, n, stream):
    """The 256^3 rough lognormal workload at full size in FP64: as 4096
    groups of 16^3 by the streamed advance, or as 32768 patches of 8^3 by the
    per-block gathering kernel (Morton-numbered): two steps (xyz, zyx), 24
    sampled blocks against the oracle's dependency-cone result, relative L1
    and Linf <= 1e-12 per variable, and the fused FP64 sums conserved to
    1e-13 of each variable's scale."""
    note(f"full size 256^3 lognormal fp64, edge {n}, stream={stream}")
    g = wl.lognormal(256, seed=2024)
    S = oracle.max_signal_speed(g, GAMMA)
    dt = 0.5 / 256 / S
    nb = (256 // n) ** 3
    picks = sorted(set(int(x) for x in wl.rng(3).integers(0, nb, size=24)) | {0, nb - 1})
    _full_size_sampled(ctx, g, n, torch.float64, 2, dt, picks, bounds=FP64, stream=stream)


@pytest.mark.parametrize("stream", [False, True])
def test_full_size_512cube_sedov_fp32(ctx, stream):
    """The headline workload at full size: 512^3 = 262144 patches of 8^3 run
    as 32768 groups of 16^3, point blast on a lognormal background with
    p_floor 1e-10, FP32, per-block or streamed: four steps, against the
    oracle on the blocks holding the blast (cells 255 and 256 on every axis
    lie in groups 15 and 16), the groups across each of their faces, and
    others spread over the grid."""
    note(f"full size 512^3 sedov fp32, 4 steps, sampled blocks, stream={stream}")
    g = wl.sedov_lognormal(512, seed=5).astype(np.float32).astype(np.float64)
    S = oracle.max_signal_speed(g, GAMMA, 1e-10)
    dt = 0.5 / 512 / S
    lin = lambda x, y, z: x + 32 * (y + 32 * z)
    centre = {lin(x, y, z) for x in (15, 16) for y in (15, 16) for z in (15, 16)}
    faces = {lin(14, 15, 16), lin(17, 16, 15), lin(15, 14, 16), lin(16, 17, 15),
             lin(16, 15, 14), lin(15, 16, 17)}
    picks = sorted(centre | faces | {0, 12345, 32767})
    _full_size_sampled(ctx, g, 16, torch.float32, 4, dt, picks, p_floor=1e-10,
                       bounds=(1e-4, 1e-3), stream=stream)


def test_full_size_uneven_boxes_fp32(ctx):
    """The uneven batch at full size: 4000 periodic boxes, 2286 of 8^3, 1143 of
    16^3 and 571 of 32^3, sound waves of amplitude 1e-3, FP32, the persistent
    gathering launch (8^3 boxes as edge-8 blocks, the rest as 16^3 groups),
    dt_b = C dh_b / S from the device; 10 steps against the oracle run over
    every box: relative L1 <= 1e-5 per variable."""
    note("full size uneven boxes fp32, persistent launch, 10 steps")
    boxes = wl.sound_wave_boxes(seed=4)
    grids = [b.astype(np.float32).astype(np.float64) for b in boxes.grids]
    edges = [g.shape[1] for g in grids]
    assert len(grids) == 4000 and sum(L ** 3 for L in edges) == 24_562_688
    efor = lambda L: 8 if L == 8 else 16
    bs = layout.boxes_blockset(edges, efor, boxes.dh)
    dev = DeviceBlocks(ctx, bs, dtype=torch.float32, gather=True)
    dev.upload(layout.boxes_to_blocks(grids, efor))
    ctx.tvd_read_flags()
    dev.run(10)
    torch.cuda.synchronize()
    st, fl, bad = ctx.tvd_read_flags()
    assert st == tvd.TVD_OK and fl == 0 and bad == 0
    got = layout.blocks_to_boxes(dev.download(), edges, efor)
    note("oracle over 4000 boxes")
    want = oracle_boxes(grids, boxes.dh, 10)
    a = np.concatenate([x.reshape(5, -1) for x in got], axis=1)
    b = np.concatenate([x.reshape(5, -1) for x in want], axis=1)
    nrm = norms(a, b)
    note(str({k: (v["relL1"], v["relL1_own"], v["relLinf"]) for k, v in nrm.items()}))
    check(nrm, FP32_SMOOTH)


def test_sedov_128cube_100_steps_fp32(ctx):
    """The point blast's 128^3 analog over all 100 steps (lognormal background
    sigma_ln = 0.5 at rest, P = 1e-5, energy 1 in the central 2^3 cells,
    p_floor 1e-10), FP32 gathering advance with the fused FP64 sums recorded
    every step, against the FP64 oracle run over the same 100 steps (its own
    dt): error per variable, conservation drift per step, health counters."""
    note("sedov 128^3 analog, 100 steps fp32")
    N, steps, pf = 128, 100, 1e-10
    g = wl.sedov_lognormal(N, seed=5).astype(np.float32).astype(np.float64)
    bs = layout.periodic_grid_blockset(N, 16, curve="morton")
    dev = DeviceBlocks(ctx, bs, dtype=torch.float32, gather=True, p_floor=pf)
    dev.upload(layout.grid_to_blocks(g, 16, bs.perm))
    ctx.tvd_read_flags()
    rec = dev.run(steps, sums_each_step=True)
    torch.cuda.synchronize()
    st, fl, bad = ctx.tvd_read_flags()
    note(f"health: floored {fl}, non-physical {bad}")
    assert bad == 0
    got = layout.blocks_to_grid(np.stack(dev.download()), g.shape, bs.perm)
    note("oracle, 100 steps")
    want, _ = oracle.run_periodic(g, steps, 0.5, 1.0 / N, GAMMA, n=32, p_floor=pf)
    nrm = norms(got, want)
    note(str({k: (f"{v['relL1']:.2e}", f"{v['relLinf']:.2e}") for k, v in nrm.items()}))
    check(nrm, (1e-4, 1e-2))
    # conservation drift of the fused FP64 sums, every step, against the exact
    # sums of the initial state on each variable's own scale
    w = (1.0 / N) ** 3
    sums = rec.cpu().numpy()
    rho = g[0]
    kin = 0.5 * (g[1] ** 2 + g[2] ** 2 + g[3] ** 2) / rho
    P = np.maximum((GAMMA - 1.0) * (g[4] - kin), pf)
    mscale = np.sum(rho * np.sqrt(GAMMA * P / rho)) * w
    drift = []
    for k in range(5):
        s0 = math.fsum((g[k].ravel() * w).tolist())
        scale = np.abs(g[k]).sum() * w if k in (0, 4) else mscale
        drift.append(np.max(np.abs(sums[:, k] - s0)) / scale)
    note(f"max conservation drift over 100 steps (rho, m_x, m_y, m_z, e): {drift}")
    assert max(drift) <= 1e-6


# ---------------------------------------------------------------------------
# multi-level batch: per-block dt and dh in one launch
# ---------------------------------------------------------------------------

def _multilevel_check(ctx, ghosted, dhs, levels, edge, cases):
    """One step of every block (8^3 patches or 16^3 patch groups, ghosted)
    with dt_b = C dh_b / S_global computed on the device, for each (dtype,
    kernel, tol) case, against the oracle's own dt and step from the same
    (FP32-rounded for FP32) input.  The plain FP64 kernel is launched level by
    level on each level's contiguous range."""
    nb = len(dhs)
    m, n = edge + 6, edge
    refs = {}
    for dtype, kernel, tol in cases:
        code = tvd.dtype_code(dtype)
        gin = ghosted.astype(np.float32).astype(np.float64) if dtype == torch.float32 else ghosted
        if dtype not in refs:
            S = oracle.max_signal_speed(np.ascontiguousarray(
                gin[:, :, 3:-3, 3:-3, 3:-3].transpose(1, 0, 2, 3, 4)).reshape(5, -1), GAMMA)
            dt_ref = 0.5 * dhs / S
            refs[dtype] = (dt_ref, np.stack(oracle.advance_ragged(list(gin), 0, dt_ref, dhs, GAMMA)))
        dt_ref, want = refs[dtype]
        u_in = torch.from_numpy(np.ascontiguousarray(gin)).to(dtype).cuda().reshape(-1)
        u_out = torch.zeros(nb * 5 * n ** 3, dtype=dtype, device="cuda")
        d_dh = torch.from_numpy(np.ascontiguousarray(dhs)).cuda()
        d_dt = torch.zeros(nb, dtype=torch.float64, device="cuda")
        smax = torch.zeros(1, dtype=torch.float64, device="cuda")
        b = tvd.Batch(code, nb, edge, d_dt=d_dt, d_dh=d_dh)
        ctx.tvd_reserve(nb)
        ctx.tvd_max_signal_speed(b, u_in, tvd.TVD_LAYOUT_GHOSTED, GAMMA, smax)
        ctx.tvd_dt_from_speed(b, smax, 0.5, d_dt)
        if kernel == tvd.TVD_KERNEL_PLAIN:
            for lev in np.unique(levels):
                ids = np.nonzero(levels == lev)[0]
                lo, hi = int(ids[0]), int(ids[-1]) + 1
                assert hi - lo == ids.size
                bl = tvd.Batch(code, hi - lo, edge, d_dt=d_dt[lo:hi], d_dh=d_dh[lo:hi])
                ctx.tvd_patch_advance(bl, u_in[lo * 5 * m ** 3:], u_out[lo * 5 * n ** 3:], 0, GAMMA,
                                      flags=kernel)
        else:
            ctx.tvd_patch_advance(b, u_in, u_out, 0, GAMMA, flags=kernel)
        torch.cuda.synchronize()
        np.testing.assert_allclose(d_dt.cpu().numpy(), dt_ref, rtol=1e-14)
        got = u_out.cpu().numpy().reshape(nb, 5, n, n, n)
        nrm = norms(got.transpose(1, 0, 2, 3, 4).reshape(5, -1),
                    want.transpose(1, 0, 2, 3, 4).reshape(5, -1))
        note(f"edge {edge} {dtype} kernel {kernel}: " +
             str({k: (f"{v['relL1']:.2e}", f"{v['relLinf']:.2e}") for k, v in nrm.items()}))
        check(nrm, (tol, FP64[1] if dtype == torch.float64 else FP32_SMOOTH[1]))
        del u_in, u_out


def test_multilevel_batch_one_launch(ctx):
    """Patches of levels 0-3 (dh halving per level) around Gaussian
    overdensities, ghosts pre-filled by sibling copy or trilinear coarse-to-
    fine interpolation; dt_b = C dh_b / S_global computed on the device.  One
    batched launch (FP32 and FP64), one persistent FP32 launch and the plain
    FP64 kernel launched level by level all match the oracle; so does the
    same hierarchy as 2^3 patch groups of 16^3 in one FP32 launch."""
    note("multi-level batch")
    ml = wl.multilevel(base=32, n_over=4, seed=5, radius=0.07)
    assert set(np.unique(ml.levels)) == {0, 1, 2, 3}
    _multilevel_check(ctx, ml.ghosted, ml.dh, ml.levels, 8,
                      [(torch.float64, tvd.TVD_KERNEL_BATCHED, 1e-12),
                       (torch.float32, tvd.TVD_KERNEL_BATCHED, 1e-5),
                       (torch.float32, tvd.TVD_KERNEL_PERSISTENT, 1e-5),
                       (torch.float64, tvd.TVD_KERNEL_PLAIN, 1e-12)])
    groups, G, gdh = ml.group_blocks()
    glev = np.array([g[0] for g in groups])
    _multilevel_check(ctx, G, gdh, glev, 16,
                      [(torch.float32, tvd.TVD_KERNEL_BATCHED, 1e-5),
                       (torch.float32, tvd.TVD_KERNEL_PERSISTENT, 1e-5)])


def test_multilevel_full_size_fp32(ctx):
    """The multi-level batch at full size: a 128^3 base (4096 patches) and
    levels 1-3 around 32 overdensities (18 152 patches in all): one persistent
    FP32 launch on the patches and on their 2^3 patch groups (2269 blocks of
    16^3), and the plain FP64 kernel per level, against the oracle."""
    note("multi-level batch, full size")
    ml = wl.multilevel()
    counts = np.bincount(ml.levels)
    note(f"patches per level {counts.tolist()}")
    assert len(counts) == 4 and counts[0] == 4096 and len(ml.patches) > 15000
    _multilevel_check(ctx, ml.ghosted, ml.dh, ml.levels, 8,
                      [(torch.float32, tvd.TVD_KERNEL_PERSISTENT, 1e-5),
                       (torch.float64, tvd.TVD_KERNEL_PLAIN, 1e-12)])
    groups, G, gdh = ml.group_blocks()
    _multilevel_check(ctx, G, gdh, np.array([g[0] for g in groups]), 16,
                      [(torch.float32, tvd.TVD_KERNEL_PERSISTENT, 1e-5)])
