"""The nested-level driver on the device (paper_0907_3390_amd.amr.NestedDevice):
three levels held as 8^3 patches or as 2^3 patch groups of 16^3 (Sec. 3.1),
every level sub-cycled in its parent's step (Sec. 2.1), each pair closed
finest first, against the oracle's recursive step: FP64 within 1e-12 and
FP32 within 1e-5 (relative L1 per level and variable, the oracle run on the
FP32-rounded start); the leaf totals are conserved over several root steps;
a captured HIP graph of two root steps replays to the eager steps' bits.
Patch groups advance in FP32 only (the flux-recording FP64 advance holds
blocks of edge 8); their conservation is checked on the full hierarchy."""
import numpy as np
import pytest
import torch

from oracle import closing, ghosts
from gpu_helpers import FP64, GAMMA, check, norms, note
from paper_0907_3390_amd import amr, tvd, workloads as wl

pytestmark = pytest.mark.gpu
NC = 32


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    c = tvd.Context(0)
    yield c
    c.close()


def _refined():
    r0 = np.zeros((4, 4, 4), dtype=bool)
    r0[1:3, 1:3, 1:3] = True
    r1 = np.zeros((8, 8, 8), dtype=bool)
    r1[3, 3, 3] = r1[3, 3, 4] = r1[3, 4, 3] = True
    return [r0, r1]


def _states(seed, f32):
    s = [wl.lognormal(NC, seed=seed, sigma_ln=0.5)]
    for lev in (1, 2):
        M = NC << lev
        g = np.meshgrid(np.arange(M), np.arange(M), np.arange(M), indexing="ij")
        f = ghosts.coarse_to_fine(s[-1], *g)
        bump = wl.smooth_random(M, seed=seed + lev, amplitude=1.0)[0:1]
        s.append(f * (1.0 + 0.05 * bump / np.abs(bump).max()))
    if f32:
        s = [a.astype(np.float32).astype(np.float64) for a in s]
    return s


def _blocks(L, states):
    e = L.n
    return [np.stack([st[:, z:z + e, y:y + e, x:x + e] for z, y, x in L.origins[lev]])
            for lev, st in enumerate(states)]


def _dense(L, blocks):
    out, e = [], L.n
    for lev, bl in enumerate(blocks):
        M = NC << lev
        g = np.zeros((5, M, M, M))
        for b, (z, y, x) in zip(bl, L.origins[lev]):
            g[:, z:z + e, y:y + e, x:x + e] = b
        out.append(g)
    return out


@pytest.mark.parametrize("dtype,n", [(torch.float64, 8), (torch.float32, 8),
                                     (torch.float32, 16)])
def test_nested_driver_matches_oracle(ctx, dtype, n):
    note(f"nested driver, three levels, dtype={dtype}, blocks of {n}^3")
    states = _states(500, dtype == torch.float32)
    dev = amr.NestedDevice(ctx, NC, _refined(), dtype=dtype, n=n)
    L = dev.L
    dev.upload([b.astype(np.float32) if dtype == torch.float32 else b for b in _blocks(L, states)])
    dt = 0.1 / NC
    want = states
    for o in (0, 1):
        dev.step(dt, o)
        want = closing.nested_step_subcycled(want, L.refined, dt, o, GAMMA)
    torch.cuda.synchronize()
    assert ctx.tvd_read_flags()[2] == 0
    got = dev.download()
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    for lev, (g, w) in enumerate(zip(got, _blocks(L, want))):
        for k in range(5):
            scale = np.abs(w[:, 0]).sum() if k in (1, 2, 3) else np.abs(w[:, k]).sum()
            err = np.abs(g[:, k] - w[:, k]).sum() / scale
            note(f"  level {lev} var {k}: relL1 {err:.1e}")
            assert err <= tol, (lev, k, err)
        check(norms(g.transpose(1, 0, 2, 3, 4).reshape(5, -1),
                    w.transpose(1, 0, 2, 3, 4).reshape(5, -1)),
              FP64 if dtype == torch.float64 else (1e-5, 1e-4))


@pytest.mark.parametrize("dtype,n", [(torch.float64, 8), (torch.float32, 8),
                                     (torch.float32, 16)])
def test_nested_gather_equals_ghosted_copies(ctx, dtype, n):
    """The driver without ghosted copies (coarse-fine cells interpolated into
    stand-ins for the missing siblings, with the coarse level interpolated
    in time on the fly; the gathering flux-recording advance) gives the same
    bits as the driver that materialises every ghosted block, over two root
    steps, with no cell counted as non-physical."""
    note(f"nested driver, gathering vs ghosted copies, dtype={dtype}, blocks of {n}^3")
    states = _states(530, dtype == torch.float32)
    ref = amr.NestedDevice(ctx, NC, _refined(), dtype=dtype, n=n)
    got = amr.NestedDevice(ctx, NC, _refined(), dtype=dtype, n=n, gather=True)
    assert got.nsrc[1] > got.nb[1]
    blocks = [b.astype(np.float32) if dtype == torch.float32 else b
              for b in _blocks(ref.L, states)]
    for d in (ref, got):
        d.upload(blocks)
    ctx.tvd_read_flags()
    dt = 0.1 / NC
    for o in (0, 1):
        ref.step(dt, o)
        got.step(dt, o)
    torch.cuda.synchronize()
    assert ctx.tvd_read_flags()[2] == 0
    for a, b in zip(ref.download(), got.download()):
        assert np.array_equal(a, b)


def test_nested_streamed_levels_equal_per_block(ctx):
    """Patch groups with stand-ins: every level advanced by the streamed
    kernel with flux records (chains along z and x over each level's blocks)
    gives the same bits as the per-block gathering advance, over two root
    steps."""
    note("nested driver, streamed levels vs per-block advance, fp32 groups")
    states = _states(531, True)
    ref = amr.NestedDevice(ctx, NC, _refined(), dtype=torch.float32, n=16, gather=True)
    got = amr.NestedDevice(ctx, NC, _refined(), dtype=torch.float32, n=16, gather=True,
                           stream_min_blocks=1)
    assert all(c is not None for c in got.chains)
    blocks = [b.astype(np.float32) for b in _blocks(ref.L, states)]
    for d in (ref, got):
        d.upload(blocks)
    ctx.tvd_read_flags()
    dt = 0.1 / NC
    for o in (0, 1):
        ref.step(dt, o)
        got.step(dt, o)
    torch.cuda.synchronize()
    assert ctx.tvd_read_flags()[2] == 0
    for a, b in zip(ref.download(), got.download()):
        assert np.array_equal(a, b)
    with pytest.raises(ValueError):
        amr.NestedDevice(ctx, NC, _refined(), dtype=torch.float32, n=16, stream_min_blocks=1)


@pytest.mark.parametrize("dtype,n", [(torch.float64, 8), (torch.float32, 16)])
def test_nested_overlap_equals_sequential(ctx, dtype, n):
    """The gathering driver with every level on a stream of its own, a
    level's first sub-step overlapping its parent's advance, gives the same
    bits as the sequential driver over two root steps."""
    note(f"nested driver, overlapped levels vs sequential, dtype={dtype}, blocks of {n}^3")
    states = _states(532, dtype == torch.float32)
    ref = amr.NestedDevice(ctx, NC, _refined(), dtype=dtype, n=n, gather=True)
    got = amr.NestedDevice(ctx, NC, _refined(), dtype=dtype, n=n, gather=True, overlap=True)
    blocks = [b.astype(np.float32) if dtype == torch.float32 else b
              for b in _blocks(ref.L, states)]
    for d in (ref, got):
        d.upload(blocks)
    ctx.tvd_read_flags()
    dt = 0.1 / NC
    for o in (0, 1):
        ref.step(dt, o)
        got.step(dt, o)
    torch.cuda.synchronize()
    assert ctx.tvd_read_flags()[2] == 0
    for a, b in zip(ref.download(), got.download()):
        assert np.array_equal(a, b)
    with pytest.raises(ValueError):
        amr.NestedDevice(ctx, NC, _refined(), dtype=dtype, n=n, overlap=True)


@pytest.mark.skip(reason="capturing the overlapped driver's forks and joins across the levels' "
                         "streams crashed the host inside hipStreamEndCapture; the driver refuses "
                         "capture in overlap mode until the cause is known")
def test_nested_overlap_graph_replay(ctx):
    """Two root steps of the overlapped driver (fork and join across the
    levels' streams) recorded into one HIP graph and replayed three times,
    with eager steps in between, against eager overlapped steps: identical
    bits after every replay."""
    note("nested driver, overlapped levels, graph replay")
    states = _states(533, True)
    mk = lambda: amr.NestedDevice(ctx, NC, _refined(), dtype=torch.float32, n=16, gather=True,
                                  overlap=True)
    eager, graph = mk(), mk()
    blocks = [b.astype(np.float32) for b in _blocks(eager.L, states)]
    for d in (eager, graph):
        d.upload(blocks)
    torch.cuda.synchronize()
    dt = 0.1 / NC
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ctx.tvd_graph_begin(s)
        for o in (0, 1):
            graph.step(dt, o)
        g = ctx.tvd_graph_end(s)
    torch.cuda.synchronize()
    try:
        for rep in range(3):
            for o in (0, 1):
                eager.step(dt, o)
            g.replay(torch.cuda.current_stream())
            torch.cuda.synchronize()
            for a, b in zip(eager.download(), graph.download()):
                assert np.array_equal(a, b), rep
    finally:
        g.close()


def test_nested_driver_conserves_over_steps(ctx):
    states = _states(510, False)
    dev = amr.NestedDevice(ctx, NC, _refined(), dtype=torch.float64)
    L = dev.L
    dev.upload(_blocks(L, states))
    before = closing.nested_leaf_sums(states, L.refined)
    scale = closing.nested_leaf_sums([np.abs(s) for s in states], L.refined)
    for s in range(4):
        dev.step(0.1 / NC, s % 2)
    torch.cuda.synchronize()
    after = closing.nested_leaf_sums(_dense(L, dev.download()), L.refined)
    rel = np.max(np.abs(after - before) / scale)
    note(f"  4 root steps (32 level-2 steps): leaf total change / scale {rel:.1e}")
    assert rel <= 1e-13


def test_nested_step_graph_replay(ctx):
    """Two root steps recorded into a HIP graph through the library's native
    capture and replayed three times, with eager steps in between, against
    the eager steps: identical bits after every replay."""
    states = _states(520, False)
    eager = amr.NestedDevice(ctx, NC, _refined(), dtype=torch.float64)
    graph = amr.NestedDevice(ctx, NC, _refined(), dtype=torch.float64)
    for d in (eager, graph):
        d.upload(_blocks(eager.L, states))
    torch.cuda.synchronize()
    dt = 0.1 / NC
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ctx.tvd_graph_begin(s)
        for o in (0, 1):
            graph.step(dt, o)
        g = ctx.tvd_graph_end(s)
    torch.cuda.synchronize()
    try:
        for rep in range(3):
            for o in (0, 1):
                eager.step(dt, o)
            g.replay(torch.cuda.current_stream())
            torch.cuda.synchronize()
            for a, b in zip(eager.download(), graph.download()):
                assert np.array_equal(a, b), rep
    finally:
        g.close()


@pytest.mark.parametrize("n,gather,stream_min", [(8, False, None), (16, False, None),
                                                 (16, True, None), (16, True, 512)])
def test_nested_full_size_conserves_fp32(ctx, n, gather, stream_min):
    """The full multi-level hierarchy (128^3 base, levels 1-3, 18 152 patches,
    the bench's configuration, as patches or as 2269 patch groups, the
    larger levels of groups optionally by the streamed advance), FP32,
    every level sub-cycled: over four root steps (32 level-3 steps) the leaf
    totals drift by no more than the FP32 rounding of the stored state (1e-6
    of each variable's scale; momentum against mass times the signal speed,
    the gas starting at rest), and no cell is floored or non-physical."""
    from paper_0907_3390_amd import layout
    note(f"nested driver, full multi-level hierarchy, fp32, blocks of {n}^3, gather {gather}, "
         f"streamed levels from {stream_min} blocks")
    ml = wl.multilevel()
    refined = layout.NestedLevels.refined_from_patches(ml.base, ml.patches)
    dev = amr.NestedDevice(ctx, ml.base, refined, dtype=torch.float32, n=n, gather=gather,
                           stream_min_blocks=stream_min)
    L = dev.L
    interior = ml.ghosted[:, :, 3:11, 3:11, 3:11]
    per = [np.zeros((k, 5, n, n, n), dtype=np.float32) for k in dev.nb]
    # leaf mask per cell: a patch's cells are leaves unless the patch is refined
    leaf = [np.ones((k, 1, n, n, n), dtype=bool) for k in dev.nb]
    for i, (l, px, py, pz) in enumerate(ml.patches):
        b, (ox, oy, oz) = L.locate(l, px, py, pz)
        per[l][b, :, oz:oz + 8, oy:oy + 8, ox:ox + 8] = interior[i]
        if l < len(refined) and refined[l][pz, py, px]:
            leaf[l][b, :, oz:oz + 8, oy:oy + 8, ox:ox + 8] = False
    dev.upload(per)

    def sums(blocks, f=lambda a: a):
        return sum((f(blocks[l].astype(np.float64)) * leaf[l]).sum(axis=(0, 2, 3, 4)) * 8.0 ** -l
                   for l in range(len(blocks)))
    before, scale = sums(per), sums(per, np.abs)
    with pytest.raises(ValueError):
        amr.NestedDevice(ctx, ml.base, refined, dtype=torch.float64, n=16)
    c_max = float(np.sqrt(5.0 / 3.0 * ml.P0 / min(b[:, 0].min() for b in per)))
    scale[1:4] = scale[0] * c_max
    dt = 0.5 / ml.base / c_max
    ctx.tvd_read_flags()
    for s in range(4):
        dev.step(dt, s % 2)
    torch.cuda.synchronize()
    flags = ctx.tvd_read_flags()
    got = dev.download()
    drift = np.max(np.abs(sums(got) - before) / scale)
    note(f"  18 152 patches, 4 root steps: leaf total drift {drift:.1e}, flags {flags}")
    assert flags[1] == 0 and flags[2] == 0
    assert all(np.isfinite(b).all() for b in got)
    assert drift <= 1e-6
