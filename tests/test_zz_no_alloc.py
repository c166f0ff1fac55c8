"""The allocation-free streamed advance (tvd_patch_advance_stream_noalloc)
against tvd_patch_advance_stream, through the C ABI.

The two entry points run the same kernels; only the home of the per-tile
partials of the fused signal speed and sums differs (the library's static
scratch array instead of the context's workspace).  Two calls in a row, the
second on a smaller batch, must give the same state bits and the same FP64
speed and sums as the workspace entry point, which shows that each call
clears what the previous one left in the shared array.  A batch beyond the
array's limit is refused before anything is launched.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import GAMMA, note
from paper_0907_3390_amd import layout, tvd, workloads as wl

pytestmark = pytest.mark.gpu

SCRATCH_PARTS = 65536


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    c = tvd.Context(0)
    yield c
    c.close()


def problem(N, n, seed, dtype):
    """A periodic N^3 lognormal state as Morton-ordered blocks of edge n,
    with its neighbour table and chains along z (forward step) and x."""
    bs = layout.periodic_grid_blockset(N, n, curve="morton")
    g = wl.lognormal(N, seed=seed, sigma_ln=0.6)
    blocks = layout.grid_to_blocks(g, n, bs.perm)
    dev = torch.device("cuda:0")
    u = torch.from_numpy(bs.pack_interior(blocks)).to(dtype=dtype, device=dev)
    nbr = torch.from_numpy(bs.nbr).to(dev)
    chains = {}
    for order, axis in ((tvd.TVD_XYZ, 2), (tvd.TVD_ZYX, 0)):
        st, bl = layout.stream_chains(bs.nbr, axis, 2)
        chains[order] = tvd.Chains(torch.from_numpy(st).to(dev), torch.from_numpy(bl).to(dev))
    code = tvd.dtype_code(dtype)
    batch = tvd.Batch(code, bs.n_blocks, n, dt=0.2 / N, dh=1.0 / N)
    return batch, nbr, chains, u


def both(ctx, batch, nbr, chains, u, order, p_floor=0.0):
    """One step through each entry point from the same input; returns
    (state, smax, sums) of the workspace call and of the no-alloc call."""
    ctx.tvd_reserve(batch.c.n_blocks * (batch.c.edge // 16) ** 2)
    res = []
    for name in ("tvd_patch_advance_stream", "tvd_patch_advance_stream_noalloc"):
        out = torch.full_like(u, float("nan"))
        smax = torch.full((1,), float("nan"), dtype=torch.float64, device=u.device)
        sums = torch.full((5,), float("nan"), dtype=torch.float64, device=u.device)
        getattr(ctx, name)(batch, nbr, chains[order], u, out, order, GAMMA, p_floor,
                           smax=smax, sums=sums)
        torch.cuda.synchronize()
        res.append((out.cpu(), smax.cpu(), sums.cpu()))
    return res


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_equals_workspace_entry_point(ctx, dtype):
    """Two calls in a row, a 64^3 grid (8 blocks of edge 32, four tiles
    each: 32 partials) then a 32^3 grid (8 blocks of edge 16: 8 partials),
    each against the workspace entry point: identical state, signal speed
    and sums, bit for bit."""
    cases = [(64, 32, 31, tvd.TVD_XYZ), (32, 16, 32, tvd.TVD_ZYX)]
    for N, n, seed, order in cases:
        note(f"noalloc vs workspace: {dtype} {N}^3 edge {n} order {order}")
        batch, nbr, chains, u = problem(N, n, seed, dtype)
        (a, sa, ma), (b, sb, mb) = both(ctx, batch, nbr, chains, u, order)
        assert torch.isfinite(a).all()
        assert torch.equal(a, b)
        assert torch.equal(sa, sb) and torch.isfinite(sa).all()
        assert torch.equal(ma, mb) and torch.isfinite(ma).all()


def test_noalloc_second_smaller_call_clears_partials(ctx):
    """A large call (4096 partials) then a small one (8 partials): each
    equals the workspace call, and the small call's fused speed and sums are
    those of its own output (recomputed by tvd_max_signal_speed and
    tvd_conservation_sums), not partly the large call's leftover partials."""
    note("noalloc: large call, then small call")
    big = problem(256, 16, 33, torch.float32)
    small = problem(32, 16, 34, torch.float32)
    (a, sa, ma), (b, sb, mb) = both(ctx, *big, tvd.TVD_XYZ)
    assert torch.equal(a, b) and torch.equal(sa, sb) and torch.equal(ma, mb)
    batch, nbr, chains, u = small
    (a, sa, ma), (b, sb, mb) = both(ctx, batch, nbr, chains, u, tvd.TVD_XYZ)
    assert torch.equal(a, b) and torch.equal(sa, sb) and torch.equal(ma, mb)
    out = b.cuda()
    s_ref = torch.zeros(1, dtype=torch.float64, device="cuda")
    m_ref = torch.zeros(5, dtype=torch.float64, device="cuda")
    ctx.tvd_max_signal_speed(batch, out, tvd.TVD_LAYOUT_INTERIOR, GAMMA, s_ref)
    ctx.tvd_conservation_sums(batch, out, tvd.TVD_LAYOUT_INTERIOR, m_ref)
    torch.cuda.synchronize()
    s_ref, m_ref = s_ref.cpu().numpy(), m_ref.cpu().numpy()
    assert float(sb[0]) == float(s_ref[0])
    # the same cells summed in another fixed order: round-off of the
    # compensated FP64 sums only (a leftover partial of the large call would
    # add a whole block's mass, about 1/4096 of the total)
    scale = np.abs(m_ref) + abs(m_ref[0])
    assert np.all(np.abs(mb.numpy() - m_ref) <= 1e-13 * scale)


def test_noalloc_refuses_more_partials_than_the_array_holds(ctx):
    """chains * tiles above 65536 with fused diagnostics (one partial per
    chain and tile): TVD_ERR_STATE, nothing launched; without diagnostics no
    partial is used and the limit does not apply (checked on an empty chain
    list, which launches nothing)."""
    dev = torch.device("cuda:0")
    # offset tables (never read: nothing is launched) so that the dense-layout
    # overlap check, which would see two small buffers as overlapping
    # block-sized ranges, does not answer first
    off = torch.zeros(1, dtype=torch.int64, device=dev)
    n = SCRATCH_PARTS + 1
    batch = tvd.Batch(tvd.TVD_F32, n, 16, dt=1e-3, dh=1e-2, d_in_off=off, d_out_off=off)

    def many_chains(n):  # n one-block chains (never read: nothing is launched)
        start = torch.arange(n + 1, dtype=torch.int32, device=dev)
        return tvd.Chains(start, torch.zeros(n, dtype=torch.int32, device=dev))

    nbr = torch.zeros(27, dtype=torch.int32, device=dev)
    u = torch.zeros(16, dtype=torch.float32, device=dev)
    v = torch.zeros(16, dtype=torch.float32, device=dev)
    sums = torch.zeros(5, dtype=torch.float64, device=dev)
    st = ctx.tvd_patch_advance_stream_noalloc(batch, nbr, many_chains(n), u, v,
                                              tvd.TVD_XYZ, GAMMA, sums=sums, check=False)
    assert st == tvd.TVD_ERR_STATE
    assert "scratch" in ctx.last_error()
    members = torch.zeros(1, dtype=torch.int32, device=dev)
    empty = tvd.Chains(torch.zeros(1, dtype=torch.int32, device=dev), members)
    st = ctx.tvd_patch_advance_stream_noalloc(batch, nbr, empty, u, v, tvd.TVD_XYZ, GAMMA,
                                              check=False)
    assert st == tvd.TVD_OK
    # edge 32: four tiles per chain count against the limit
    n32 = SCRATCH_PARTS // 4 + 1
    b32 = tvd.Batch(tvd.TVD_F32, n32, 32, dt=1e-3, dh=1e-2, d_in_off=off, d_out_off=off)
    st = ctx.tvd_patch_advance_stream_noalloc(b32, nbr, many_chains(n32), u, v,
                                              tvd.TVD_XYZ, GAMMA, sums=sums, check=False)
    assert st == tvd.TVD_ERR_STATE
    torch.cuda.synchronize()
