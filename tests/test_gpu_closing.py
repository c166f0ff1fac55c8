"""GPU parity of the closing step (Sec. 2.1 step 3; Sec. 3.1) through the C
ABI:

* the patch-boundary flux records of the flux-recording advance against the
  oracle's records (FP64 1e-12, FP32 1e-5 relative L1 per variable), for 8^3
  patches, 16^3 patch groups and a mixed batch, both sweep orders, batched
  and persistent kernels; neighbouring blocks' shared faces carry identical
  bits, and the advanced state is the one the plain advance produces;
* restriction and flux correction on seeded inputs against the oracle's, bit
  for bit (the same operations in the same order on both sides);
* a whole two-level step on the device (ghost fills, flux-recording advance
  of both levels, restriction, correction) against the oracle's two-level
  step (FP64, 1e-12), conserving the leaf totals;
* the full multi-level hierarchy: the leaf totals are conserved through a
  step closed level pair by level pair, finest first, and after restriction
  the root level's total equals the leaf total.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import closing
from gpu_helpers import FP64, GAMMA, check, norms, note
from paper_0907_3390_amd import layout, tvd, workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    c = tvd.Context(0)
    yield c
    c.close()


def _rel_l1(got, want):
    """Worst over the five variables of sum |got - want| / sum |want|, records
    given as lists of arrays (3, NQ, 5, n, n)."""
    worst = 0.0
    for k in range(5):
        d = sum(float(np.abs(g[:, :, k] - w[:, :, k]).sum()) for g, w in zip(got, want))
        s = sum(float(np.abs(w[:, :, k]).sum()) for w in want)
        worst = max(worst, d / s)
    return worst


def _rel_linf(got, want):
    """Worst over the five variables of max |got - want| / max |want|."""
    worst = 0.0
    for k in range(5):
        d = max(float(np.abs(g[:, :, k] - w[:, :, k]).max()) for g, w in zip(got, want))
        s = max(float(np.abs(w[:, :, k]).max()) for w in want)
        worst = max(worst, d / s)
    return worst


def _records(flat, edges, offs):
    return [flat[o:o + layout.flux_record_size(int(e))].reshape(3, int(e) // 8 + 1, 5, int(e), int(e))
            for e, o in zip(edges, offs)]


def _advance_flux(ctx, dtype, ghosted_list, edges, order, flags, dt, dh):
    """Flux-recording advance of a list of ghosted blocks (host FP64 arrays);
    returns (interiors, records) as FP64 numpy lists."""
    code = tvd.dtype_code(dtype)
    edges = np.asarray(edges, dtype=np.int32)
    bs = layout.BlockSet(edges, np.full(len(edges), dh), np.zeros((len(edges), 27), np.int32))
    u_in = torch.from_numpy(np.concatenate([g.ravel() for g in ghosted_list])).to(dtype).cuda()
    u_out = torch.zeros(bs.out_total, dtype=dtype, device="cuda")
    foff = layout.flux_offsets(edges)
    nflux = int(foff[-1] + layout.flux_record_size(int(edges[-1])))
    flux = torch.full((nflux,), float("nan"), dtype=dtype, device="cuda")
    uniform = bs.uniform_edge
    if uniform:
        b = tvd.Batch(code, bs.n_blocks, uniform, dt=dt, dh=dh)
        d_foff = None
    else:
        d_edge = torch.from_numpy(edges).cuda()
        d_in = torch.from_numpy(bs.in_off).cuda()
        d_out = torch.from_numpy(bs.out_off).cuda()
        b = tvd.Batch(code, bs.n_blocks, 0, d_edge=d_edge, d_in_off=d_in, d_out_off=d_out,
                      dt=dt, dh=dh)
        d_foff = torch.from_numpy(foff).cuda()
    ctx.tvd_reserve(bs.n_blocks)
    ctx.tvd_read_flags()
    ctx.tvd_patch_advance_flux(b, u_in, u_out, flux, d_foff, order, GAMMA, flags=flags)
    torch.cuda.synchronize()
    fl, bad = ctx.tvd_read_flags()[1:]
    assert bad == 0
    outs = bs.unpack_interior(u_out.double().cpu().numpy())
    recs = _records(flux.double().cpu().numpy(), edges, foff)
    # the state is the one the advance without records produces
    u_ref = torch.zeros_like(u_out)
    ctx.tvd_patch_advance(b, u_in, u_ref, order, GAMMA, flags=flags)
    torch.cuda.synchronize()
    assert torch.equal(u_ref, u_out)
    return outs, recs


@pytest.mark.parametrize("dtype,n,flags", [
    (torch.float64, 8, tvd.TVD_KERNEL_BATCHED),
    (torch.float32, 8, tvd.TVD_KERNEL_BATCHED),
    (torch.float32, 16, tvd.TVD_KERNEL_BATCHED),
    (torch.float32, 8, tvd.TVD_KERNEL_PERSISTENT),
    (torch.float32, 16, tvd.TVD_KERNEL_PERSISTENT),
])
@pytest.mark.parametrize("order", [0, 1])
def test_flux_records_match_oracle(ctx, dtype, n, flags, order):
    note(f"flux records dtype={dtype} n={n} flags={flags} order={order}")
    N = 32
    g = wl.lognormal(N, seed=50 + n + order, sigma_ln=0.6)
    if dtype == torch.float32:
        g = g.astype(np.float32).astype(np.float64)
    blocks = oracle.periodic_ghosted_blocks(g, n)
    dt, dh = 0.2 / N, 1.0 / N
    want_out, want_rec = oracle.advance_ragged(list(blocks), order, dt, dh, GAMMA, fluxes=True)
    got_out, got_rec = _advance_flux(ctx, dtype, list(blocks), [n] * len(blocks), order, flags, dt, dh)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    err = _rel_l1(got_rec, want_rec)
    einf = _rel_linf(got_rec, want_rec)
    note(f"  record relL1 {err:.2e}, relLinf {einf:.2e}")
    assert err <= tol
    assert einf <= (1e-12 if dtype == torch.float64 else 1e-4)
    assert not any(np.isnan(r).any() for r in got_rec)
    # neighbouring blocks report the same bits on the face they share
    nb = N // n
    for b, rec in enumerate(got_rec):
        c = [b % nb, (b // nb) % nb, b // (nb * nb)]
        for d in range(3):
            cn = list(c)
            cn[d] = (c[d] + 1) % nb
            assert np.array_equal(rec[d, -1], got_rec[cn[0] + nb * (cn[1] + nb * cn[2])][d, 0])


def test_flux_records_mixed_edges_persistent(ctx):
    """A batch of periodic boxes cut into 16^3 groups and 8^3 patches, with
    record offsets, in one persistent launch."""
    note("flux records, mixed edges, persistent")
    grids = [wl.lognormal(32, seed=61, sigma_ln=0.5), wl.lognormal(16, seed=62, sigma_ln=0.5),
             wl.lognormal(16, seed=63, sigma_ln=0.5)]
    edge_for = lambda L: 16 if L >= 32 else 8
    blocks, edges = [], []
    for gr in grids:
        gr32 = gr.astype(np.float32).astype(np.float64)
        e = edge_for(gr.shape[1])
        bl = oracle.periodic_ghosted_blocks(gr32, e)
        blocks += list(bl)
        edges += [e] * len(bl)
    dt, dh = 0.1 / 32, 1.0 / 32
    want_out, want_rec = oracle.advance_ragged(blocks, 1, dt, dh, GAMMA, fluxes=True)
    got_out, got_rec = _advance_flux(ctx, torch.float32, blocks, edges, 1,
                                     tvd.TVD_KERNEL_PERSISTENT, dt, dh)
    err = _rel_l1(got_rec, want_rec)
    einf = _rel_linf(got_rec, want_rec)
    note(f"  record relL1 {err:.2e}, relLinf {einf:.2e}")
    assert err <= 1e-5
    assert einf <= 1e-4


def _refined():
    r = np.zeros((4, 4, 4), dtype=bool)
    r[1, 1, 1] = r[1, 1, 2] = r[1, 2, 1] = True
    r[3, 0, 3] = True
    return r


def _fine_grid(L, blocks, Nc):
    """Fine interior blocks in RefinedLevels order -> (5, 2Nc, 2Nc, 2Nc) grid
    (zero outside refined patches)."""
    n = L.n
    out = np.zeros((5, 2 * Nc, 2 * Nc, 2 * Nc), dtype=blocks[0].dtype)
    for blk, (oz, oy, ox) in zip(blocks, L.origins):
        out[:, oz:oz + n, oy:oy + n, ox:ox + n] = blk
    return out


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n", [8, 16])
def test_restrict_bitwise(ctx, dtype, n):
    note(f"restriction dtype={dtype} n={n}")
    Nc = 32
    L = layout.RefinedLevels(Nc, _refined(), n)
    npd = np.float64 if dtype == torch.float64 else np.float32
    r = wl.rng(70 + n)
    coarse = r.lognormal(size=(5, Nc, Nc, Nc)).astype(npd)
    fine_blocks = r.lognormal(size=(L.fine.n_blocks, 5, n, n, n)).astype(npd)
    rr, _, _ = L.tables()
    code = tvd.dtype_code(dtype)
    c_dev = torch.from_numpy(layout.grid_to_blocks(coarse, 8)).cuda().reshape(-1)
    f_dev = torch.from_numpy(fine_blocks).cuda().reshape(-1)
    cb = tvd.Batch(code, L.coarse.n_blocks, 8, dt=1e-3, dh=1.0 / Nc)
    fb = tvd.Batch(code, L.fine.n_blocks, n, dt=1e-3, dh=0.5 / Nc)
    ctx.tvd_read_flags()
    ctx.tvd_restrict(cb, c_dev, fb, f_dev, torch.from_numpy(rr).cuda())
    torch.cuda.synchronize()
    assert ctx.tvd_read_flags()[2] == 0
    got = layout.blocks_to_grid(c_dev.cpu().numpy().reshape(-1, 5, 8, 8, 8), coarse.shape)
    want = coarse.copy()
    fine = _fine_grid(L, fine_blocks, Nc)
    for pz, py, px in np.argwhere(L.refined):
        want[:, 8 * pz:8 * pz + 8, 8 * py:8 * py + 8, 8 * px:8 * px + 8] = closing.restrict(
            fine[:, 16 * pz:16 * pz + 16, 16 * py:16 * py + 16, 16 * px:16 * px + 16])
    assert np.array_equal(got, want)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n", [8, 16])
def test_flux_correct_bitwise(ctx, dtype, n):
    note(f"flux correction dtype={dtype} n={n}")
    Nc = 32
    L = layout.RefinedLevels(Nc, _refined(), n)
    npd = np.float64 if dtype == torch.float64 else np.float32
    r = wl.rng(80 + n)
    coarse = r.lognormal(size=(5, Nc, Nc, Nc)).astype(npd)
    crec = r.standard_normal((L.coarse.n_blocks,) + (3, 2, 5, 8, 8)).astype(npd)
    frec = r.standard_normal((L.fine.n_blocks, 3, n // 8 + 1, 5, n, n)).astype(npd)
    _, fr, count = L.tables()
    dt, dh = 3e-3, 1.0 / Nc
    code = tvd.dtype_code(dtype)
    c_dev = torch.from_numpy(layout.grid_to_blocks(coarse, 8)).cuda().reshape(-1)
    cb = tvd.Batch(code, L.coarse.n_blocks, 8, dt=dt, dh=dh)
    fb = tvd.Batch(code, L.fine.n_blocks, n, dt=dt, dh=0.5 / Nc)
    ctx.tvd_read_flags()
    ctx.tvd_flux_correct(cb, c_dev, torch.from_numpy(crec).cuda().reshape(-1), None, fb,
                         torch.from_numpy(frec).cuda().reshape(-1), None,
                         torch.from_numpy(fr).cuda(), count)
    torch.cuda.synchronize()
    assert ctx.tvd_read_flags()[2] == 0
    got = layout.blocks_to_grid(c_dev.cpu().numpy().reshape(-1, 5, 8, 8, 8), coarse.shape)
    P = Nc // 8
    faces = closing.fine_face_fluxes(list(frec), L.refined, n, 2 * Nc)
    want = closing.flux_correct(coarse, L.refined, crec.reshape(P, P, P, 3, 2, 5, 8, 8), faces,
                                dt / dh)
    assert np.array_equal(got, want)
    assert not np.array_equal(got, coarse)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n", [8, 16])
def test_close_level_matches_separate_calls(ctx, dtype, n):
    """The one-launch closing of a level pair gives the bits of restriction
    followed by the six correction passes (seeded states and records)."""
    note(f"one-launch closing dtype={dtype} n={n}")
    Nc = 32
    L = layout.RefinedLevels(Nc, _refined(), n)
    npd = np.float64 if dtype == torch.float64 else np.float32
    r = wl.rng(95 + n)
    coarse = layout.grid_to_blocks(r.lognormal(size=(5, Nc, Nc, Nc)).astype(npd), 8)
    fine = r.lognormal(size=(L.fine.n_blocks, 5, n, n, n)).astype(npd)
    crec = r.standard_normal((L.coarse.n_blocks, layout.flux_record_size(8))).astype(npd)
    frec = r.standard_normal((L.fine.n_blocks, layout.flux_record_size(n))).astype(npd)
    rr, fr, count = L.tables()
    gr, gs = layout.group_face_rows(fr)
    code = tvd.dtype_code(dtype)
    cb = tvd.Batch(code, L.coarse.n_blocks, 8, dt=2e-3, dh=1.0 / Nc)
    fb = tvd.Batch(code, L.fine.n_blocks, n, dt=2e-3, dh=0.5 / Nc)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    f_dev, c_rec, f_rec = dev(fine).reshape(-1), dev(crec).reshape(-1), dev(frec).reshape(-1)
    a = dev(coarse).reshape(-1)
    b = a.clone()
    ctx.tvd_read_flags()
    ctx.tvd_restrict(cb, a, fb, f_dev, dev(rr))
    ctx.tvd_flux_correct(cb, a, c_rec, None, fb, f_rec, None, dev(fr), count)
    ctx.tvd_close_level(cb, b, c_rec, None, fb, f_dev, f_rec, None, dev(rr), dev(gr), dev(gs))
    torch.cuda.synchronize()
    assert ctx.tvd_read_flags()[2] == 0
    assert torch.equal(a, b)
    assert not torch.equal(b, dev(coarse).reshape(-1))


def _device_two_level_step(ctx, L, coarse, fine_blocks, dt, order, dtype):
    """The two-level step on the device: periodic sibling ghost fill of the
    coarse patches, coarse-fine ghost fill of the fine blocks (from the coarse
    level at the old time), flux-recording advance of both, restriction,
    flux correction.  Returns (coarse grid, fine blocks)."""
    Nc, n = L.Nc, L.n
    code = tvd.dtype_code(dtype)
    nc, nf = L.coarse.n_blocks, L.fine.n_blocks
    c_int = torch.from_numpy(layout.grid_to_blocks(coarse, 8)).to(dtype).cuda().reshape(-1)
    f_int = torch.from_numpy(np.ascontiguousarray(fine_blocks)).to(dtype).cuda().reshape(-1)
    c_gh = torch.zeros(nc * 5 * 14 ** 3, dtype=dtype, device="cuda")
    f_gh = torch.zeros(nf * 5 * (n + 6) ** 3, dtype=dtype, device="cuda")
    c_out = torch.zeros(nc * 5 * 512, dtype=dtype, device="cuda")
    f_out = torch.zeros(nf * 5 * n ** 3, dtype=dtype, device="cuda")
    c_flux = torch.zeros(nc * layout.flux_record_size(8), dtype=dtype, device="cuda")
    f_flux = torch.zeros(nf * layout.flux_record_size(n), dtype=dtype, device="cuda")
    cb = tvd.Batch(code, nc, 8, dt=dt, dh=1.0 / Nc)
    fb = tvd.Batch(code, nf, n, dt=dt, dh=0.5 / Nc)
    c_nbr = torch.from_numpy(L.coarse.nbr).cuda()
    f_nbr = torch.from_numpy(L.fine.nbr).cuda()
    rr, fr, count = L.tables()
    ctx.tvd_read_flags()
    ctx.tvd_fill_ghosts(cb, c_nbr, c_int, c_gh)
    ctx.tvd_fill_ghosts_amr(fb, f_nbr, f_int, f_gh, cb, c_int, torch.from_numpy(L.cnbr).cuda(),
                            torch.from_numpy(L.corigin).cuda())
    ctx.tvd_patch_advance_flux(cb, c_gh, c_out, c_flux, None, order, GAMMA)
    ctx.tvd_patch_advance_flux(fb, f_gh, f_out, f_flux, None, order, GAMMA)
    ctx.tvd_restrict(cb, c_out, fb, f_out, torch.from_numpy(rr).cuda())
    ctx.tvd_flux_correct(cb, c_out, c_flux, None, fb, f_flux, None, torch.from_numpy(fr).cuda(),
                         count)
    torch.cuda.synchronize()
    assert ctx.tvd_read_flags()[2] == 0
    cg = layout.blocks_to_grid(c_out.double().cpu().numpy().reshape(-1, 5, 8, 8, 8),
                               (5, Nc, Nc, Nc))
    return cg, f_out.double().cpu().numpy().reshape(nf, 5, n, n, n)


@pytest.mark.parametrize("dtype,n", [(torch.float64, 8), (torch.float32, 8),
                                     (torch.float32, 16)])
@pytest.mark.parametrize("order", [0, 1])
def test_two_level_step(ctx, dtype, n, order):
    """FP64 (8^3 patches; FP64 groups do not fit the LDS) within 1e-12 of the
    oracle, FP32 within 1e-5 of the oracle run on the FP32-rounded start; the
    leaf totals are conserved to round-off (FP32: to its last bits)."""
    note(f"two-level step dtype={dtype} n={n} order={order}")
    Nc = 32
    L = layout.RefinedLevels(Nc, _refined(), n)
    coarse = wl.lognormal(Nc, seed=90 + n + order, sigma_ln=0.5)
    fine = wl.lognormal(2 * Nc, seed=91 + n + order, sigma_ln=0.5)
    if dtype == torch.float32:
        coarse = coarse.astype(np.float32).astype(np.float64)
        fine = fine.astype(np.float32).astype(np.float64)
    fine_blocks = np.stack([fine[:, oz:oz + n, oy:oy + n, ox:ox + n] for oz, oy, ox in L.origins])
    dt = 0.2 / (2 * Nc) / 4.0
    cg, fblk = _device_two_level_step(ctx, L, coarse, fine_blocks, dt, order, dtype)
    want_c, want_f = closing.two_level_step(coarse, fine, L.refined, n, dt, order, GAMMA)
    fg = _fine_grid(L, list(fblk), Nc)
    err_c = np.abs(cg - want_c).sum() / np.abs(want_c).sum()
    mask = np.repeat(np.repeat(np.repeat(L.refined, 16, 0), 16, 1), 16, 2)
    err_f = np.abs(fg[:, mask] - want_f[:, mask]).sum() / np.abs(want_f[:, mask]).sum()
    note(f"  coarse relL1 {err_c:.2e}, fine relL1 {err_f:.2e}")
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert err_c <= tol and err_f <= tol
    bounds = FP64 if dtype == torch.float64 else (1e-5, 1e-4)
    check(norms(cg, want_c), bounds)
    check(norms(fg[:, mask], want_f[:, mask]), bounds)
    before = closing.leaf_sums(coarse, fine, L.refined)
    after = closing.leaf_sums(cg, fg, L.refined)
    scale = closing.leaf_sums(np.abs(coarse), np.abs(fine), L.refined)
    rel = np.max(np.abs(after - before) / scale)
    note(f"  leaf total change / scale {rel:.1e}")
    assert rel <= (1e-13 if dtype == torch.float64 else 2e-7)


def _hierarchy_sums(ml, blocks, n, leaf_only):
    """Sums of the five variables times dh^3 over the interiors of the
    hierarchy's patches: the leaves only, or (leaf_only False) per level."""
    present = set(ml.patches)
    per_level = {}
    for i, (lev, px, py, pz) in enumerate(ml.patches):
        refined = (lev + 1, 2 * px, 2 * py, 2 * pz) in present
        if leaf_only and refined:
            continue
        key = 0 if leaf_only else lev
        per_level.setdefault(key, []).append(i)
    out = {}
    for key, ids in per_level.items():
        vol = ml.dh[ids] ** 3
        sel = blocks[ids].reshape(len(ids), 5, -1).sum(axis=2)
        out[key] = np.array([math.fsum((sel[:, k] * vol).tolist()) for k in range(5)])
    return out[0] if leaf_only else out


@pytest.fixture(scope="module")
def hierarchy():
    return wl.multilevel()


@pytest.mark.parametrize("mode", ["fp64_patches", "fp32_groups"])
def test_multilevel_closing_conserves_full_size(ctx, hierarchy, mode):
    """The full multi-level hierarchy (128^3 base, levels 0-3) in one
    flux-recording launch with one dt on every level (FP64 8^3 patches,
    batched; FP32 2^3 patch groups, persistent), then restriction and flux
    correction level pair by level pair, finest first (one launch per pair):
    the leaf totals are conserved to round-off (FP32: to its last bits), and
    the root level's total equals the leaf total after restriction.  Without
    the closing step the totals drift by orders of magnitude more."""
    note(f"multi-level closing, full size, {mode}")
    ml = hierarchy
    if mode == "fp64_patches":
        dtype, edge, kernel = torch.float64, 8, tvd.TVD_KERNEL_BATCHED
        ghosted, dhs = ml.ghosted, ml.dh
        blocks_of = lambda a: a                                  # patches are the blocks
    else:
        dtype, edge, kernel = torch.float32, 16, tvd.TVD_KERNEL_PERSISTENT
        groups, ghosted, dhs = ml.group_blocks()
        gidx = {g: i for i, g in enumerate(groups)}

        def blocks_of(a):                                        # groups -> patches
            out = np.empty((len(ml.patches), 5, 8, 8, 8), dtype=a.dtype)
            for i, (lev, px, py, pz) in enumerate(ml.patches):
                g = a[gidx[(lev, px // 2, py // 2, pz // 2)]]
                out[i] = g[:, 8 * (pz & 1):8 * (pz & 1) + 8, 8 * (py & 1):8 * (py & 1) + 8,
                           8 * (px & 1):8 * (px & 1) + 8]
            return out
    nb = len(dhs)
    note(f"  {nb} blocks of {edge}^3, patches per level {np.bincount(ml.levels).tolist()}")
    tabs = ml.closing(edge)
    code = tvd.dtype_code(dtype)
    u_in = torch.from_numpy(np.ascontiguousarray(ghosted)).to(dtype).cuda().reshape(-1)
    interior = np.ascontiguousarray(ghosted[:, :, 3:-3, 3:-3, 3:-3])
    if dtype == torch.float32:
        interior = interior.astype(np.float32).astype(np.float64)
    S = oracle.max_signal_speed(np.ascontiguousarray(interior.transpose(1, 0, 2, 3, 4)), GAMMA)
    dt = 0.5 * float(np.min(dhs)) / S
    d_dh = torch.from_numpy(np.ascontiguousarray(dhs)).cuda()
    b = tvd.Batch(code, nb, edge, dt=dt, d_dh=d_dh)
    u_out = torch.zeros(nb * 5 * edge ** 3, dtype=dtype, device="cuda")
    flux = torch.zeros(nb * layout.flux_record_size(edge), dtype=dtype, device="cuda")
    ctx.tvd_reserve(nb)
    ctx.tvd_read_flags()
    ctx.tvd_patch_advance_flux(b, u_in, u_out, flux, None, 0, GAMMA, flags=kernel)
    torch.cuda.synchronize()
    raw = u_out.double().cpu().numpy().reshape(nb, 5, edge, edge, edge)
    dev = lambda a: torch.from_numpy(a).cuda()
    for lev in sorted(tabs, reverse=True):
        rr, fr, count = tabs[lev]
        gr, gs = layout.group_face_rows(fr)
        ctx.tvd_close_level(b, u_out, flux, None, b, u_out, flux, None, dev(rr), dev(gr), dev(gs))
    torch.cuda.synchronize()
    assert ctx.tvd_read_flags()[2] == 0
    got = u_out.double().cpu().numpy().reshape(nb, 5, edge, edge, edge)
    P_in, P_raw, P_got = blocks_of(interior), blocks_of(raw), blocks_of(got)
    before = _hierarchy_sums(ml, P_in, 8, True)
    scale = _hierarchy_sums(ml, np.abs(P_in), 8, True)
    # the gas starts at rest: momentum is measured against total mass times
    # the signal speed
    scale[1:4] = scale[0] * S
    after = _hierarchy_sums(ml, P_got, 8, True)
    leak = _hierarchy_sums(ml, P_raw, 8, True)
    rel = np.abs(after - before) / scale
    rel_raw = np.abs(leak - before) / scale
    note(f"  leaf total change / scale {rel.max():.1e} (without the closing step {rel_raw.max():.1e})")
    tol = 1e-12 if dtype == torch.float64 else 1e-6
    assert np.all(rel <= tol)
    assert rel_raw[0] > (1e3 if dtype == torch.float64 else 10.0) * max(rel[0], 1e-16)
    # the root level covers the whole box: after restriction its total is
    # the leaf total
    root = _hierarchy_sums(ml, P_got, 8, False)[0]
    assert np.all(np.abs(root - after) <= tol * scale)


@pytest.mark.parametrize("dtype,n", [(torch.float64, 8), (torch.float32, 8), (torch.float32, 16)])
@pytest.mark.parametrize("order", [0, 1])
def test_flux_records_gathering_advance(ctx, dtype, n, order):
    """tvd_patch_advance_flux_gather (ghost zones read from the neighbours'
    interiors, one source-only block appended) gives the same state and the
    same flux records, bit for bit, as tvd_patch_advance_flux on the
    ghosted copies, in writing and in accumulating mode."""
    note(f"gathering flux-recording advance dtype={dtype} n={n} order={order}")
    N = 32
    g = wl.lognormal(N, seed=70 + n + order, sigma_ln=0.6)
    if dtype == torch.float32:
        g = g.astype(np.float32).astype(np.float64)
    bs = layout.periodic_grid_blockset(N, n)
    nb, code = bs.n_blocks, tvd.dtype_code(dtype)
    batch = tvd.Batch(code, nb, n, dt=0.2 / N, dh=1.0 / N)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    interior = dev(bs.pack_interior(layout.grid_to_blocks(g, n))).to(dtype)
    # one extra source-only block (never named by the table): the source count
    # may exceed n_blocks
    src = torch.cat([interior, torch.full((5 * n ** 3,), float("nan"), dtype=dtype,
                                          device="cuda")])
    ghosted = torch.zeros(bs.in_total, dtype=dtype, device="cuda")
    ctx.tvd_fill_ghosts(batch, dev(bs.nbr), interior, ghosted)
    rs = layout.flux_record_size(n)
    for acc in (0, 1):
        out_a = torch.zeros(bs.out_total, dtype=dtype, device="cuda")
        out_b = torch.zeros_like(out_a)
        rec_a = torch.ones(nb * rs, dtype=dtype, device="cuda")
        rec_b = torch.ones_like(rec_a)
        ctx.tvd_patch_advance_flux(batch, ghosted, out_a, rec_a, None, order, GAMMA,
                                   flux_weight=0.5, accumulate=acc)
        ctx.tvd_patch_advance_flux_gather(batch, dev(bs.nbr), nb + 1, src, out_b, rec_b, None,
                                          order, GAMMA, flux_weight=0.5, accumulate=acc)
        torch.cuda.synchronize()
        assert torch.equal(out_a, out_b)
        assert torch.equal(rec_a, rec_b)
        assert torch.isfinite(rec_b).all()
