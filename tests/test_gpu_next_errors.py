"""Error handling of the closing-step, Poisson and gravity entry points
through the C ABI: arguments the host can check are rejected before any
launch; rows the host cannot check (device tables) are checked by the
kernels, skipped, and counted as non-physical, leaving the other rows'
results as they would be without them."""
import numpy as np
import pytest
import torch

from gpu_helpers import GAMMA
from paper_0907_3390_amd import layout, tvd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    c = tvd.Context(0)
    yield c
    c.close()


def _status(fn):
    try:
        fn()
    except tvd.TvdError as e:
        return e.status
    return tvd.TVD_OK


def test_host_checked_arguments(ctx):
    d = torch.zeros(64 * 5 * 14 ** 3, dtype=torch.float64, device="cuda")
    o = torch.zeros(64 * 5 * 512, dtype=torch.float64, device="cuda")
    f = torch.zeros(64 * layout.flux_record_size(8), dtype=torch.float64, device="cuda")
    b = tvd.Batch(tvd.TVD_F64, 64, 8, dt=1e-3, dh=1.0 / 32)
    # the plain kernel records no fluxes
    assert _status(lambda: ctx.tvd_patch_advance_flux(b, d, o, f, None, 0, GAMMA,
                                                      flags=tvd.TVD_KERNEL_PLAIN)) == tvd.TVD_ERR_UNSUPPORTED
    # records over the state
    assert _status(lambda: ctx.tvd_patch_advance_flux(b, d, o, o, None, 0, GAMMA)) == tvd.TVD_ERR_ALIAS
    # SOR: omega outside (0, 2), no iterations, overlapping buffers
    phi = torch.zeros(2 * 18 ** 3, dtype=torch.float32, device="cuda")
    rho = torch.ones(2 * 4096, dtype=torch.float32, device="cuda")
    out = torch.zeros(2 * 4096, dtype=torch.float32, device="cuda")
    assert _status(lambda: ctx.tvd_poisson_sor(tvd.TVD_F32, 2, phi, rho, out, 1.0, 0.1,
                                               omega=2.5)) == tvd.TVD_ERR_INVALID_ARG
    assert _status(lambda: ctx.tvd_poisson_sor(tvd.TVD_F32, 2, phi, rho, out, 1.0, 0.1,
                                               max_iter=0)) == tvd.TVD_ERR_INVALID_ARG
    assert _status(lambda: ctx.tvd_poisson_sor(tvd.TVD_F32, 2, phi, rho, phi, 1.0, 0.1)) == tvd.TVD_ERR_ALIAS
    # gravity: mixed edges are not taken
    edges = torch.tensor([8, 16], dtype=torch.int32, device="cuda")
    offs = torch.zeros(2, dtype=torch.int64, device="cuda")
    bm = tvd.Batch(tvd.TVD_F32, 2, 0, d_edge=edges, d_in_off=offs, d_out_off=offs, dt=1.0, dh=1.0)
    assert _status(lambda: ctx.tvd_gravity(bm, out, phi)) == tvd.TVD_ERR_UNSUPPORTED


def test_bad_rows_are_skipped_and_counted(ctx):
    Nc, n = 32, 8
    ref = np.zeros((4, 4, 4), dtype=bool)
    ref[1, 1, 1] = True
    L = layout.RefinedLevels(Nc, ref, n)
    rr, fr, _ = L.tables()
    gr, gs = layout.group_face_rows(fr)
    r = np.random.default_rng(5)
    coarse = r.standard_normal(L.coarse.n_blocks * 5 * 512)
    fine = r.standard_normal(L.fine.n_blocks * 5 * 512)
    crec = r.standard_normal(L.coarse.n_blocks * layout.flux_record_size(8))
    frec = r.standard_normal(L.fine.n_blocks * layout.flux_record_size(8))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    cb = tvd.Batch(tvd.TVD_F64, L.coarse.n_blocks, 8, dt=1e-3, dh=1.0 / Nc)
    fb = tvd.Batch(tvd.TVD_F64, L.fine.n_blocks, 8, dt=1e-3, dh=0.5 / Nc)

    def close(rows_r, rows_f, start):
        u = dev(coarse)
        ctx.tvd_read_flags()
        ctx.tvd_close_level(cb, u, dev(crec), None, fb, dev(fine), dev(frec), None, dev(rows_r),
                            dev(rows_f), dev(start))
        torch.cuda.synchronize()
        return u.cpu().numpy(), ctx.tvd_read_flags()[2]

    good, bad0 = close(rr, gr, gs)
    assert bad0 == 0 and not np.array_equal(good, coarse)
    # a restriction row naming a fine block past the end: skipped and counted
    # once (its edge is unknown), the other rows unchanged
    rr_bad = np.concatenate([rr, [[L.fine.n_blocks + 3, 0, 0, 0, 0]]]).astype(np.int32)
    got, bad = close(rr_bad, gr, gs)
    assert bad == 1 and np.array_equal(got, good)
    # a restriction row whose coarse cells leave the block: its 4^3 cells counted
    rr_off = np.concatenate([rr, [[0, 0, 6, 0, 0]]]).astype(np.int32)
    got, bad = close(rr_off, gr, gs)
    assert bad == 64 and np.array_equal(got, good)
    # a face row whose offsets leave the coarse block: skipped and counted
    gr_bad = gr.copy()
    gr_bad[0, 4] = 7            # oa + 4 > 8
    got, bad = close(rr, gr_bad, gs)
    assert bad == 16
    # a group whose rows name two coarse blocks: skipped as a whole, once
    gr_mix = gr.copy()
    if gs[1] - gs[0] > 1:
        gr_mix[gs[0] + 1, 0] = (gr_mix[gs[0], 0] + 1) % L.coarse.n_blocks
        got, bad = close(rr, gr_mix, gs)
        assert bad == 1


def test_empty_inputs_are_no_ops(ctx):
    """Zero blocks, groups, elements or rows: every entry point returns OK
    and leaves its buffers as they were."""
    sentinel = lambda n, dt=torch.float32: torch.full((n,), 7.0, dtype=dt, device="cuda")
    u, o, f = sentinel(5 * 14 ** 3), sentinel(5 * 512), sentinel(layout.flux_record_size(8))
    b0 = tvd.Batch(tvd.TVD_F32, 0, 8, dt=1e-3, dh=1.0 / 32)
    ctx.tvd_patch_advance_flux(b0, u, o, f, None, 0, GAMMA)
    ctx.tvd_gravity(b0, o, u)
    a, c = sentinel(64), sentinel(64)
    ctx.tvd_lerp(tvd.TVD_F32, 0, a, a, c, 0.5)
    phi, rho, out = sentinel(18 ** 3), sentinel(4096), sentinel(4096)
    ctx.tvd_poisson_sor(tvd.TVD_F32, 0, phi, rho, out, 1.0, 0.1)
    b1 = tvd.Batch(tvd.TVD_F32, 1, 8, dt=1e-3, dh=1.0 / 32)
    uc = sentinel(5 * 512)
    ctx.tvd_restrict(b1, uc, b1, o, None)
    ctx.tvd_close_level(b1, uc, f, None, b1, o, f, None, None, None, None)
    ctx.tvd_flux_correct(b1, uc, f, None, b1, f, None, None, [0] * 6)
    torch.cuda.synchronize()
    for t in (u, o, f, a, c, phi, rho, out, uc):
        assert bool((t == 7.0).all())
