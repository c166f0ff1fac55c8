"""The two-level step driven on the device (paper_0907_3390_amd.amr), with one
dt on both levels and with the fine level sub-cycled in two steps of dt/2
(weighted flux records, coarse ghost data interpolated in time), against the
oracle's two-level steps: FP64 within 1e-12, FP32 within 1e-5 of the oracle
run on the FP32-rounded start; the leaf totals are conserved over several
steps of alternating sweep order."""
import numpy as np
import pytest
import torch

from oracle import closing
from gpu_helpers import FP64, GAMMA, check, norms, note
from paper_0907_3390_amd import amr, tvd, workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    c = tvd.Context(0)
    yield c
    c.close()


def _refined():
    r = np.zeros((4, 4, 4), dtype=bool)
    r[1, 1, 1] = r[1, 1, 2] = r[1, 2, 1] = True
    r[3, 0, 3] = True
    return r


def _state(Nc, seed, f32):
    coarse = wl.lognormal(Nc, seed=seed, sigma_ln=0.5)
    fine = wl.lognormal(2 * Nc, seed=seed + 1, sigma_ln=0.5)
    if f32:
        coarse = coarse.astype(np.float32).astype(np.float64)
        fine = fine.astype(np.float32).astype(np.float64)
    return coarse, fine


@pytest.mark.parametrize("dtype,n", [(torch.float64, 8), (torch.float32, 8), (torch.float32, 16)])
@pytest.mark.parametrize("subcycle", [False, True])
def test_two_level_driver_matches_oracle(ctx, dtype, n, subcycle):
    note(f"two-level driver dtype={dtype} n={n} subcycle={subcycle}")
    Nc = 32
    coarse, fine = _state(Nc, 400 + n + 10 * subcycle, dtype == torch.float32)
    dev = amr.TwoLevelDevice(ctx, Nc, _refined(), n, dtype=dtype)
    L = dev.L
    fb = np.stack([fine[:, z:z + n, y:y + n, x:x + n] for z, y, x in L.origins])
    dev.upload(coarse, fb)
    dt = 0.2 / (2 * Nc) / 4.0
    dev.step(dt, 0, subcycle=subcycle)
    torch.cuda.synchronize()
    assert ctx.tvd_read_flags()[2] == 0
    got_c, got_f = dev.download()
    step = closing.two_level_step_subcycled if subcycle else closing.two_level_step
    want_c, want_f = step(coarse, fine, L.refined, n, dt, 0, GAMMA)
    want_fb = np.stack([want_f[:, z:z + n, y:y + n, x:x + n] for z, y, x in L.origins])
    err_c = np.abs(got_c - want_c).sum() / np.abs(want_c).sum()
    err_f = np.abs(got_f - want_fb).sum() / np.abs(want_fb).sum()
    note(f"  coarse relL1 {err_c:.1e}, fine {err_f:.1e}")
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert err_c <= tol and err_f <= tol
    bounds = FP64 if dtype == torch.float64 else (1e-5, 1e-4)
    check(norms(got_c, want_c), bounds)
    check(norms(got_f.transpose(1, 0, 2, 3, 4).reshape(5, -1),
                want_fb.transpose(1, 0, 2, 3, 4).reshape(5, -1)), bounds)


@pytest.mark.parametrize("subcycle", [False, True])
def test_two_level_driver_conserves_over_steps(ctx, subcycle):
    Nc, n = 32, 8          # FP64 blocks are 8^3 patches (16^3 groups do not fit the LDS)
    coarse, fine = _state(Nc, 430, False)
    dev = amr.TwoLevelDevice(ctx, Nc, _refined(), n, dtype=torch.float64)
    L = dev.L
    fb = np.stack([fine[:, z:z + n, y:y + n, x:x + n] for z, y, x in L.origins])
    dev.upload(coarse, fb)
    full = lambda fbl: _fine_grid(L, fbl, Nc)
    before = closing.leaf_sums(coarse, full(fb), L.refined)
    scale = closing.leaf_sums(np.abs(coarse), np.abs(full(fb)), L.refined)
    dt = 0.2 / (2 * Nc) / 4.0
    for s in range(6):
        dev.step(dt, s % 2, subcycle=subcycle)
    torch.cuda.synchronize()
    c, f = dev.download()
    after = closing.leaf_sums(c, full(f), L.refined)
    rel = np.max(np.abs(after - before) / scale)
    note(f"  6 steps subcycle={subcycle}: leaf total change / scale {rel:.1e}")
    assert rel <= 1e-13


def _fine_grid(L, blocks, Nc):
    n = L.n
    out = np.zeros((5, 2 * Nc, 2 * Nc, 2 * Nc))
    for blk, (oz, oy, ox) in zip(blocks, L.origins):
        out[:, oz:oz + n, oy:oy + n, ox:ox + n] = blk
    return out


def test_two_level_step_graph_replay(ctx):
    """Two sub-cycled two-level steps (orders xyz, zyx) recorded into a HIP
    graph through the library's native capture and replayed three times, with
    eager work in between, against the same steps run eagerly: identical
    bits after every replay (the sequence holds no memset and no host
    round trip)."""
    Nc, n = 32, 8
    coarse, fine = _state(Nc, 440, False)
    eager = amr.TwoLevelDevice(ctx, Nc, _refined(), n, dtype=torch.float64)
    graph = amr.TwoLevelDevice(ctx, Nc, _refined(), n, dtype=torch.float64)
    L = eager.L
    fb = np.stack([fine[:, z:z + n, y:y + n, x:x + n] for z, y, x in L.origins])
    for d in (eager, graph):
        d.upload(coarse, fb)
    torch.cuda.synchronize()
    dt = 0.2 / (2 * Nc) / 4.0
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ctx.tvd_graph_begin(s)
        for o in (0, 1):
            graph.step(dt, o, subcycle=True)
        g = ctx.tvd_graph_end(s)
    torch.cuda.synchronize()
    try:
        for rep in range(3):
            for o in (0, 1):
                eager.step(dt, o, subcycle=True)
            g.replay(torch.cuda.current_stream())
            torch.cuda.synchronize()
            ce, fe = eager.download()
            cg, fg = graph.download()
            assert np.array_equal(ce, cg) and np.array_equal(fe, fg), rep
    finally:
        g.close()
