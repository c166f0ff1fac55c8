"""GPU parity on the method's degenerate cases, against the FP64 oracle.

* Pressure floor (the reading P* = max(P, p_floor) in the fluxes, the sound
  speed and the signal speed, the stored energy untouched): a cold,
  supersonic lognormal state whose pressures lie around the floor, so that
  at least 10 % of the initial cells are floored and the floor changes the
  result well beyond the parity bounds, in FP64 (<= 1e-12 relative L1 and
  Linf) and FP32 (the rough-data bounds), with every kernel.
* gamma = 1 (pressureless gas: P = 0, c_s = 0, c = |v_d|) with a third of
  the cells at rest, where the freezing speed is exactly 0 and the split
  fluxes and the limiter's inputs vanish (the FP32 limiter's a + b = 0
  branch).
"""
import numpy as np
import pytest
import torch

from gpu_helpers import FP32_ROUGH, FP64, check, norms, note, oracle_periodic, worst
from paper_0907_3390_amd import layout, tvd, workloads as wl
from paper_0907_3390_amd.driver import DeviceBlocks

pytestmark = pytest.mark.gpu

# (label, dtype, block edge, kernel flags, gather, stream)
MODES = {
    "fp64-plain-8": (torch.float64, 8, tvd.TVD_KERNEL_PLAIN, False, False),
    "fp64-batched-8": (torch.float64, 8, tvd.TVD_KERNEL_BATCHED, True, False),
    "fp64-stream-16": (torch.float64, 16, tvd.TVD_KERNEL_AUTO, True, True),
    "fp32-batched-16": (torch.float32, 16, tvd.TVD_KERNEL_BATCHED, True, False),
    "fp32-persistent-8": (torch.float32, 8, tvd.TVD_KERNEL_PERSISTENT, True, False),
    "fp32-stream-16": (torch.float32, 16, tvd.TVD_KERNEL_AUTO, True, True),
    "fp32-stream-32": (torch.float32, 32, tvd.TVD_KERNEL_AUTO, True, True),
}


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    c = tvd.Context(0)
    yield c
    c.close()


def run_mode(ctx, grid, steps, mode, p_floor=0.0, gamma=5.0 / 3.0):
    dtype, n, kernel, gather, stream = MODES[mode]
    N = grid.shape[3]
    bs = layout.periodic_grid_blockset(N, n, curve="morton")
    dev = DeviceBlocks(ctx, bs, dtype=dtype, gather=gather, stream=stream, kernel=kernel,
                       p_floor=p_floor, gamma=gamma)
    dev.upload(layout.grid_to_blocks(grid, n, bs.perm))
    ctx.tvd_read_flags()
    dev.run(steps)
    torch.cuda.synchronize()
    st, floored, bad = ctx.tvd_read_flags()
    out = layout.blocks_to_grid(np.stack(dev.download()), grid.shape, bs.perm)
    return out, floored, bad


def cold_supersonic(N, seed, p_floor, gamma=5.0 / 3.0):
    """Lognormal density, Gaussian velocities of unit spread (Mach ~ 100),
    pressures lognormal around the floor."""
    r = wl.rng(seed)
    rho = np.exp(r.standard_normal((N, N, N)) - 0.5)
    v = r.standard_normal((3, N, N, N))
    P = p_floor * np.exp(1.5 * r.standard_normal((N, N, N)))
    return wl.conserved(rho, v[0], v[1], v[2], P, gamma)


def floored_fraction(u, p_floor, gamma=5.0 / 3.0):
    kin = 0.5 * (u[1] ** 2 + u[2] ** 2 + u[3] ** 2) / u[0]
    return float(np.mean((gamma - 1.0) * (u[4] - kin) < p_floor))


@pytest.mark.parametrize("mode", list(MODES))
def test_pressure_floor_parity(ctx, mode):
    """A cold supersonic state with p_floor 1e-4: about half of the initial
    cells are floored (>= 10 % required).  The supersonic flow shocks and
    heats the gas, so few cells stay below the floor after the first step;
    the floor's effect on the result is therefore required instead: the
    oracle without the floor differs from the oracle with it by at least 10x
    the parity bound (relative L1), so a device that skipped the floor would
    fail.  The GPU matches the oracle with the floor after 4 steps and
    reports floored cells."""
    dtype = MODES[mode][0]
    note(f"pressure floor parity, {mode}")
    pf = 1e-4
    g = cold_supersonic(32, seed=41, p_floor=pf)
    if dtype == torch.float32:
        g = g.astype(np.float32).astype(np.float64)
    frac0 = floored_fraction(g, pf)
    assert frac0 >= 0.1
    want, _ = oracle_periodic(g, 4, p_floor=pf)
    free, _ = oracle_periodic(g, 4, p_floor=0.0)
    bounds = FP64 if dtype == torch.float64 else FP32_ROUGH
    effect = worst(norms(free, want))
    assert effect >= 10 * bounds[0], effect
    got, floored, bad = run_mode(ctx, g, 4, mode, p_floor=pf)
    nrm = norms(got, want)
    note(f"  initial floored fraction {frac0:.2f}, floor effect {effect:.1e}, device floored "
         f"count {floored}, " +
         str({k: (f"{v['relL1']:.1e}", f"{v['relLinf']:.1e}") for k, v in nrm.items()}))
    assert floored > 0 and bad == 0
    check(nrm, bounds)


@pytest.mark.parametrize("mode", list(MODES))
def test_pressureless_with_cells_at_rest(ctx, mode):
    """gamma = 1: P = 0 and c_s = 0 everywhere, c = |v_d|; a third of the
    cells are at rest, so their freezing speed and split fluxes are exactly
    zero.  6 steps against the oracle; no cell becomes non-physical."""
    dtype = MODES[mode][0]
    note(f"pressureless gamma = 1 with cells at rest, {mode}")
    r = wl.rng(42)
    N = 32
    rho = np.exp(0.5 * r.standard_normal((N, N, N)) - 0.125)
    v = 0.5 * r.standard_normal((3, N, N, N))
    v[:, r.random((N, N, N)) < 1.0 / 3.0] = 0.0
    g = wl.conserved(rho, v[0], v[1], v[2], 0.0, gamma=1.0)
    if dtype == torch.float32:
        g = g.astype(np.float32).astype(np.float64)
    want, _ = oracle_periodic(g, 6, gamma=1.0)
    got, floored, bad = run_mode(ctx, g, 6, mode, gamma=1.0)
    nrm = norms(got, want, gamma=1.0)
    # momentum on the largest rho |v| (there is no sound speed)
    for k, nm in enumerate(["m_x", "m_y", "m_z"]):
        scale = np.max(np.abs(want[1 + k]))
        nrm[nm]["relLinf"] = float(np.abs(got[1 + k] - want[1 + k]).max() / scale)
        nrm[nm]["relL1"] = float(np.abs(got[1 + k] - want[1 + k]).sum() /
                                 np.abs(want[1 + k]).sum())
    note("  " + str({k: (f"{v['relL1']:.1e}", f"{v['relLinf']:.1e}") for k, v in nrm.items()}))
    assert bad == 0
    check(nrm, FP64 if dtype == torch.float64 else FP32_ROUGH)
