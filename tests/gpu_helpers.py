"""Shared glue for the GPU tests: error norms and oracle reference runs.

The norms follow the parity definitions: relative L1 over the sum of |b| for
density and energy, and for each momentum component the L1 difference over
the sum of rho * c_s of the reference (the natural momentum scale), with the
own-norm reported too.
"""
from __future__ import annotations

import sys

import numpy as np

import oracle

GAMMA = 5.0 / 3.0


def note(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def norms(a, b, gamma=GAMMA):
    """Per-variable error norms of a against reference b, both (5, ...)."""
    a = np.asarray(a, dtype=np.float64).reshape(5, -1)
    b = np.asarray(b, dtype=np.float64).reshape(5, -1)
    rho = b[0]
    kin = 0.5 * (b[1] ** 2 + b[2] ** 2 + b[3] ** 2) / rho
    P = np.maximum((gamma - 1.0) * (b[4] - kin), 0.0)
    cs = np.sqrt(gamma * P / rho)
    scale = np.sum(rho * cs)
    out = {}
    names = ["rho", "m_x", "m_y", "m_z", "e"]
    mscale = max(float(np.max(rho * cs)), 1e-300)
    for k, nm in enumerate(names):
        d = np.abs(a[k] - b[k])
        own = np.sum(np.abs(b[k]))
        own_max = max(np.abs(b[k]).max(), 1e-300)
        out[nm] = {
            "relL1": d.sum() / (own if k in (0, 4) else max(scale, 1e-300)),
            "relL1_own": d.sum() / max(own, 1e-300),
            # elementwise: the largest difference against the variable's
            # largest magnitude (momentum: against the largest rho c_s)
            "relLinf": d.max() / (own_max if k in (0, 4) else max(mscale, own_max)),
            "relLinf_own": d.max() / own_max,
        }
    return out


def worst(nrm, key="relL1"):
    return max(v[key] for v in nrm.values())


# Parity bounds (relative L1, relative Linf per variable).  FP64: the same
# arithmetic in another order, differences at round-off (1e-16 per
# operation).  FP32: each step rounds O(100) operations per cell at 6e-8, a
# per-cell relative error of about 1e-6 after ten steps; the largest cell is
# allowed 100x that on smooth data and 1000x on rough data, where limiter
# switches and shocks amplify round-off differences locally.
FP64 = (1e-12, 1e-12)
FP32_SMOOTH = (1e-5, 1e-4)
FP32_ROUGH = (1e-5, 1e-3)


def check(nrm, bounds):
    """Assert both norms of every variable within (L1, Linf) bounds."""
    l1, linf = bounds
    assert worst(nrm, "relL1") <= l1, {k: v["relL1"] for k, v in nrm.items()}
    assert worst(nrm, "relLinf") <= linf, {k: v["relLinf"] for k, v in nrm.items()}


def oracle_periodic(grid, steps, n=8, cfl=0.5, gamma=GAMMA, p_floor=0.0):
    N = grid.shape[3]
    return oracle.run_periodic(np.asarray(grid, dtype=np.float64), steps, cfl, 1.0 / N, gamma,
                               n=n, p_floor=p_floor)


def cone_blocks(grid, n, picks, steps, dt, dh, gamma=GAMMA, p_floor=0.0):
    """Oracle outputs of the blocks `picks` (block indices, x fastest) of a
    periodic grid cut into n^3 blocks after `steps` steps (xyz, zyx, ...) of
    fixed dt, computed from each block's dependency cone only: a step needs
    three ghost cells per side, so `steps` steps need a region of
    n + 6 * steps cells around the block.  Returns {pick: (5, n, n, n)}."""
    _, Nz, Ny, Nx = grid.shape
    nbx, nby = Nx // n, Ny // n
    out = {}
    for b in picks:
        bx, by, bz = b % nbx, (b // nbx) % nby, b // (nbx * nby)
        h = 3 * steps
        # region [start - h, start + n + h) with periodic wrap
        idx = [np.arange(s * n - h, s * n + n + h) for s in (bz, by, bx)]
        sub = grid[:, idx[0] % Nz][:, :, idx[1] % Ny][:, :, :, idx[2] % Nx]
        for s in range(steps):
            # the sub-grid is one ghosted block: a step keeps the cells with
            # full support and drops three cells per side
            sub = oracle.advance_blocks(np.ascontiguousarray(sub[None]), s % 2, dt, dh, gamma,
                                        p_floor)[0]
        out[b] = sub
    return out


def oracle_boxes(grids, dhs, steps, cfl=0.5, gamma=GAMMA, p_floor=0.0):
    """Independent periodic boxes advanced together by the oracle: before
    every even step S is the Eq. (CFL) signal speed over all boxes and box i
    takes dt_i = cfl * dh_i / S; each box is one ghosted block (periodic wrap
    by three cells), so the region rule runs over the whole box."""
    state = [np.asarray(g, dtype=np.float64) for g in grids]
    dhs = np.asarray(dhs, dtype=np.float64)
    dt = None
    for s in range(steps):
        if s % 2 == 0:
            S = max(oracle.max_signal_speed(g, gamma, p_floor) for g in state)
            dt = cfl * dhs / S
        ghosted = [np.pad(g, ((0, 0), (3, 3), (3, 3), (3, 3)), mode="wrap") for g in state]
        state = oracle.advance_ragged(ghosted, s % 2, dt, dhs, gamma, p_floor)
    return state
