"""A two-level periodic hierarchy advanced on the device, step by step.

Sequencing only: every step is a fixed order of C-ABI calls (the kernels do
all the arithmetic), on device-resident state.  The coarse level is an
Nc^3 periodic grid of 8^3 patches; the refined patches are replaced on the
next level by fine blocks of edge 8 or 16 (layout.RefinedLevels).

One step (Sec. 2.1 and 2.2; Sec. 3.1 for the fluxes and the closing step):
  * the coarse level: sibling ghost fill, advance writing flux records;
  * the fine level: coarse-fine ghost fill (sibling copy, else Min-Mod
    limited interpolation from the coarse level at the old time), advance
    writing flux records, with the same dt (uniform time step), or, with
    sub-cycling, twice with dt/2, the second time with ghost zones from the
    coarse level half-way through its step (linear in time) and the other
    sweep order, the records summed with weight 1/2 each;
  * the closing step: restriction of the fine level into its coarse patches
    and the coarse-fine flux correction, one launch.
"""
from __future__ import annotations

import numpy as np
import torch

from . import layout, tvd

GAMMA = 5.0 / 3.0


class TwoLevelDevice:
    def __init__(self, ctx: tvd.Context, Nc: int, refined, n: int, dtype=torch.float64,
                 gamma: float = GAMMA):
        self.ctx, self.dtype, self.gamma = ctx, dtype, gamma
        self.L = L = layout.RefinedLevels(Nc, refined, n)
        self.code = tvd.dtype_code(dtype)
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        z = lambda k: torch.zeros(k, dtype=dtype, device="cuda")
        nc, nf = L.coarse.n_blocks, L.fine.n_blocks
        self.nc, self.nf, self.n = nc, nf, n
        self.c_int, self.c_gh, self.c_out = z(nc * 5 * 512), z(nc * 5 * 14 ** 3), z(nc * 5 * 512)
        self.c_half = z(nc * 5 * 512)
        m = n + 6
        self.f_int, self.f_gh, self.f_mid = z(nf * 5 * n ** 3), z(nf * 5 * m ** 3), z(nf * 5 * n ** 3)
        self.c_flux = z(nc * layout.flux_record_size(8))
        self.f_flux = z(nf * layout.flux_record_size(n))
        self.c_nbr, self.f_nbr = dev(L.coarse.nbr), dev(L.fine.nbr)
        self.cnbr, self.corigin = dev(L.cnbr), dev(L.corigin)
        rr, fr, _ = L.tables()
        gr, gs = layout.group_face_rows(fr)
        self.rr, self.gr, self.gs = dev(rr), dev(gr), dev(gs)

    def upload(self, coarse_grid, fine_blocks):
        """Coarse grid (5, Nc, Nc, Nc); fine interiors (B, 5, n, n, n) in
        RefinedLevels order."""
        self.c_int.copy_(torch.from_numpy(layout.grid_to_blocks(coarse_grid, 8)).reshape(-1))
        self.f_int.copy_(torch.from_numpy(np.ascontiguousarray(fine_blocks)).reshape(-1))

    def download(self):
        """(coarse grid, fine interiors) as FP64 numpy arrays."""
        Nc = self.L.Nc
        c = layout.blocks_to_grid(self.c_int.double().cpu().numpy().reshape(-1, 5, 8, 8, 8),
                                  (5, Nc, Nc, Nc))
        f = self.f_int.double().cpu().numpy().reshape(self.nf, 5, self.n, self.n, self.n)
        return c, f

    def _batches(self, dt):
        Nc = self.L.Nc
        cb = tvd.Batch(self.code, self.nc, 8, dt=dt, dh=1.0 / Nc)
        return cb

    def _fine(self, coarse_src, fine_src, fine_dst, dt, order, weight, acc):
        ctx, Nc = self.ctx, self.L.Nc
        fb = tvd.Batch(self.code, self.nf, self.n, dt=dt, dh=0.5 / Nc)
        cb = tvd.Batch(self.code, self.nc, 8, dt=dt, dh=1.0 / Nc)
        ctx.tvd_fill_ghosts_amr(fb, self.f_nbr, fine_src, self.f_gh, cb, coarse_src, self.cnbr,
                                self.corigin)
        ctx.tvd_patch_advance_flux(fb, self.f_gh, fine_dst, self.f_flux, None, order, self.gamma,
                                   flux_weight=weight, accumulate=acc)
        return fb

    def step(self, dt: float, order: int, subcycle: bool = False):
        """One coarse step of dt (sweep order `order`) with the closing step;
        the fine level takes one step of dt, or two of dt/2 when `subcycle`."""
        ctx = self.ctx
        cb = self._batches(dt)
        ctx.tvd_fill_ghosts(cb, self.c_nbr, self.c_int, self.c_gh)
        ctx.tvd_patch_advance_flux(cb, self.c_gh, self.c_out, self.c_flux, None, order, self.gamma)
        if not subcycle:
            fb = self._fine(self.c_int, self.f_int, self.f_mid, dt, order, 1.0, 0)
            f_new = self.f_mid
        else:
            self._fine(self.c_int, self.f_int, self.f_mid, 0.5 * dt, order, 0.5, 0)
            ctx.tvd_lerp(self.code, self.nc * 5 * 512, self.c_int, self.c_out, self.c_half, 0.5)
            # the second sub-step reads the first's result and writes the
            # level's new state back into f_int
            fb = self._fine(self.c_half, self.f_mid, self.f_int, 0.5 * dt, 1 - order, 0.5, 1)
            f_new = self.f_int
        ctx.tvd_close_level(cb, self.c_out, self.c_flux, None, fb, f_new, self.f_flux, None,
                            self.rr, self.gr, self.gs)
        self.c_int, self.c_out = self.c_out, self.c_int
        if f_new is self.f_mid:
            self.f_int, self.f_mid = self.f_mid, self.f_int
