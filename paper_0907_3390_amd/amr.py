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
        ctx.tvd_reserve(max(nc, nf))
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


class NestedDevice:
    """A periodic hierarchy on any number of levels (layout.NestedLevels),
    held as 8^3 patches or as 2^3 patch groups of 16^3 (n = 16; Sec. 3.1),
    advanced on the device, every level sub-cycled.

    One root step of dt (Sec. 2.1, a level's update: advance, let the finer
    level catch up, correct with it):
      * level 0: sibling ghost fill, advance writing flux records;
      * level l >= 1, inside each step of dt' of level l-1: two steps of
        dt'/2 (sweep orders o, then 1 - o), each a coarse-fine ghost fill
        (sibling copy, else interpolation from level l-1 at the start of the
        step for the first, half-way through it, linear in time, for the
        second) and an advance writing this sub-step's flux records; after
        each, level l+1 catches up in the same way and level l is closed
        with it (restriction, flux correction with level l+1's records
        averaged over the step);
      * level l's records over its parent's step: the mean of its two
        sub-steps' records (tvd_lerp at 1/2);
      * finally level 0 is closed with level 1.
    Per level: interior, new and ghosted states, flux record buffers (one on
    level 0, one per sub-step and their mean on the others); per coarse level
    a time-interpolated state."""

    def __init__(self, ctx: tvd.Context, Nc: int, refined, dtype=torch.float64,
                 gamma: float = GAMMA, n: int = 8, gather: bool = False,
                 stream_min_blocks: int | None = None, stream_chain_len: int | None = None,
                 overlap: bool = False):
        if n == 16 and dtype != torch.float32:
            raise ValueError("patch groups (n = 16) advance in FP32: the flux-recording FP64 "
                             "advance holds blocks of edge 8 only")
        if overlap and not gather:
            raise ValueError("overlapped levels need the gathering driver (gather = True)")
        if stream_min_blocks is not None and not (gather and n == 16):
            raise ValueError("the streamed advance with flux records takes FP32 patch groups "
                             "with stand-ins (n = 16, gather = True)")
        self.ctx, self.dtype, self.gamma = ctx, dtype, gamma
        self.L = L = layout.NestedLevels(Nc, refined, n)
        self.n = n
        self.gather = gather
        self.code = tvd.dtype_code(dtype)
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        z = lambda k: torch.zeros(k, dtype=dtype, device="cuda")
        self.nb = [b.n_blocks for b in L.blocks]
        ctx.tvd_reserve(max(self.nb))
        rs = layout.flux_record_size(n)
        self.cells = n ** 3
        if gather:
            # interiors followed by the stand-ins for missing siblings, which
            # the coarse-fine fill writes and the gathering advance reads
            st = [L.stand_ins(lev) for lev in range(L.n_levels)]
            self.vnbr = [dev(t) for t, _ in st]
            self.nsrc = [k for _, k in st]
        else:
            self.nsrc = list(self.nb)
        self.u = [z(k * 5 * n ** 3) for k in self.nsrc]
        self.u_new = [z(k * 5 * n ** 3) for k in self.nsrc]
        if not gather:
            self.u_gh = [z(k * 5 * (n + 6) ** 3) for k in self.nb]
            self.u_half = [z(k * 5 * n ** 3) for k in self.nb[:-1]]
        # level 0 takes one step per root step, the others two
        self.rec = [[z(n * rs)] if lev == 0 else [z(n * rs), z(n * rs)]
                    for lev, n in enumerate(self.nb)]
        self.rec_mean = [None] + [z(n * rs) for n in self.nb[1:]]
        self.nbr = [dev(b.nbr) for b in L.blocks]
        # levels of at least stream_min_blocks blocks advance by the streamed
        # kernel, over chains along z (forward order) and x (backward order)
        # of at most stream_chain_len blocks (default driver.default_chain_len);
        # smaller levels keep the per-block kernel, whose one workgroup per
        # block fills more of the chip than a level's few chains would
        self.chains = [None] * L.n_levels
        if stream_min_blocks is not None:
            from .driver import default_chain_len
            for lev in range(L.n_levels):
                if self.nb[lev] < stream_min_blocks:
                    continue
                cl = stream_chain_len or default_chain_len(self.nb[lev])
                ch = {}
                for order, axis in ((tvd.TVD_XYZ, 2), (tvd.TVD_ZYX, 0)):
                    st_, bl_ = layout.stream_chains(st[lev][0][:self.nb[lev]], axis, cl)
                    ch[order] = tvd.Chains(dev(st_), dev(bl_))
                self.chains[lev] = ch
        self.cnbr = [None] + [dev(t) for t in L.cnbr[1:]]
        self.corigin = [None] + [dev(t) for t in L.corigin[1:]]
        # overlap: level l >= 1 works on a stream of its own, and its first
        # sub-step inside a step of level l-1 runs while level l-1 advances
        # (it reads only level l-1's old state); events order the rest
        self.overlap = overlap
        if overlap:
            nl = L.n_levels
            self.streams = [None] + [torch.cuda.Stream() for _ in range(1, nl)]
            self.ev_fork = [torch.cuda.Event() for _ in range(nl)]
            self.ev_adv = [torch.cuda.Event() for _ in range(nl)]
            self.ev_done = [torch.cuda.Event() for _ in range(nl)]
        self.rows = {}
        for lev, (rr, fr, _) in L.tables().items():
            gr, gs = layout.group_face_rows(fr)
            self.rows[lev] = (dev(rr), dev(gr), dev(gs))

    def upload(self, states):
        """Per level the block interiors (B_l, 5, n, n, n) in NestedLevels
        order."""
        for buf, s, k in zip(self.u, states, self.nb):
            buf[:k * 5 * self.cells].copy_(torch.from_numpy(np.ascontiguousarray(s)).reshape(-1))

    def download(self):
        """Per level the block interiors (B_l, 5, n, n, n), FP64 numpy."""
        n = self.n
        return [b[:k * 5 * n ** 3].double().cpu().numpy().reshape(k, 5, n, n, n)
                for b, k in zip(self.u, self.nb)]

    def _batch(self, lev, dt):
        return tvd.Batch(self.code, self.nb[lev], self.n, dt=dt, dh=1.0 / (self.L.Nc << lev))

    def _close(self, lev, dt, stream=None):
        rr, gr, gs = self.rows[lev]
        self.ctx.tvd_close_level(self._batch(lev, dt), self.u_new[lev], self.rec[lev][self._k[lev]],
                                 None, self._batch(lev + 1, 0.5 * dt), self.u[lev + 1],
                                 self.rec_mean[lev + 1], None, rr, gr, gs, stream=stream)

    def _subcycle(self, lev, dt, order):
        """Level lev takes two steps of dt/2 inside level lev-1's step of dt,
        whose old state is u[lev-1] and whose advanced one u_new[lev-1]."""
        if self.gather:
            return self._subcycle_gather(lev, dt, order)
        ctx, h = self.ctx, 0.5 * dt
        ctx.tvd_lerp(self.code, self.nb[lev - 1] * 5 * self.cells, self.u[lev - 1],
                     self.u_new[lev - 1], self.u_half[lev - 1], 0.5)
        fb, cb = self._batch(lev, h), self._batch(lev - 1, h)
        for k in (0, 1):
            o = order if k == 0 else 1 - order
            src = self.u[lev - 1] if k == 0 else self.u_half[lev - 1]
            ctx.tvd_fill_ghosts_amr(fb, self.nbr[lev], self.u[lev], self.u_gh[lev], cb, src,
                                    self.cnbr[lev], self.corigin[lev])
            ctx.tvd_patch_advance_flux(fb, self.u_gh[lev], self.u_new[lev], self.rec[lev][k], None,
                                       o, self.gamma)
            if lev + 1 < self.L.n_levels:
                self._k[lev] = k
                self._subcycle(lev + 1, h, o)
                self._close(lev, h)
            self.u[lev], self.u_new[lev] = self.u_new[lev], self.u[lev]
        ctx.tvd_lerp(self.code, self.nb[lev] * layout.flux_record_size(self.n), self.rec[lev][0],
                     self.rec[lev][1], self.rec_mean[lev], 0.5)

    def _advance_gather(self, lev, batch, rec, order, stream=None):
        """Level lev's advance with flux records, ghost zones read from the
        siblings and stand-ins: streamed over chains, or per block."""
        if self.chains[lev] is not None:
            self.ctx.tvd_patch_advance_stream_flux(batch, self.vnbr[lev], self.nsrc[lev],
                                                   self.chains[lev][order], self.u[lev],
                                                   self.u_new[lev], rec, None, order,
                                                   self.gamma, stream=stream)
        else:
            self.ctx.tvd_patch_advance_flux_gather(batch, self.vnbr[lev], self.nsrc[lev],
                                                   self.u[lev], self.u_new[lev], rec, None, order,
                                                   self.gamma, stream=stream)

    def _advance_then_child(self, lev, batch, rec, order, dt, s):
        """Overlap: level lev's advance on stream s, with level lev+1's two
        sub-steps of dt/2 (o = order first) on its own stream, forked before
        the advance (the first sub-step needs only level lev's old state;
        the second waits for the advance), then the closing of the pair on
        s once both are done."""
        c = lev + 1
        cs = self.streams[c]
        self.ev_fork[lev].record(s)
        cs.wait_event(self.ev_fork[lev])
        self._advance_gather(lev, batch, rec, order, stream=s)
        self.ev_adv[lev].record(s)
        self._run_level(c, dt, order, cs, self.ev_adv[lev])
        self.ev_done[c].record(cs)
        s.wait_event(self.ev_done[c])
        self._close(lev, dt, stream=s)

    def _run_level(self, lev, dt, order, s, parent_advanced):
        """Overlap: level lev's two sub-steps of dt/2 inside its parent's step
        of dt, issued on stream s; parent_advanced is recorded after the
        parent's advance, which the second sub-step's coarse-fine fill (the
        parent's old and new states, w = 1/2) needs."""
        ctx, h = self.ctx, 0.5 * dt
        fb, cb = self._batch(lev, h), self._batch(lev - 1, h)
        for k in (0, 1):
            o = order if k == 0 else 1 - order
            if k == 1:
                s.wait_event(parent_advanced)
            ctx.tvd_fill_coarse_fine(fb, self.vnbr[lev], self.nsrc[lev], self.u[lev], cb,
                                     self.u[lev - 1], self.u_new[lev - 1], 0.5 * k,
                                     self.cnbr[lev], self.corigin[lev], stream=s)
            self._k[lev] = k
            if lev + 1 < self.L.n_levels:
                self._advance_then_child(lev, fb, self.rec[lev][k], o, h, s)
            else:
                self._advance_gather(lev, fb, self.rec[lev][k], o, stream=s)
            self.u[lev], self.u_new[lev] = self.u_new[lev], self.u[lev]
        ctx.tvd_lerp(self.code, self.nb[lev] * layout.flux_record_size(self.n), self.rec[lev][0],
                     self.rec[lev][1], self.rec_mean[lev], 0.5, stream=s)

    def _subcycle_gather(self, lev, dt, order):
        """_subcycle without ghosted copies: the coarse-fine fill writes only
        the interpolated ghost cells, into the stand-ins for missing
        siblings, from the coarse level interpolated in time on the fly, and
        the gathering advance reads the rest from the siblings."""
        ctx, h = self.ctx, 0.5 * dt
        fb, cb = self._batch(lev, h), self._batch(lev - 1, h)
        for k in (0, 1):
            o = order if k == 0 else 1 - order
            ctx.tvd_fill_coarse_fine(fb, self.vnbr[lev], self.nsrc[lev], self.u[lev], cb,
                                     self.u[lev - 1], self.u_new[lev - 1], 0.5 * k,
                                     self.cnbr[lev], self.corigin[lev])
            self._advance_gather(lev, fb, self.rec[lev][k], o)
            if lev + 1 < self.L.n_levels:
                self._k[lev] = k
                self._subcycle(lev + 1, h, o)
                self._close(lev, h)
            self.u[lev], self.u_new[lev] = self.u_new[lev], self.u[lev]
        ctx.tvd_lerp(self.code, self.nb[lev] * layout.flux_record_size(self.n), self.rec[lev][0],
                     self.rec[lev][1], self.rec_mean[lev], 0.5)

    def step(self, dt: float, order: int):
        """One root step of dt in sweep order `order` (every level sub-cycled,
        every pair closed)."""
        ctx = self.ctx
        self._k = [0] * self.L.n_levels
        b0 = self._batch(0, dt)
        if self.overlap and self.L.n_levels > 1:
            if torch.cuda.is_current_stream_capturing():
                # capturing the forks and joins across the levels' streams
                # crashed the host inside the runtime's end of capture;
                # refused until the cause is known
                raise RuntimeError("the overlapped driver (overlap=True) cannot be captured "
                                   "into a graph; use the sequential driver")
            self._advance_then_child(0, b0, self.rec[0][0], order, dt,
                                     torch.cuda.current_stream())
            self.u[0], self.u_new[0] = self.u_new[0], self.u[0]
            return
        if self.gather:
            # the root grid is complete: every ghost cell is a sibling's
            self._advance_gather(0, b0, self.rec[0][0], order)
        else:
            ctx.tvd_fill_ghosts(b0, self.nbr[0], self.u[0], self.u_gh[0])
            ctx.tvd_patch_advance_flux(b0, self.u_gh[0], self.u_new[0], self.rec[0][0], None,
                                       order, self.gamma)
        if self.L.n_levels > 1:
            self._subcycle(1, dt, order)
            self._close(0, dt)
        self.u[0], self.u_new[0] = self.u_new[0], self.u[0]
