"""Device-resident step sequencing over a set of blocks.

Each step runs entirely in libtvd kernels on one stream, with no host round
trip: before every even step the time step comes from the Eq. (CFL) signal
speed of the current state (kept in device memory), the ghost zones are
refilled from sibling interiors, and the state is advanced by one triple,
forward xyz on even steps and backward zyx on odd steps, the pair sharing
one dt (Sec. 2.2).  In gather mode the refill and the advance are one
kernel: the advance reads ghost cells from the neighbours' interiors and
writes the other of two interior buffers.  The signal speed of an odd step's output is fused into
that step's advance, and the conservation sums can be fused into any step.
torch only provides the device buffers and the stream.
"""
from __future__ import annotations

import numpy as np
import torch

from . import layout, tvd
from .layout import BlockSet


def default_chain_len(tiles: int, slots: int = 1024) -> int:
    """Chain length of the streamed advance for `tiles` block-face tiles: as
    long as possible (each chain repeats the first two sweeps on six ghost
    planes) while leaving about `slots` chains (two workgroups on each of the
    256 compute units, twice over) to spread over the chip; 4 to 64 blocks."""
    return int(min(64, max(4, tiles // slots)))


class DeviceBlocks:
    """Interior and ghosted buffers, tables and per-block dt/dh on one GPU."""

    def __init__(self, ctx: tvd.Context, bs: BlockSet, dtype=torch.float32,
                 device="cuda:0", gamma: float = 5.0 / 3.0, p_floor: float = 0.0,
                 cfl: float = 0.5, kernel: int = tvd.TVD_KERNEL_AUTO, gather: bool = False,
                 stream: bool = False, chain_len: int | None = None):
        self.ctx = ctx
        self.bs = bs
        self.dtype = dtype
        self.device = torch.device(device)
        self.gamma = gamma
        self.p_floor = p_floor
        self.cfl = cfl
        self.kernel = kernel
        self.stream = stream
        self.gather = gather or stream
        gather = self.gather
        dev = self.device
        self.interior = torch.zeros(bs.out_total, dtype=dtype, device=dev)
        if gather:
            self.spare = torch.zeros(bs.out_total, dtype=dtype, device=dev)
            self.ghosted = None
        else:
            self.ghosted = torch.zeros(bs.in_total, dtype=dtype, device=dev)
        self.nbr = torch.from_numpy(bs.nbr).to(dev)
        self.dh = torch.from_numpy(bs.dh).to(dev)
        self.dt = torch.zeros(bs.n_blocks, dtype=torch.float64, device=dev)
        self.smax = torch.zeros(1, dtype=torch.float64, device=dev)
        self.sums = torch.zeros(5, dtype=torch.float64, device=dev)
        uniform = bs.uniform_edge
        code = tvd.dtype_code(dtype)
        if uniform is not None:
            # dense packing, no offset tables
            self.batch = tvd.Batch(code, bs.n_blocks, uniform, d_dt=self.dt, d_dh=self.dh)
            self.batch_const = tvd.Batch(code, bs.n_blocks, uniform, d_dh=self.dh)
        else:
            self.edges = torch.from_numpy(bs.edges).to(dev)
            self.in_off = torch.from_numpy(bs.in_off).to(dev)
            self.out_off = torch.from_numpy(bs.out_off).to(dev)
            self.batch = tvd.Batch(code, bs.n_blocks, 0, d_edge=self.edges, d_in_off=self.in_off,
                                   d_out_off=self.out_off, d_dt=self.dt, d_dh=self.dh)
            self.batch_const = self.batch
        quads = 1
        if stream:
            # chains along z for the forward step, along x for the backward one
            if uniform not in (16, 32):
                raise ValueError("the streamed advance takes a uniform block edge of 16 or 32")
            quads = (uniform // 16) ** 2
            self.set_chains(default_chain_len(bs.n_blocks * quads) if chain_len is None
                            else chain_len)
        ctx.tvd_reserve(bs.n_blocks * quads)
        self.step_index = 0

    def set_chains(self, chain_len: int):
        """Chains of at most chain_len blocks for the streamed advance: along
        z for the forward step, along x for the backward one."""
        self.chain_len = chain_len
        self.chains = {}
        for order, axis in ((tvd.TVD_XYZ, 2), (tvd.TVD_ZYX, 0)):
            st, bl = layout.stream_chains(self.bs.nbr, axis, chain_len)
            self.chains[order] = tvd.Chains(torch.from_numpy(st).to(self.device),
                                            torch.from_numpy(bl).to(self.device))

    # -- data movement (host <-> device), not part of a step ----------------
    def upload(self, blocks):
        flat = self.bs.pack_interior(blocks)
        self.interior.copy_(torch.from_numpy(flat).to(self.dtype))

    def download(self) -> list:
        return self.bs.unpack_interior(self.interior.cpu().numpy())

    # -- the step ---------------------------------------------------------------
    def signal_speed(self):
        self.ctx.tvd_max_signal_speed(self.batch, self.interior, tvd.TVD_LAYOUT_INTERIOR,
                                      self.gamma, self.smax, self.p_floor)

    def set_dt_from_speed(self):
        self.ctx.tvd_dt_from_speed(self.batch, self.smax, self.cfl, self.dt)

    def fill_ghosts(self):
        self.ctx.tvd_fill_ghosts(self.batch, self.nbr, self.interior, self.ghosted)

    def advance(self, order: int, fuse_speed: bool = False, fuse_sums: bool = False):
        smax = self.smax if fuse_speed else None
        sums = self.sums if fuse_sums else None
        if self.stream:
            self.ctx.tvd_patch_advance_stream(self.batch, self.nbr, self.chains[order],
                                              self.interior, self.spare, order, self.gamma,
                                              self.p_floor, self.kernel, smax=smax, sums=sums)
            self.interior, self.spare = self.spare, self.interior
        elif self.gather:
            self.ctx.tvd_patch_advance_gather(self.batch, self.nbr, self.interior, self.spare,
                                              order, self.gamma, self.p_floor, self.kernel,
                                              smax=smax, sums=sums)
            self.interior, self.spare = self.spare, self.interior
        else:
            self.ctx.tvd_patch_advance(self.batch, self.ghosted, self.interior, order,
                                       self.gamma, self.p_floor, self.kernel, smax=smax,
                                       sums=sums)

    def step(self, fused: bool = True, sums: bool = False):
        """One step; even steps take a fresh dt, odd steps reuse it."""
        s = self.step_index
        if s % 2 == 0:
            if not (fused and s > 0):
                self.signal_speed()
            self.set_dt_from_speed()
        if not self.gather:
            self.fill_ghosts()
        self.advance(s % 2, fuse_speed=fused and s % 2 == 1, fuse_sums=sums)
        self.step_index += 1

    def run(self, steps: int, fused: bool = True, sums_each_step: bool = False):
        """Run steps; returns the per-step sums (device tensor) if requested."""
        rec = torch.zeros((steps, 5), dtype=torch.float64, device=self.device) if sums_each_step else None
        for i in range(steps):
            self.step(fused=fused, sums=sums_each_step)
            if rec is not None:
                rec[i].copy_(self.sums)
        return rec

    def capture(self, steps: int, fused: bool = True, sums: bool = False, stream=None):
        """Record `steps` steps (an even number, so that the pair structure
        and the ping-pong buffers come back to where they started) into a HIP
        graph through the library's native capture; returns the graph.  The
        recorded work does not run: replay it with graph.replay()."""
        if steps % 2:
            raise ValueError("capture whole xyz/zyx pairs")
        if self.step_index % 2:
            raise ValueError("capture must start on an even step")
        if self.step_index == 0 and fused:
            raise ValueError("run one pair first: the fused speed of an odd step seeds dt")
        s = torch.cuda.Stream() if stream is None else stream
        s.wait_stream(torch.cuda.current_stream())
        start = self.step_index
        with torch.cuda.stream(s):
            self.ctx.tvd_graph_begin(s)
            try:
                for _ in range(steps):
                    self.step(fused=fused, sums=sums)
            except Exception:
                self.ctx.tvd_graph_end(s).close()
                raise
            g = self.ctx.tvd_graph_end(s)
        self.step_index = start
        self.graph_steps = steps
        return g

    def replay(self, graph, stream=None):
        graph.replay(stream)
        self.step_index += self.graph_steps

    def conservation_sums(self):
        self.ctx.tvd_conservation_sums(self.batch, self.interior, tvd.TVD_LAYOUT_INTERIOR, self.sums)
        return self.sums


def timed_dt_host(dev: DeviceBlocks) -> np.ndarray:
    return dev.dt.cpu().numpy()
