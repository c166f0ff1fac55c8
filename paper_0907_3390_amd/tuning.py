"""Block-edge (patch-group size) selection by measurement.

The launch variant of one block edge (workgroup size, LDS layout, pencil
split) is chosen by the library's own tuner (tvd_autotune) on the caller's
data.  The block edge itself fixes the data layout: the same cells can be cut
into 8^3 patches or into 2^3 groups of them (16^3 blocks, Sec. 3.1), so
choosing it means building each candidate layout and timing it.  This module
does that for a set of independent periodic boxes: every candidate layout is
uploaded, run for one warm-up pair of steps, captured as a HIP graph of one
xyz/zyx pair and replayed; the fastest layout wins.
"""
from __future__ import annotations

import numpy as np
import torch

from . import layout, tvd
from .driver import DeviceBlocks


def graph_ms_per_step(dev: DeviceBlocks, pairs: int = 4, stream=None) -> float:
    """Mean device time of one step, from `pairs` replays of a graph holding
    one xyz/zyx pair (the device must have run at least one pair)."""
    side = torch.cuda.Stream() if stream is None else stream
    g = dev.capture(2, stream=side)
    try:
        dev.replay(g, stream=side)  # untimed
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(side)
        for _ in range(pairs):
            dev.replay(g, stream=side)
        b.record(side)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / (2 * pairs)
    finally:
        g.close()


def boxes_device(ctx, grids, dhs, edge_for, dtype=torch.float32, gather=True,
                 kernel=tvd.TVD_KERNEL_AUTO, gamma=5.0 / 3.0, cfl=0.5) -> DeviceBlocks:
    """Independent periodic boxes cut into blocks of edge edge_for(L), uploaded."""
    edges = [g.shape[1] for g in grids]
    bs = layout.boxes_blockset(edges, edge_for, dhs)
    dev = DeviceBlocks(ctx, bs, dtype=dtype, gather=gather, kernel=kernel, gamma=gamma, cfl=cfl)
    dev.upload(layout.boxes_to_blocks(grids, edge_for))
    return dev


def tune_block_edge(ctx, grids, dhs, candidates: dict, dtype=torch.float32, pairs: int = 4,
                    gamma=5.0 / 3.0, cfl=0.5):
    """Time each candidate layout (name -> edge_for(L) giving the block edge of
    a box of edge L) on the given boxes and return (best name, {name: ms per
    step}).  A candidate with a uniform block edge first lets tvd_autotune
    pick that edge's launch variant on the same data."""
    times = {}
    for name, edge_for in candidates.items():
        dev = boxes_device(ctx, grids, dhs, edge_for, dtype=dtype, gamma=gamma, cfl=cfl)
        if dev.bs.uniform_edge is not None:
            dev.dt.fill_(cfl * float(np.min(dev.bs.dh)) / 4.0)
            ctx.tvd_autotune(dev.batch, dev.nbr, dev.interior, dev.spare, gamma, reps=2)
        dev.run(2)
        times[name] = graph_ms_per_step(dev, pairs)
        del dev
        torch.cuda.empty_cache()
    best = min(times, key=times.get)
    return best, times
