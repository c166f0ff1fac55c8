#!/usr/bin/env python3
"""Throughput of the relaxing-TVD patch advance on one MI355X.

Headline workload: a periodic 512^3 grid, i.e. 262144 octree patches of 8^3
cells run as 32768 Morton-ordered 2^3 patch groups of 16^3: a point blast
(energy 1 as thermal energy in the central 2^3 cells, Sec. 4.3 set-up) on a
lognormal background (sigma_ln = 0.5, gas at rest, P = 1e-5), gamma = 5/3,
CFL 0.5, pressure floor 1e-10, seeded.  A step is one pass of the whole hot
path on the device: the Eq. (CFL) time step on even steps (from the signal
speed fused into the previous odd step), one triple of 1-D sweeps (xyz on
even steps, zyx on odd steps) gathering the ghost zones from the 26
neighbours' interiors, the fused signal speed on odd steps and the fused
FP64 compensated conservation sums on every step.  The timed steps are
replays of a HIP graph of one xyz/zyx pair; odd --steps / --warmup are
rounded up to whole pairs (both counts are reported).

Reported (one JSON line on stdout):
* value: cell-updates/s of the FP32 batched kernel, inputs resident in HBM;
* roofline: the advance kernel's algorithmic FP32 work and HBM bytes per
  launch over its average duration (HIP events on the launch stream)
  against the FP32 vector peak and 8 TB/s, with the HBM traffic from the
  committed rocprofv3 counters when they were taken on the current kernel;
* fp64_plain, l1_vs_fp64: the same steps with the plain FP64 per-patch
  kernel on the same FP32-rounded initial state, and the relative L1 error
  per variable of the FP32 result against it;
* lognormal_256cube: the same measurements on a rough 256^3 state
  (lognormal density sigma_ln = 1, Gaussian velocities), with the batched
  kernel in FP64 on 8^3 patches and in FP32 on single 8^3 patches;
* cpu_baseline: the FP64 oracle, built for the host, on the host cores over
  a bounded sample of the headline workload;
* with --extras: the coarse-fine ghost fill, the multi-level batch, the
  closing step, the nested sub-cycled step, red-black SOR, the gravity
  operator and the uneven batch of 4000 boxes.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_GRID = 256
SEED = 2024
# the headline workload: 512^3 point blast on a lognormal background
N_BLAST = 512
SEED_BLAST = 5
P_FLOOR_BLAST = 1e-10
GAMMA = 5.0 / 3.0
CFL = 0.5
HBM_PEAK_GBS = 8000.0
# FP32 vector peak without packed FP32 (turned off in this build):
# 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
FP32_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_stream_fp32_edge16_512blast_traffic.txt")
# the sources the headline kernel (k_stream<float, 16, ...>) is compiled from
KERNEL_SOURCES = ["paper_0907_3390_amd/csrc/tvd_k_stream_f32.hip",
                  "paper_0907_3390_amd/csrc/tvd_stream.hpp",
                  "paper_0907_3390_amd/csrc/tvd_stream_params.hpp",
                  "paper_0907_3390_amd/csrc/tvd_block.hpp",
                  "paper_0907_3390_amd/csrc/tvd_device.hpp",
                  "paper_0907_3390_amd/csrc/tvd_internal.hpp"]
METRIC = "cell-updates/s (FP32 batched vs FP64 plain) at stated L1 error; HBM GB/s % of peak"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def flops_per_block(n: int) -> int:
    """Algorithmic FP32 work of one step on one block of edge n: a split-flux
    evaluation is 45 flops, a pencil of M = n+6 cells 45M + 5(M-1) + 60(M-2)
    + 65(n+1) + 15n (FMA = 2, add/mul/compare/reciprocal/sqrt = 1), and the
    region rule needs (n+6)^2 + n(n+6) + n^2 pencils."""
    M = n + 6
    pencil = 45 * M + 5 * (M - 1) + 60 * (M - 2) + 65 * (n + 1) + 15 * n
    return pencil * (M * M + n * M + n * n)


def pencil_flops(n: int) -> int:
    """Algorithmic FP32 work of one 1-D update of a pencil of n+6 cells with
    n outputs (the same count as flops_per_block)."""
    M = n + 6
    return 45 * M + 5 * (M - 1) + 60 * (M - 2) + 65 * (n + 1) + 15 * n


def flops_per_cell_stream(planes: int) -> float:
    """Algorithmic FP32 work per cell-update of the streamed schedule on a
    chain of `planes` planes of a 16 x 16 tile: the first two sweeps on 22
    and 16 pencils of 16 outputs for each of planes + 6 planes (three ghost
    planes at each chain end), the third sweep once per cell of each column
    (45 + 5 + 60 + 65 + 15 = 190 flops per cell of an endless pencil,
    planes + 6 cells passed through)."""
    return (planes + 6) / planes * ((22 + 16) * pencil_flops(16) / 256.0 + 190.0)


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(variant):
    """HBM bytes per launch of the headline kernel (mean over the forward and
    backward launches) from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources and on the launch variant the
    run uses: the summary holds one `traffic[chain length,second sweep]`
    entry per variant profiled (the chain length and the second sweep's
    split change which addresses are read and written)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None, "no counter summary"
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_source_hash():
        return None, "kernel changed since the counters were taken"
    if variant is None:
        return None, "no launch variant recorded"
    key = f"traffic[{variant['chain_len']},{variant['second_sweep']}]"
    if key not in kv:
        return None, f"no counters for variant {key[8:-1]} in the summary"
    return float(kv[key]), ("rocprofv3 FETCH_SIZE x2 + WRITE_SIZE, "
                            + os.path.relpath(TRAFFIC_FILE, ROOT))


def make_ic(N=N_GRID):
    """The rough lognormal state (sigma_ln = 1, Gaussian velocities), FP32-rounded;
    the FP64 runs start from the same values."""
    from paper_0907_3390_amd import workloads as wl
    g = wl.lognormal(N, seed=SEED, sigma_ln=1.0, vel_sigma_rel=0.3, P0=1.0, gamma=GAMMA)
    return g.astype(np.float32).astype(np.float64)


def make_blast(N=N_BLAST):
    """The point blast on a lognormal background (sigma_ln = 0.5, gas at rest,
    P = 1e-5, energy 1 in the central 2^3 cells), FP32-rounded."""
    from paper_0907_3390_amd import workloads as wl
    g = wl.sedov_lognormal(N, seed=SEED_BLAST, sigma_ln=0.5)
    return g.astype(np.float32).astype(np.float64)


def tune_stream(ctx, dev, candidates, reps=2):
    """Time one xyz/zyx pair (fused speed and sums, as in the timed step) per
    (chain length, second-sweep layout) candidate on the real state, after
    an untimed pair, writing a scratch buffer; keep the fastest."""
    import torch
    from paper_0907_3390_amd import tvd
    stream = torch.cuda.current_stream()
    dev.dt.fill_(CFL / dev.bs.n_blocks)  # any small dt: the state is not kept
    times = {}
    for L, flags in candidates:
        dev.set_chains(L)
        dev.kernel = flags
        state = dev.interior.clone()
        for r in range(reps + 1):
            if r == 1:
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
            for o in (0, 1):
                dev.advance(o, fuse_speed=o == 1, fuse_sums=True)
        b.record(stream)
        torch.cuda.synchronize()
        times[(L, flags)] = a.elapsed_time(b) / reps
        dev.interior.copy_(state)
        del state
    (L, flags), ms = min(times.items(), key=lambda kv: kv[1])
    dev.set_chains(L)
    dev.kernel = flags
    return {"chain_len": L, "second_sweep": second_sweep(flags, dev.dtype),
            "ms_per_pair": ms,
            "candidates_ms_per_pair": {
                f"chain {k[0]}, {'whole' if second_sweep(k[1], dev.dtype)[0] == 'w' else 'halves'}": v
                for k, v in times.items()}}


def second_sweep(flags, dtype):
    """The second-sweep layout the streamed advance runs for `flags`
    (TVD_KERNEL_AUTO: half pencils in FP32, whole pencils in FP64)."""
    import torch
    from paper_0907_3390_amd import tvd
    whole = flags == tvd.TVD_STREAM_WHOLE_B or (flags == tvd.TVD_KERNEL_AUTO and dtype == torch.float64)
    return "whole pencils" if whole else "half pencils"


def run_gpu(ctx, grid32, n, dtype, kernel, steps, warmup, gather=False, tune=False,
            p_floor=0.0, sums=False, stream=False, chain_len=None):
    """Warm up, then time `steps` steps (an even number) twice: eagerly with
    HIP events around every advance launch (for the kernel's average
    duration), and as replays of a HIP graph holding one xyz/zyx pair (for
    the step rate).  A step is the device time step on even steps, the
    advance (gathering ghost cells from the neighbours' interiors, or after
    a separate sibling fill), the fused signal speed on odd steps and, with
    `sums`, the fused FP64 compensated conservation sums on every step."""
    import torch
    from paper_0907_3390_amd import layout, tvd
    from paper_0907_3390_amd.driver import DeviceBlocks
    N = grid32.shape[3]
    # blocks numbered along a Morton curve: each XCD's contiguous share of the
    # blocks is a compact brick, so neighbours' ghost data meet in its L2
    bs = layout.periodic_grid_blockset(N, n, curve="morton")
    dev = DeviceBlocks(ctx, bs, dtype=dtype, gamma=GAMMA, cfl=CFL, kernel=kernel, gather=gather,
                       p_floor=p_floor, stream=stream, chain_len=chain_len)
    dev.upload(layout.grid_to_blocks(grid32, n, bs.perm))
    info = {"blocks": bs.n_blocks, "edge": n}
    if sums:
        # exact sums of the initial state (the reference for the drift)
        dev.conservation_sums()
        info["sums0"] = dev.sums.cpu().numpy().tolist()
    if stream and not tune:
        info["variant"] = {"chain_len": dev.chain_len, "second_sweep": second_sweep(kernel, dtype)}
    if tune and stream:
        col = N // n
        lens = sorted({L for L in (col // 4, col // 2, col) if 2 <= L <= 64})
        info["variant"] = tune_stream(ctx, dev, [(L, f) for L in lens
                                                 for f in (tvd.TVD_STREAM_HALF_B,
                                                           tvd.TVD_STREAM_WHOLE_B)])
        log(f"bench: streamed advance tuned {info['variant']}")
    elif tune:
        # pick the launch variant on the real data (scratch output), untimed
        dev.signal_speed()
        dev.set_dt_from_speed()
        scratch = dev.spare if gather else dev.interior.clone()
        src = dev.interior if gather else dev.ghosted
        if not gather:
            dev.fill_ghosts()
        idx, ms = ctx.tvd_autotune(dev.batch, dev.nbr if gather else None, src, scratch, GAMMA,
                                   p_floor=p_floor, reps=3)
        info["variant"] = dict(zip(("index", "edge", "threads", "lds_pad", "split"),
                                   tvd.variants()[idx]))
        info["variant"]["tuned_ms_per_pair"] = ms
        log(f"bench: tuned variant {info['variant']}")
    ctx.tvd_read_flags()
    for _ in range(warmup):
        dev.step(sums=sums)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    adv_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
    for k in range(steps):
        s = dev.step_index
        if s % 2 == 0:
            dev.set_dt_from_speed()
        if not gather:
            dev.fill_ghosts()
        adv_ev[k][0].record(stream)
        dev.advance(s % 2, fuse_speed=(s % 2 == 1), fuse_sums=sums)
        adv_ev[k][1].record(stream)
        dev.step_index += 1
    torch.cuda.synchronize()
    info["adv_ms"] = [a.elapsed_time(b) for a, b in adv_ev]
    # graph-captured pair, replayed steps/2 times
    side = torch.cuda.Stream()
    graph = dev.capture(2, stream=side, sums=sums)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(side)
    for _ in range(steps // 2):
        dev.replay(graph, stream=side)
    stop.record(side)
    torch.cuda.synchronize()
    info["wall_s"] = time.perf_counter() - t0
    info["total_ms"] = start.elapsed_time(stop)
    graph.close()
    info["steps_run"] = dev.step_index
    if sums:
        info["sums"] = dev.sums.cpu().numpy().tolist()
    st, info["floored"], info["nonphysical"] = ctx.tvd_read_flags()
    return dev, info


def run_uneven(ctx, graph_steps=50):
    """The uneven batch: 4000 independent periodic boxes (2286 of 8^3, 1143 of
    16^3, 571 of 32^3) with sound waves of amplitude 1e-3, FP32, gathering
    advance.  The block edge is chosen by measurement (every box as 8^3
    patches, or the 16^3 and 32^3 boxes as 16^3 patch groups in one persistent
    mixed-edge launch), then `graph_steps` steps are captured as one HIP graph
    and replayed; the mixed layout is also timed with one launch per edge."""
    import torch
    from paper_0907_3390_amd import layout, tvd, tuning, workloads as wl
    from paper_0907_3390_amd.driver import DeviceBlocks
    boxes = wl.sound_wave_boxes(seed=4)
    grids = [g.astype(np.float32).astype(np.float64) for g in boxes.grids]
    cells = sum(g.shape[1] ** 3 for g in grids)
    cands = {"all 8^3": lambda L: 8, "8^3 boxes as 8, others as 16^3 groups":
             lambda L: 8 if L == 8 else 16}
    best, times = tuning.tune_block_edge(ctx, grids, boxes.dh, cands, gamma=GAMMA, cfl=CFL)
    log(f"bench: uneven batch, block-edge tuner {times} -> {best}")
    res = {"workload": "4000 periodic boxes 2286 x 8^3 + 1143 x 16^3 + 571 x 32^3, sound waves "
                       "amplitude 1e-3, FP32, gathering advance, seed 4",
           "cells": cells, "block_edge_tuner_ms_per_step": times, "chosen_layout": best}
    for name, kernel in (("persistent", tvd.TVD_KERNEL_AUTO),
                         ("per_edge_launches", tvd.TVD_KERNEL_BATCHED)):
        if name == "per_edge_launches" and best == "all 8^3":
            continue
        dev = tuning.boxes_device(ctx, grids, boxes.dh, cands[best], kernel=kernel, gamma=GAMMA,
                                  cfl=CFL)
        dev.run(2)
        side = torch.cuda.Stream()
        g = dev.capture(graph_steps, stream=side)
        dev.replay(g, stream=side)  # untimed
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(side)
        dev.replay(g, stream=side)
        b.record(side)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        g.close()
        res[name] = {"value": cells * graph_steps / (ms * 1e-3), "unit": "cell-updates/s",
                     "ms_per_step": ms / graph_steps, "graph_steps": graph_steps,
                     "blocks": dev.bs.n_blocks}
        log(f"bench: uneven batch {name}: {res[name]['value'] / 1e9:.2f} G cell-updates/s")
        del dev
        torch.cuda.empty_cache()
    # the 571 boxes of 32^3 alone: each box one edge-32 block, streamed along
    # itself, against the same boxes as 16^3 groups (per-block gathering)
    big = [i for i, g in enumerate(grids) if g.shape[1] == 32]
    bg, bd = [grids[i] for i in big], [boxes.dh[i] for i in big]
    bcells = len(big) * 32 ** 3
    sub = {"boxes": len(big), "cells": bcells}
    for name, e, stream in (("edge32_streamed", 32, True), ("groups16_per_block", 16, False)):
        bs = layout.boxes_blockset([32] * len(bg), lambda L, e=e: e, bd)
        dev = DeviceBlocks(ctx, bs, dtype=torch.float32, gather=True, stream=stream,
                           gamma=GAMMA, cfl=CFL)
        dev.upload(layout.boxes_to_blocks(bg, lambda L, e=e: e))
        if not stream:
            dev.dt.fill_(CFL * float(np.min(bs.dh)) / 4.0)
            ctx.tvd_autotune(dev.batch, dev.nbr, dev.interior, dev.spare, GAMMA, reps=2)
        dev.run(2)
        ms = tuning.graph_ms_per_step(dev, pairs=10)
        sub[name] = {"value": bcells / (ms * 1e-3), "unit": "cell-updates/s", "ms_per_step": ms,
                     "blocks": bs.n_blocks}
        log(f"bench: uneven batch, 32^3 boxes {name}: {sub[name]['value'] / 1e9:.2f} G "
            f"cell-updates/s ({ms:.3f} ms per step)")
        del dev
        torch.cuda.empty_cache()
    res["boxes_32cube"] = sub
    st, fl, bad = ctx.tvd_read_flags()
    res["health"] = {"floored": fl, "nonphysical": bad}
    return res


def run_multilevel(ctx, ml, reps=10):
    """The multi-level batch: a 128^3 base of 8^3 patches and levels 1-3
    around 32 seeded overdensities (18 152 patches, properly nested, ghost
    zones pre-filled by sibling copy or trilinear coarse-to-fine
    interpolation), per-block dt_b = C dh_b / S computed on the device.
    Timed: one step of every patch as one persistent FP32 launch on the
    patches and on their 2^3 patch groups (16^3 blocks), against the plain
    FP64 kernel launched level by level."""
    import torch
    from paper_0907_3390_amd import tvd
    groups, G, gdh = ml.group_blocks()
    cells = len(ml.patches) * 512
    res = {"workload": "multi-level batch: 128^3 base + levels 1-3 around 32 Gaussian "
                       "overdensities (seed 3), ghosts pre-filled, gas at rest, P = 1",
           "patches": len(ml.patches), "patches_per_level": np.bincount(ml.levels).tolist(),
           "patch_groups": len(groups), "cells": cells}
    stream = torch.cuda.current_stream()
    for name, ghosted, dhs, levels, edge, dtype, kernel in (
            ("fp32_persistent_patches", ml.ghosted, ml.dh, ml.levels, 8, torch.float32,
             tvd.TVD_KERNEL_PERSISTENT),
            ("fp32_persistent_groups", G, gdh, np.array([g[0] for g in groups]), 16, torch.float32,
             tvd.TVD_KERNEL_PERSISTENT),
            ("fp64_plain_per_level", ml.ghosted, ml.dh, ml.levels, 8, torch.float64,
             tvd.TVD_KERNEL_PLAIN)):
        nb, m = len(dhs), edge + 6
        code = tvd.dtype_code(dtype)
        u_in = torch.from_numpy(np.ascontiguousarray(ghosted)).to(dtype).cuda().reshape(-1)
        u_out = torch.zeros(nb * 5 * edge ** 3, dtype=dtype, device="cuda")
        d_dh = torch.from_numpy(np.ascontiguousarray(dhs)).cuda()
        d_dt = torch.zeros(nb, dtype=torch.float64, device="cuda")
        smax = torch.zeros(1, dtype=torch.float64, device="cuda")
        b = tvd.Batch(code, nb, edge, d_dt=d_dt, d_dh=d_dh)
        ctx.tvd_reserve(nb)
        ctx.tvd_max_signal_speed(b, u_in, tvd.TVD_LAYOUT_GHOSTED, GAMMA, smax)
        ctx.tvd_dt_from_speed(b, smax, CFL, d_dt)
        if kernel == tvd.TVD_KERNEL_PLAIN:
            ranges = []
            for lev in np.unique(levels):
                ids = np.nonzero(levels == lev)[0]
                lo, hi = int(ids[0]), int(ids[-1]) + 1
                ranges.append((tvd.Batch(code, hi - lo, edge, d_dt=d_dt[lo:hi], d_dh=d_dh[lo:hi]),
                               u_in[lo * 5 * m ** 3:], u_out[lo * 5 * edge ** 3:]))

            def step(o):
                for bl, ui, uo in ranges:
                    ctx.tvd_patch_advance(bl, ui, uo, o, GAMMA, flags=kernel)
        else:
            def step(o):
                ctx.tvd_patch_advance(b, u_in, u_out, o, GAMMA, flags=kernel)
        for o in (0, 1):
            step(o)
        a = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for r in range(reps):
            step(r % 2)
        e.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(e) / reps
        res[name] = {"value": cells / (ms * 1e-3), "unit": "cell-updates/s", "ms_per_step": ms,
                     "blocks": nb, "block_edge": edge,
                     "launches_per_step": len(np.unique(levels)) if kernel == tvd.TVD_KERNEL_PLAIN else 1}
        log(f"bench: multi-level {name}: {res[name]['value'] / 1e9:.2f} G cell-updates/s")
        del u_in, u_out
        torch.cuda.empty_cache()
    res["speedup_fp32_groups_vs_fp64_plain"] = (res["fp32_persistent_groups"]["value"] /
                                                res["fp64_plain_per_level"]["value"])
    return res


def run_closing(ctx, ml, reps=10):
    """The closing step on the multi-level hierarchy (FP32, one dt on every
    level): the advance writing the patch-boundary flux records of every
    block (one persistent launch), then, level pair by level pair from the
    finest, the restriction of the fine blocks into their parents and the
    coarse-fine flux correction (six passes).  Timed with HIP events on the
    launch stream over `reps` steps: the advance with and without records,
    and the closing alone, as one launch per level pair (tvd_close_level) and
    as separate restriction and six correction passes.  The closing kernels are bound by HBM;
    their algorithmic bytes: restriction reads the fine interior and writes
    1/8 of it; correction reads and writes one coarse cell and reads one
    coarse and four fine fluxes per coarse face cell and variable."""
    import torch
    from paper_0907_3390_amd import layout, tvd
    res = {"workload": "multi-level batch (128^3 base, levels 1-3, 18 152 patches), FP32, one dt"}
    stream = torch.cuda.current_stream()
    groups, G, gdh = ml.group_blocks()
    for name, ghosted, dhs, edge in (("groups", G, gdh, 16), ("patches", ml.ghosted, ml.dh, 8)):
        tabs = ml.closing(edge)
        nb = len(dhs)
        cells = nb * edge ** 3
        u_in = torch.from_numpy(np.ascontiguousarray(ghosted)).float().cuda().reshape(-1)
        u_out = torch.zeros(nb * 5 * edge ** 3, dtype=torch.float32, device="cuda")
        flux = torch.zeros(nb * layout.flux_record_size(edge), dtype=torch.float32, device="cuda")
        d_dh = torch.from_numpy(np.ascontiguousarray(dhs)).cuda()
        sm = torch.zeros(1, dtype=torch.float64, device="cuda")
        ctx.tvd_reserve(nb)
        ctx.tvd_max_signal_speed(tvd.Batch(tvd.TVD_F32, nb, edge, d_dh=d_dh), u_in,
                                 tvd.TVD_LAYOUT_GHOSTED, GAMMA, sm)
        dt = CFL * float(np.min(dhs)) / float(sm.item())   # one dt on every level
        b = tvd.Batch(tvd.TVD_F32, nb, edge, dt=dt, d_dh=d_dh)
        dev = {}
        for lev, (rr, fr, cnt) in tabs.items():
            gr, gs = layout.group_face_rows(fr)
            dev[lev] = tuple(torch.from_numpy(a).cuda() for a in (rr, fr, gr, gs)) + (cnt,)

        def advance(o, rec):
            if rec:
                ctx.tvd_patch_advance_flux(b, u_in, u_out, flux, None, o, GAMMA,
                                           flags=tvd.TVD_KERNEL_PERSISTENT)
            else:
                ctx.tvd_patch_advance(b, u_in, u_out, o, GAMMA, flags=tvd.TVD_KERNEL_PERSISTENT)

        def close():
            # one launch per level pair, finest pair first
            for lev in sorted(dev, reverse=True):
                rr, fr, gr, gs, cnt = dev[lev]
                ctx.tvd_close_level(b, u_out, flux, None, b, u_out, flux, None, rr, gr, gs)

        def close_separate():
            # restriction, then six correction passes, per level pair
            for lev in sorted(dev, reverse=True):
                rr, fr, gr, gs, cnt = dev[lev]
                ctx.tvd_restrict(b, u_out, b, u_out, rr)
                ctx.tvd_flux_correct(b, u_out, flux, None, b, flux, None, fr, cnt)

        def timed(fn):
            fn(0)
            a = torch.cuda.Event(enable_timing=True)
            e = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for r in range(reps):
                fn(r % 2)
            e.record(stream)
            torch.cuda.synchronize()
            return a.elapsed_time(e) / reps

        ms_plain = timed(lambda o: advance(o, False))
        ms_flux = timed(lambda o: advance(o, True))
        ms_close = timed(lambda o: close())
        ms_close_sep = timed(lambda o: close_separate())
        n_rr = sum(len(v[0]) for v in tabs.values())
        n_fr = sum(len(v[1]) for v in tabs.values())
        h = edge // 2
        # algorithmic bytes of one closing (FP32)
        b_restrict = n_rr * 4 * 5 * (edge ** 3 + h ** 3)
        b_correct = n_fr * 4 * 5 * h * h * (2 + 1 + 4)
        rec_bytes = nb * 4 * layout.flux_record_size(edge)
        res[name] = {
            "blocks": nb, "block_edge": edge, "restrict_rows": n_rr, "face_rows": n_fr,
            "launches_per_closing": len(tabs),
            "closing_separate_calls_ms": ms_close_sep,
            "advance_ms": ms_plain, "advance_with_records_ms": ms_flux,
            "record_overhead": ms_flux / ms_plain - 1.0,
            "record_bytes_per_step": rec_bytes,
            "closing_ms": ms_close,
            "closing_algorithmic_bytes": b_restrict + b_correct,
            "closing_GBs": (b_restrict + b_correct) / (ms_close * 1e-3) / 1e9,
            "step_with_closing": {"value": cells / ((ms_flux + ms_close) * 1e-3),
                                  "unit": "cell-updates/s"},
        }
        log(f"bench: closing ({name}): advance {ms_plain:.3f} ms, with records {ms_flux:.3f} ms, "
            f"closing {ms_close:.3f} ms ({res[name]['closing_GBs']:.0f} GB/s algorithmic; "
            f"{ms_close_sep:.3f} ms as separate calls), "
            f"step {res[name]['step_with_closing']['value'] / 1e9:.2f} G cell-updates/s")
        del u_in, u_out, flux
        torch.cuda.empty_cache()
    return res


def run_nested(ctx, ml, reps=4, n=8, gather=False, stream_min_blocks=None,
               stream_chain_len=None, overlap=False):
    """The multi-level hierarchy advanced with every level sub-cycled (FP32,
    as 8^3 patches or, n = 16, as 2^3 patch groups): one root step is one
    step of level 0, two of level 1, four of level 2 and eight of level 3,
    each level closed with the next finer one after each of its steps
    (amr.NestedDevice).  Timed with HIP events
    over `reps` root steps run eagerly, and as replays of a HIP graph of two
    root steps (xyz, zyx).  Also reports the drift of the leaf totals over
    the timed steps (host sums of the downloaded state).  stream_min_blocks:
    levels of at least that many groups advance by the streamed kernel."""
    import torch
    from paper_0907_3390_amd import amr, layout, tvd
    refined = layout.NestedLevels.refined_from_patches(ml.base, ml.patches)
    top = len(refined)
    dev = amr.NestedDevice(ctx, ml.base, refined, dtype=torch.float32, n=n, gather=gather,
                           stream_min_blocks=stream_min_blocks, stream_chain_len=stream_chain_len,
                           overlap=overlap)
    L = dev.L
    interior = ml.ghosted[:, :, 3:11, 3:11, 3:11]
    per = [np.zeros((k, 5, n, n, n), dtype=np.float32) for k in dev.nb]
    # per-cell leaf mask: a patch's cells are leaves unless it is refined
    leaf = [np.ones((k, 1, n, n, n), dtype=bool) for k in dev.nb]
    for i, (l, px, py, pz) in enumerate(ml.patches):
        b, (ox, oy, oz) = L.locate(l, px, py, pz)
        per[l][b, :, oz:oz + 8, oy:oy + 8, ox:ox + 8] = interior[i]
        if l < top and refined[l][pz, py, px]:
            leaf[l][b, :, oz:oz + 8, oy:oy + 8, ox:ox + 8] = False
    dev.upload(per)

    def leaf_sums(blocks, f=lambda a: a):
        return sum((f(blocks[l].astype(np.float64)) * leaf[l]).sum(axis=(0, 2, 3, 4)) * 8.0 ** -l
                   for l in range(len(blocks)))
    before = leaf_sums(per)
    scale = leaf_sums(per, np.abs)
    sm = torch.zeros(1, dtype=torch.float64, device="cuda")
    u_in = torch.from_numpy(np.ascontiguousarray(ml.ghosted)).float().cuda().reshape(-1)
    d_dh = torch.from_numpy(np.ascontiguousarray(ml.dh)).cuda()
    ctx.tvd_reserve(len(ml.dh))
    ctx.tvd_max_signal_speed(tvd.Batch(tvd.TVD_F32, len(ml.dh), 8, d_dh=d_dh), u_in,
                             tvd.TVD_LAYOUT_GHOSTED, GAMMA, sm)
    dt = CFL * (1.0 / ml.base) / float(sm.item())
    del u_in
    stream = torch.cuda.current_stream()
    dev.step(dt, 0)
    dev.step(dt, 1)
    a = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for r in range(reps):
        dev.step(dt, r % 2)
    e.record(stream)
    torch.cuda.synchronize()
    ms_eager = a.elapsed_time(e) / reps
    ms_graph = None
    if not overlap:  # the overlapped driver is not captured (amr.NestedDevice.step)
        s = torch.cuda.Stream()
        s.wait_stream(stream)
        with torch.cuda.stream(s):
            ctx.tvd_graph_begin(s)
            for o in (0, 1):
                dev.step(dt, o)
            g = ctx.tvd_graph_end(s)
        torch.cuda.synchronize()
        try:
            g.replay(stream)
            a.record(stream)
            for r in range(reps // 2):
                g.replay(stream)
            e.record(stream)
            torch.cuda.synchronize()
            ms_graph = a.elapsed_time(e) / (2 * (reps // 2))
        finally:
            g.close()
    else:
        # as many root steps as the graph replays would have run
        for r in range(2 + 2 * (reps // 2)):
            dev.step(dt, r % 2)
    after = leaf_sums(dev.download())
    steps = 2 + reps + 2 + 2 * (reps // 2)
    updates = sum((1 << l) * k * n ** 3 for l, k in enumerate(dev.nb))
    # the gas starts at rest: momentum is measured against mass times the
    # largest signal speed
    scale[1:4] = scale[0] * float(sm.item())
    drift = float(np.max(np.abs(after - before) / scale))
    held = "18 152 patches of 8^3" if n == 8 else "2269 patch groups of 16^3"
    how = ("coarse-fine cells interpolated into stand-ins for missing siblings, ghost zones "
           "gathered by the advance" if gather else "ghosted copies filled before every advance")
    res = {"workload": f"multi-level hierarchy (128^3 base, levels 1-3, {held}), "
                       f"FP32, every level sub-cycled, every pair closed; {how}",
           "ghost_zones": "gathered" if gather else "ghosted copies",
           "streamed_levels": [lev for lev, c in enumerate(dev.chains) if c is not None],
           "levels_overlapped": overlap,
           "blocks_per_level": dev.nb, "block_edge": n, "cell_updates_per_root_step": updates,
           "root_step_ms_eager": ms_eager, "root_step_ms_graph": ms_graph,
           "value": updates / ((ms_graph or ms_eager) * 1e-3), "unit": "cell-updates/s",
           "root_steps_run": steps, "leaf_total_drift": drift}
    log(f"bench: nested sub-cycled step ({n}^3 blocks, gather {gather}, overlap {overlap}, "
        f"streamed levels {res['streamed_levels']}, chains of {stream_chain_len}): "
        f"{ms_eager:.3f} ms eager, "
        f"{ms_graph or float('nan'):.3f} ms as graph replay "
        f"per root step ({updates / 1e6:.1f} M cell-updates), {res['value'] / 1e9:.2f} G "
        f"cell-updates/s; leaf totals drift {drift:.1e} over {steps} root steps")
    return res


def run_poisson(ctx, reps=5, n_groups=4096):
    """Red-black SOR for the Poisson equation on patch groups (18^3 potential,
    16^3 density, Dirichlet ghosts): n_groups groups (the 2^3 patch groups of
    a 256^3 domain), lognormal densities, seeded.  Timed with HIP events:
    50 iterations per group (fixed count), and solves run to the stopping
    rule (optimal omega, 16 unit roundoffs), FP32 and FP64.  A cell update
    moves 4 LDS values (three neighbour reads and the write; the other three
    operands are in registers), which bounds the kernel: the LDS peak is
    128 B per clock per CU."""
    import torch
    from paper_0907_3390_amd import tvd
    r = np.random.default_rng(SEED + 7)
    rho = r.lognormal(0.0, 1.0, size=(n_groups, 16, 16, 16))
    c = (np.arange(-1, 17) + 0.5) / 16
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    phi = (np.sin(2 * x) * np.cos(3 * y) + 0.5 * z * z)[None] * r.uniform(0.5, 2.0, (n_groups, 1, 1, 1))
    lds_peak = 256 * 128 * 2.4e9
    res = {"workload": f"{n_groups} patch groups (16^3 + 1 ghost layer), lognormal density (seed {SEED + 7}), "
                       "Dirichlet ghosts from a smooth potential, G = 1, dh = 1/256"}
    stream = torch.cuda.current_stream()
    for name, dtype in (("fp32", torch.float32), ("fp64", torch.float64)):
        code = tvd.dtype_code(dtype)
        es = 4 if dtype == torch.float32 else 8
        p_in = torch.from_numpy(phi).to(dtype).cuda().reshape(-1)
        rh = torch.from_numpy(rho).to(dtype).cuda().reshape(-1)
        out = torch.zeros(n_groups * 4096, dtype=dtype, device="cuda")
        iters = torch.zeros(n_groups, dtype=torch.int32, device="cuda")

        def timed(**kw):
            ctx.tvd_poisson_sor(code, n_groups, p_in, rh, out, 1.0, 1.0 / 256, iters=iters, **kw)
            a = torch.cuda.Event(enable_timing=True)
            e = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                ctx.tvd_poisson_sor(code, n_groups, p_in, rh, out, 1.0, 1.0 / 256, iters=iters, **kw)
            e.record(stream)
            torch.cuda.synchronize()
            return a.elapsed_time(e) / reps

        ms_fixed = timed(min_iter=50, max_iter=50)
        updates = n_groups * 4096 * 50
        ms_conv = timed(max_iter=1000)
        it = iters.cpu().numpy()
        upd_conv = n_groups * 4096 * float(it.sum()) / n_groups
        res[name] = {
            "fixed_50_iterations_ms": ms_fixed,
            "cell_updates_per_s": updates / (ms_fixed * 1e-3),
            "lds_GBs": updates * 4 * es / (ms_fixed * 1e-3) / 1e9,
            "lds_frac": updates * 4 * es / (ms_fixed * 1e-3) / lds_peak,
            "converged_ms": ms_conv, "iterations_min_mean_max": [int(it.min()), float(it.mean()), int(it.max())],
            "converged_groups_per_s": n_groups / (ms_conv * 1e-3),
            "converged_cell_updates_per_s": upd_conv / (ms_conv * 1e-3),
        }
        log(f"bench: SOR {name}: {res[name]['cell_updates_per_s'] / 1e9:.1f} G cell-updates/s at 50 "
            f"iterations ({res[name]['lds_frac'] * 100:.0f} % of the LDS peak); to convergence "
            f"{ms_conv:.3f} ms for {n_groups} groups, {it.mean():.1f} iterations on average")
        del p_in, rh, out
        torch.cuda.empty_cache()
    return res


def run_gravity(ctx, grid32, reps=20):
    """The self-gravity operator G on the 256^3 state as 4096 groups of 16^3
    (FP32, in place), with a seeded potential of one ghost layer per group.
    HBM-bound: per cell it reads rho, m and e (5 values) and the potential,
    and writes m and e (4 values); the potential is read with its ghost layer
    ((18/16)^3 values per cell)."""
    import torch
    from paper_0907_3390_amd import layout, tvd
    n = 16
    u = torch.from_numpy(layout.grid_to_blocks(grid32, n)).float().cuda().reshape(-1)
    nb = (N_GRID // n) ** 3
    phi = torch.from_numpy(np.random.default_rng(SEED + 9).standard_normal((nb, 18, 18, 18))).float().cuda()
    b = tvd.Batch(tvd.TVD_F32, nb, n, dt=1e-9, dh=1.0 / N_GRID)
    stream = torch.cuda.current_stream()
    ctx.tvd_gravity(b, u, phi)
    a = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        ctx.tvd_gravity(b, u, phi)
    e.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(e) / reps
    cells = N_GRID ** 3
    alg = cells * 4 * (5 + 4) + nb * 18 ** 3 * 4
    del u, phi
    torch.cuda.empty_cache()
    res = {"workload": "256^3 lognormal state as 4096 groups of 16^3, FP32, seeded potential",
           "ms": ms, "cell_updates_per_s": cells / (ms * 1e-3),
           "algorithmic_bytes": alg, "GBs": alg / (ms * 1e-3) / 1e9,
           "hbm_frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    log(f"bench: gravity operator {ms:.3f} ms ({res['GBs']:.0f} GB/s, "
        f"{res['hbm_frac'] * 100:.0f} % of 8 TB/s)")
    return res


def run_amr_fill(ctx, reps=20):
    """Coarse-fine ghost fill (sibling copy, else Min-Mod limited linear
    interpolation from the coarser level): a periodic 256^3 coarse level
    (32768 patches of 8^3) under a fine box of 256^3 fine cells (a 128^3
    coarse region refined), cut into 8^3 patches and 16^3 patch groups.
    Reported per fill: ghosted cells written per second and the algorithmic
    bytes (ghosted blocks written, fine interiors and the coarse cells read
    once) over the fill time, against 8 TB/s."""
    import torch
    from paper_0907_3390_amd import layout, tvd, workloads as wl
    Nc = 256
    coarse_grid = wl.lognormal(Nc, seed=SEED, sigma_ln=1.0).astype(np.float32)
    origin, shape = (128, 128, 128), (256, 256, 256)
    fine = wl.smooth_random(256, seed=SEED + 1, amplitude=0.3).astype(np.float32)
    res = {"workload": "coarse 256^3 lognormal (32768 patches) under a 256^3-cell fine box "
                       "(fine origin 128 along each axis), FP32"}
    c_in = torch.from_numpy(layout.grid_to_blocks(coarse_grid, 8)).cuda().reshape(-1)
    for n in (8, 16):
        for curve in ("morton", "linear"):
            coarse_bs, fine_bs, cnbr, corigin = layout.two_level(Nc, origin, shape, n, curve=curve)
            m = n + 6
            nb = fine_bs.n_blocks
            f_in = torch.from_numpy(layout.grid_to_blocks(fine, n, fine_bs.perm)).cuda().reshape(-1)
            f_gh = torch.empty(nb * 5 * m ** 3, dtype=torch.float32, device="cuda")
            nbr = torch.from_numpy(fine_bs.nbr).cuda()
            cn = torch.from_numpy(cnbr).cuda()
            co = torch.from_numpy(corigin).cuda()
            fb = tvd.Batch(tvd.TVD_F32, nb, n, dt=1e-3, dh=0.5 / Nc)
            cb = tvd.Batch(tvd.TVD_F32, coarse_bs.n_blocks, 8, dt=1e-3, dh=1.0 / Nc)
            ctx.tvd_fill_ghosts_amr(fb, nbr, f_in, f_gh, cb, c_in, cn, co)
            a = torch.cuda.Event(enable_timing=True)
            e = torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                ctx.tvd_fill_ghosts_amr(fb, nbr, f_in, f_gh, cb, c_in, cn, co)
            e.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(e) / reps
            # cells interpolated: ghost cells of blocks on the box surface
            ghost_cells = nb * (m ** 3 - n ** 3)
            bytes_alg = nb * m ** 3 * 20 + nb * n ** 3 * 20 + (128 + 4) ** 3 * 20
            key = f"edge{n}" if curve == "morton" else f"edge{n}_linear_numbering"
            res[key] = {"blocks": nb, "block_order": curve, "ms": ms,
                        "ghosted_cells_per_s": nb * m ** 3 / (ms * 1e-3),
                        "ghost_cells": ghost_cells,
                        "algorithmic_GBs": bytes_alg / (ms * 1e-3) / 1e9,
                        "hbm_frac": bytes_alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
            log(f"bench: coarse-fine ghost fill, edge {n}, {curve} numbering: {ms:.3f} ms, "
                f"{res[key]['algorithmic_GBs']:.0f} GB/s algorithmic")
            del f_in, f_gh
            torch.cuda.empty_cache()
    st, fl, bad = ctx.tvd_read_flags()
    res["health"] = {"nonphysical": bad}
    return res


def run_host_pipeline_bench(ctx, grid32, reps=3):
    """The host-resident advance (tvd_patch_advance_host) of the 256^3 level
    as 4096 patch groups of 16^3 held in host memory, FP32.

    table1: one launch of 1024 groups (the paper's GPU solver call of N_s x
    N_g groups) with N_s = 1, 2, 4, 8 streams: per group, the copy down, the
    advance and the copy up as each stream sees them, the GPU's span, and
    the transfer time as a share of the advance time (exposed: span minus
    advance); the preparation and closing steps are not in these figures, as
    in the paper's hydrodynamic timing table.
    level: the whole level in four launches of N_s = 4 x N_g = 256 groups,
    with the host's preparation and closing steps overlapped with the GPU
    (Sec. 3.5) or not: wall time and host-inclusive cell-updates/s."""
    import torch
    from paper_0907_3390_amd import layout, tvd
    n, N = 16, grid32.shape[3]
    bs = layout.periodic_grid_blockset(N, n, curve="morton")
    u = bs.pack_interior(layout.grid_to_blocks(grid32, n, bs.perm)).astype(np.float32)
    out = np.empty_like(u)
    batch = tvd.Batch(tvd.TVD_F32, bs.n_blocks, n, dt=0.2 / N, dh=1.0 / N)
    threads = max(1, min(16, os.cpu_count() or 1))
    res = {"workload": f"{N}^3 lognormal level as {bs.n_blocks} patch groups of 16^3 in host "
                       f"memory (pageable), FP32", "host_threads": threads,
           "staging": "page-locked host staging (torch pin_memory), device staging per stream"}

    def run(ns, ng, concurrent, nblocks):
        streams = [torch.cuda.Stream() for _ in range(ns)]
        pipe = tvd.HostPipeline(streams, ng, threads, concurrent)
        hb, db = pipe.stage_bytes(tvd.TVD_F32, n)
        pipe.attach(torch.empty(hb, dtype=torch.uint8, pin_memory=True),
                    torch.empty(db, dtype=torch.uint8, device="cuda"))
        b = tvd.Batch(tvd.TVD_F32, nblocks, n, dt=0.2 / N, dh=1.0 / N)
        nbr = np.ascontiguousarray(bs.nbr[:nblocks]) if nblocks < bs.n_blocks else bs.nbr
        if nblocks < bs.n_blocks:
            # the first nblocks groups with their neighbours folded into the
            # subset (a copy pattern of the same size; the values are not kept)
            nbr = np.ascontiguousarray(nbr % nblocks).astype(np.int32)
        best = None
        for _ in range(reps + 1):
            _, t = ctx.tvd_patch_advance_host(b, nbr, u, out, pipe, 0, GAMMA, 0.0, times=True)
            if best is None or t["wall"] < best["wall"]:
                best = t
        return best

    table = {}
    per_launch = 1024
    for ns in (1, 2, 4, 8):
        t = run(ns, per_launch // ns, False, per_launch)
        g = per_launch
        table[f"N_s={ns}"] = {
            "N_g": per_launch // ns,
            "copy_down_us_per_group": 1e3 * t["copy_down"] / g,
            "advance_us_per_group": 1e3 * t["advance"] / g,
            "copy_up_us_per_group": 1e3 * t["copy_up"] / g,
            "gpu_span_us_per_group": 1e3 * t["gpu_span"] / g,
            "transfer_share_of_advance": (t["copy_down"] + t["copy_up"]) / t["advance"],
            "exposed_transfer_share_of_advance": (t["gpu_span"] - t["advance"]) / t["advance"],
            "host_prepare_ms": t["host_prepare"], "host_close_ms": t["host_close"]}
        log(f"bench: host pipeline N_s={ns}: span {t['gpu_span']:.2f} ms, advance "
            f"{t['advance']:.2f} ms, down {t['copy_down']:.2f} ms, up {t['copy_up']:.2f} ms")
    res["table1"] = table
    res["table1_bytes"] = {"down_per_group": 5 * 22 ** 3 * 4, "up_per_group": 5 * 16 ** 3 * 4}
    level = {}
    for concurrent in (False, True):
        t = run(4, 256, concurrent, bs.n_blocks)
        level["concurrent" if concurrent else "sequential"] = {
            "wall_ms": t["wall"], "cell_updates_per_s": N ** 3 / (t["wall"] * 1e-3),
            "host_prepare_ms": t["host_prepare"], "host_close_ms": t["host_close"],
            "copy_down_ms": t["copy_down"], "advance_ms": t["advance"], "copy_up_ms": t["copy_up"],
            "gpu_span_ms": t["gpu_span"]}
        log(f"bench: host pipeline level, concurrent={concurrent}: {t['wall']:.1f} ms")
    level["overlap_saving"] = 1.0 - level["concurrent"]["wall_ms"] / level["sequential"]["wall_ms"]
    res["level_N_s4_N_g256"] = level
    res["paper_context"] = {
        "note": "the paper's hydrodynamic solver per patch group (Tesla T10 / 8800 GTX, PCIe "
                "gen 1-2), context only",
        "kernel_us_per_group": {"GraCCA": 252, "NCHC": 144, "CQSE": 150},
        "copy_down_us_per_group": {"GraCCA": 71, "NCHC": 51, "CQSE": 44},
        "copy_up_us_per_group": {"GraCCA": 46, "NCHC": 64, "CQSE": 29},
        "transfer_share_one_stream": {"GraCCA": 0.464, "NCHC": 0.799, "CQSE": 0.487},
        "transfer_share_four_streams": {"NCHC": 0.229, "CQSE": 0.180}}
    return res


def host_cpu():
    """Model name and logical CPU count of the host, and the OpenMP thread
    count the oracle is run with."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count(),
            "omp_num_threads": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))}


def native_oracle():
    """Build the C oracle for this host's CPU (-O3 -march=native) into a
    temporary directory and bind it; the arithmetic is the same C source
    with FP contraction off.  Returns the compile flags used, or the shipped
    build's if gcc is not usable here."""
    import tempfile

    import oracle
    out = os.path.join(tempfile.mkdtemp(prefix="oracle_native_"), "liboracle.so")
    try:
        oracle.build(out=out, native=True)
        oracle.use_library(out)
        return " ".join(oracle.CFLAGS_NATIVE)
    except Exception as e:  # the shipped build stays in use
        log(f"bench: native oracle build failed ({e}); using the shipped build")
        return " ".join(oracle.CFLAGS)


def sample_ghosted_blocks(grid, n, picks):
    """Ghosted blocks (edge n + 6) of the periodic grid for the x-fastest
    block indices `picks`, cut straight from the grid with periodic wrap."""
    _, Nz, Ny, Nx = grid.shape
    nbx, nby = Nx // n, Ny // n
    out = np.empty((len(picks), 5, n + 6, n + 6, n + 6))
    for i, b in enumerate(picks):
        bx, by, bz = b % nbx, (b // nbx) % nby, b // (nbx * nby)
        iz = np.arange(bz * n - 3, bz * n + n + 3) % Nz
        iy = np.arange(by * n - 3, by * n + n + 3) % Ny
        ix = np.arange(bx * n - 3, bx * n + n + 3) % Nx
        out[i] = grid[(slice(None),) + np.ix_(iz, iy, ix)]
    return out


def cpu_baseline(grid, p_floor, budget_s=15.0, sample_blocks=16384):
    """The FP64 oracle (as it stands, built for this host) on the host cores
    over a bounded sample of the same workload: `sample_blocks` 8^3 patches
    of the initial state with their ghost zones cut from the periodic grid,
    advanced by one step (alternating xyz / zyx) at a time, repeated until
    `budget_s` seconds of advance have run; then one step of 2048 of them on
    one thread.  Only the advance is timed, like the GPU's kernel."""
    import oracle
    flags = native_oracle()
    N = grid.shape[3]
    dh = 1.0 / N
    nb_all = (N // 8) ** 3
    picks = np.sort(np.random.default_rng(SEED).choice(nb_all, size=min(sample_blocks, nb_all),
                                                       replace=False))
    blocks = sample_ghosted_blocks(grid.astype(np.float64), 8, picks)
    dt = CFL * dh / oracle.max_signal_speed(grid.astype(np.float64), GAMMA, p_floor)
    threads = host_cpu()["omp_num_threads"]
    oracle.set_threads(threads)
    steps = 0
    c = oracle.Counts()
    while c.seconds < budget_s and steps < 50:
        oracle.advance_blocks(blocks, steps % 2, dt, dh, GAMMA, p_floor, counts=c)
        steps += 1
    used, adv = c.threads, c.seconds
    oracle.set_threads(1)
    c1 = oracle.Counts()
    oracle.advance_blocks(blocks[:2048], 0, dt, dh, GAMMA, p_floor, counts=c1)
    t1 = c1.seconds
    oracle.set_threads(threads)
    cpu = host_cpu()
    return {"value": steps * len(picks) * 512 / adv, "unit": "cell-updates/s", "cores": used,
            "kind": "oracle",
            "sample": f"{len(picks)} of the {nb_all} 8^3 patches of the initial state (seeded "
                      f"pick, ghost zones cut from the periodic grid), one FP64 step repeated "
                      f"{steps} times, {adv:.1f} s inside the C advance timed (ghost cut, "
                      f"marshalling and CFL speed not timed)",
            "host": cpu, "oracle_cflags": flags,
            "single_thread": {"value": 2048 * 512 / t1, "unit": "cell-updates/s", "cores": 1,
                              "sample": "one step of 2048 of the sampled patches, FP64"}}


def copy_bandwidth(nbytes=1 << 30, reps=5):
    """Measured device-to-device copy rate (read + write bytes per second) of
    a plain copy of known size, for comparison with the 8 TB/s peak."""
    import torch
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        y.copy_(x)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del x, y
    return {"bytes_per_copy": nbytes, "read_plus_write_GBs": 2 * nbytes / (ms * 1e-3) / 1e9,
            "ms": ms}


def whole_pairs(k: int, least: int) -> int:
    """Steps come in xyz/zyx pairs sharing one dt: round up to a whole pair."""
    return max(least, k + (k % 2))


def l1_norms(a, b):
    """Relative L1 per variable of a against reference b, both (5, ...):
    rho and e on their own norm, momentum on the sum of rho c_s (and on its
    own norm)."""
    nrm = {}
    for k, nm in enumerate(["rho", "m_x", "m_y", "m_z", "e"]):
        nrm[nm] = float(np.abs(a[k] - b[k]).sum() / np.abs(b[k]).sum())
    rho = b[0]
    kin = 0.5 * (b[1] ** 2 + b[2] ** 2 + b[3] ** 2) / rho
    cs = np.sqrt(GAMMA * np.maximum((GAMMA - 1) * (b[4] - kin), 0) / rho)
    scale = (rho * cs).sum()
    for k, nm in enumerate(["m_x", "m_y", "m_z"]):
        nrm[nm + "_scale"] = float(np.abs(a[k + 1] - b[k + 1]).sum() / scale)
    return nrm


def download_grid(dev, shape):
    """The device state as a (5, Nz, Ny, Nx) FP64 grid."""
    from paper_0907_3390_amd import layout
    return layout.blocks_to_grid(np.stack(dev.download()).astype(np.float64), shape, dev.bs.perm)


def compare_fp32_fp64(ctx, g32, grid, steps, warmup, p_floor, sums, label):
    """The plain FP64 per-patch kernel over the same steps from the same
    FP32-rounded state, and the L1 error of the FP32 result g32 against it."""
    import torch
    from paper_0907_3390_amd import layout, tvd
    N = grid.shape[3]
    log(f"bench: {label}: FP64 plain, edge 8, {warmup}+{steps}+{steps} steps")
    dev64, r64 = run_gpu(ctx, grid, 8, torch.float64, tvd.TVD_KERNEL_PLAIN, steps, warmup,
                         p_floor=p_floor, sums=sums)
    v64 = N ** 3 * steps / (r64["total_ms"] * 1e-3)
    g64 = download_grid(dev64, (5, N, N, N))
    del dev64
    torch.cuda.empty_cache()
    nrm = l1_norms(g32, g64)
    nrm["after_steps"] = r64["steps_run"]
    res = {"value": v64, "unit": "cell-updates/s", "ms_per_step": r64["total_ms"] / steps,
           "avg_launch_ms": float(np.mean(r64["adv_ms"])), "blocks": r64["blocks"],
           "block_edge": 8, "health": {"floored": r64["floored"],
                                       "nonphysical": r64["nonphysical"]}}
    log(f"bench: {label}: FP64 plain {v64 / 1e9:.3f} G cell-updates/s; relL1 {nrm}")
    return res, nrm, g64


def headline_record(r, cells, steps, n, label, workload, stream_planes=None):
    """Throughput, roofline and health of one FP32 gathering-advance run
    (per-block kernel, or streamed over chains of `stream_planes` planes)."""
    value = cells * steps / (r["total_ms"] * 1e-3)
    nb = r["blocks"]
    # algorithmic bytes of one launch: the ghosted block in (gathered from the
    # neighbours' interiors) and the interior out
    bytes_launch = nb * ((n + 6) ** 3 + n ** 3) * 5 * 4
    adv_avg_ms = float(np.mean(r["adv_ms"]))
    achieved = bytes_launch / (adv_avg_ms * 1e-3) / 1e9
    if stream_planes:
        flops_launch = int(cells * flops_per_cell_stream(stream_planes))
    else:
        flops_launch = nb * flops_per_block(n)
    tflops = flops_launch / (adv_avg_ms * 1e-3) / 1e12
    rec = {"value": value, "unit": "cell-updates/s", "ms_per_step": r["total_ms"] / steps,
           "workload": workload, "blocks": nb, "block_edge": n,
           "advance_cell_updates_per_s": cells / (adv_avg_ms * 1e-3),
           "avg_launch_ms": adv_avg_ms, "algorithmic_flops_per_launch": flops_launch,
           "algorithmic_bytes_per_launch": bytes_launch,
           "TFLOPs": tflops, "GBs": achieved,
           "variant": r.get("variant"),
           "health": {"floored": r["floored"], "nonphysical": r["nonphysical"]}}
    log(f"bench: {label}: {value / 1e9:.2f} G cell-updates/s, advance {adv_avg_ms:.3f} ms "
        f"({achieved:.0f} GB/s, {tflops:.1f} TFLOP/s)")
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--headline-only", action="store_true",
                    help="only the 512^3 headline run (for profiling)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 plain comparisons")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-variant tuner")
    ap.add_argument("--no-config2", action="store_true", help="skip the 256^3 lognormal runs")
    ap.add_argument("--chain-len", type=int, default=None,
                    help="with --no-tune: chain length of the streamed headline run")
    ap.add_argument("--whole-b", action="store_true",
                    help="with --no-tune: second sweep in whole pencils in the headline run")
    ap.add_argument("--per-block", action="store_true",
                    help="with --headline-only: also time the per-block advance (profiling)")
    ap.add_argument("--extras", action="store_true",
                    help="also run the ghost fill, multi-level, closing, nested, Poisson, "
                         "gravity and uneven-batch measurements")
    ap.add_argument("--only", choices=["amr_fill", "nested", "uneven", "gravity"], default=None,
                    help="run only this measurement and print its record (profiling)")
    args = ap.parse_args()
    if args.only:
        import torch
        from paper_0907_3390_amd import tvd, workloads as wl
        assert torch.cuda.is_available(), "bench.py needs a GPU"
        ctx = tvd.Context(0)
        if args.only == "nested":
            ml = wl.multilevel()
            rec = {"nested_subcycled_step": run_nested(ctx, ml, n=16, gather=True),
                   "overlapped_levels": run_nested(ctx, ml, n=16, gather=True, overlap=True),
                   "ghosted_copies": run_nested(ctx, ml, n=16)}
        elif args.only == "uneven":
            rec = {"uneven_batch": run_uneven(ctx)}
        elif args.only == "gravity":
            rec = {"gravity_operator": run_gravity(ctx, make_ic().astype(np.float32))}
        else:
            rec = {"amr_ghost_fill": run_amr_fill(ctx)}
        ctx.close()
        print(json.dumps(rec), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    steps = whole_pairs(args.steps, 2)
    warmup = whole_pairs(args.warmup, 2)
    if (steps, warmup) != (args.steps, args.warmup):
        log(f"bench: steps/warmup {args.steps}/{args.warmup} rounded up to whole xyz/zyx pairs: "
            f"{steps}/{warmup}")

    import torch
    from paper_0907_3390_amd import tvd
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    ctx = tvd.Context(0)
    t_start = time.perf_counter()

    # ---- headline: 512^3 point blast, FP32 patch groups, FP64 sums every step
    log(f"bench: building the {N_BLAST}^3 point-blast state (seed {SEED_BLAST})")
    grid5 = make_blast()
    cells5 = N_BLAST ** 3
    n = 16
    wl5 = (f"{N_BLAST}^3 periodic grid = {(N_BLAST // 8) ** 3} patches of 8^3 run as "
           f"{(N_BLAST // 16) ** 3} Morton-ordered 2^3 patch groups of 16^3; point blast (energy 1 "
           f"in the central 2^3 cells) on a lognormal background sigma_ln=0.5 at rest, P=1e-5, "
           f"gamma=5/3, CFL 0.5, p_floor 1e-10, seed {SEED_BLAST}")
    log(f"bench: headline FP32, edge {n}, streamed advance, {warmup}+{steps}+{steps} steps, "
        f"sums every step")
    dev5, r5 = run_gpu(ctx, grid5, n, torch.float32,
                       tvd.TVD_STREAM_WHOLE_B if args.whole_b else tvd.TVD_KERNEL_AUTO, steps,
                       warmup, gather=True, tune=not args.no_tune, p_floor=P_FLOOR_BLAST,
                       sums=True, stream=True, chain_len=args.chain_len)
    planes5 = dev5.chain_len * n
    head = headline_record(r5, cells5, steps, n, "512^3 blast FP32 streamed", wl5,
                           stream_planes=planes5)
    value = head["value"]
    traffic, traffic_note = measured_traffic(r5.get("variant"))
    # conservation drift of the fused FP64 sums after all steps run
    s0, s1 = np.array(r5["sums0"]), np.array(r5["sums"])
    drift = {nm: float(abs(s1[k] - s0[k]) / abs(s0[k]))
             for k, nm in enumerate(["rho", "m_x", "m_y", "m_z", "e"]) if k in (0, 4)}
    drift["momentum_over_mass"] = float(np.max(np.abs(s1[1:4] - s0[1:4])) / abs(s0[0]))
    out = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "steps_requested": args.steps,
        "warmup_requested": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl5, "cells": cells5, "blocks": head["blocks"], "block_edge": n,
                   "precision": "fp32 state and arithmetic; fp64 dt, signal speed and "
                                "compensated conservation sums",
                   "ghost_zones": "gathered from the 26 neighbours inside the advance",
                   "schedule": f"streamed: chains of {dev5.chain_len} blocks along the axis swept "
                               f"last (z forward, x backward), 16 x 16 tiles, slabs of 8 planes",
                   "step": "device dt (even steps), advance, fused signal speed (odd steps), "
                           "fused FP64 compensated sums (every step)",
                   "block_order": "Morton curve"},
        "roofline": {"bound": "alu", "achieved": head["TFLOPs"], "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": head["TFLOPs"] / FP32_PEAK_TFLOPS,
                     "traffic": traffic, "traffic_source": traffic_note,
                     "peak_note": "FP32 vector without packed FP32 (packed instructions are off "
                                  "in this build); 157.3 TFLOP/s with packed FP32",
                     "frac_of_packed_peak": head["TFLOPs"] / 157.3,
                     "kernel": f"k_stream<float,{n}>",
                     "avg_launch_ms": head["avg_launch_ms"],
                     "algorithmic_flops_per_launch": head["algorithmic_flops_per_launch"],
                     "algorithmic_flops_per_cell_update": flops_per_cell_stream(planes5),
                     "flops_note": "the streamed schedule's own region-rule work (first two "
                                   "sweeps on 22 + 16 pencils per plane and tile, third sweep "
                                   "once per cell); the per-block schedule on 16^3 groups needs "
                                   f"{flops_per_block(16) / 4096:.0f} flop per cell-update",
                     "hbm": {"achieved": head["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": head["GBs"] / HBM_PEAK_GBS,
                             "algorithmic_bytes_per_launch": head["algorithmic_bytes_per_launch"]}},
        "advance_cell_updates_per_s": head["advance_cell_updates_per_s"],
        "timing": "steps replayed as a HIP graph of one xyz/zyx pair; advance duration from "
                  "HIP events on the launch stream around eager launches of the same steps",
        "variant": head["variant"], "health": head["health"],
        "conservation_drift_after_run": drift,
    }
    g32 = download_grid(dev5, grid5.shape) if not args.headline_only else None
    del dev5
    torch.cuda.empty_cache()
    # the per-block gathering advance on the same state and step, for comparison
    if not args.headline_only or args.per_block:
        log("bench: 512^3 blast FP32, per-block gathering advance for comparison")
        dpb, rpb = run_gpu(ctx, grid5, n, torch.float32, tvd.TVD_KERNEL_AUTO, steps, warmup,
                           gather=True, tune=not args.no_tune, p_floor=P_FLOOR_BLAST, sums=True)
        pb = headline_record(rpb, cells5, steps, n, "512^3 blast FP32 per-block", wl5)
        if g32 is not None:
            same = np.array_equal(download_grid(dpb, grid5.shape), g32)
            pb["bitwise_equal_to_streamed"] = bool(same)
        out["per_block_gather"] = pb
        out["speedup_streamed_vs_per_block"] = value / pb["value"]
        del dpb
        torch.cuda.empty_cache()
    # a plain copy of known size: the peak measured on this machine, and the
    # calibration of the HBM counters when this run is profiled
    out["hbm_copy_measured"] = copy_bandwidth()
    out["roofline"]["hbm"]["frac_of_measured_copy"] = (
        head["GBs"] / out["hbm_copy_measured"]["read_plus_write_GBs"])
    log(f"bench: plain 1 GiB copy {out['hbm_copy_measured']['read_plus_write_GBs']:.0f} GB/s")
    if not args.no_fp64 and not args.headline_only:
        res64, nrm, g64 = compare_fp32_fp64(ctx, g32, grid5, steps, warmup, P_FLOOR_BLAST, True,
                                            "512^3 blast")
        del g64
        out["fp64_plain"] = res64
        out["speedup_fp32_batched_vs_fp64_plain"] = value / res64["value"]
        out["l1_vs_fp64"] = nrm
    del g32
    torch.cuda.empty_cache()

    # ---- 256^3 rough lognormal grid: FP32 vs FP64 plain, FP64 batched, FP32 on patches
    if not args.no_config2 and not args.headline_only:
        grid2 = make_ic()
        wl2 = ("256^3 periodic grid = 32768 patches of 8^3, lognormal rho sigma_ln=1, Gaussian v "
               "sigma=0.3 c_s, P=1, gamma=5/3, CFL 0.5, seed 2024")
        log("bench: 256^3 lognormal FP32, edge 16, streamed advance")
        dev2, r2 = run_gpu(ctx, grid2, 16, torch.float32, tvd.TVD_KERNEL_AUTO, steps, warmup,
                           gather=True, tune=not args.no_tune, sums=True, stream=True)
        c2 = headline_record(r2, N_GRID ** 3, steps, 16, "256^3 lognormal FP32 streamed",
                             wl2 + " (run as 4096 2^3 patch groups of 16^3)",
                             stream_planes=dev2.chain_len * 16)
        g2_32 = download_grid(dev2, grid2.shape)
        del dev2
        torch.cuda.empty_cache()
        log("bench: 256^3 lognormal FP32, per-block gathering advance")
        dpb, rpb = run_gpu(ctx, grid2, 16, torch.float32, tvd.TVD_KERNEL_AUTO, steps, warmup,
                           gather=True, tune=not args.no_tune, sums=True)
        c2["per_block_gather"] = headline_record(rpb, N_GRID ** 3, steps, 16,
                                                 "256^3 lognormal FP32 per-block", wl2)
        c2["per_block_gather"]["bitwise_equal_to_streamed"] = bool(
            np.array_equal(download_grid(dpb, grid2.shape), g2_32))
        del dpb
        torch.cuda.empty_cache()
        if not args.no_fp64:
            res64, nrm, g64 = compare_fp32_fp64(ctx, g2_32, grid2, steps, warmup, 0.0, True,
                                                "256^3 lognormal")
            c2["fp64_plain"] = res64
            c2["speedup_fp32_batched_vs_fp64_plain"] = c2["value"] / res64["value"]
            c2["l1_vs_fp64"] = nrm
            for name, dtype, e, strm in (("fp64_streamed_edge16", torch.float64, 16, True),
                                         ("fp64_batched", torch.float64, 8, False),
                                         ("fp32_batched_edge8", torch.float32, 8, False)):
                log(f"bench: 256^3 lognormal {name}, edge {e}")
                dv, rr = run_gpu(ctx, grid2, e, dtype, tvd.TVD_KERNEL_AUTO, steps, warmup,
                                 gather=True, tune=not args.no_tune, sums=True, stream=strm)
                c2[name] = {"value": N_GRID ** 3 * steps / (rr["total_ms"] * 1e-3),
                            "unit": "cell-updates/s", "ms_per_step": rr["total_ms"] / steps,
                            "avg_launch_ms": float(np.mean(rr["adv_ms"])),
                            "blocks": rr["blocks"], "block_edge": e, "variant": rr.get("variant")}
                if dtype == torch.float64:
                    from paper_0907_3390_amd import layout
                    gb = layout.blocks_to_grid(np.stack(dv.download()), g64.shape, dv.bs.perm)
                    c2[name]["max_rel_diff_vs_fp64_plain"] = float(
                        max(np.abs(gb[k] - g64[k]).max() / np.abs(g64[k]).max() for k in range(5)))
                del dv
                torch.cuda.empty_cache()
                log(f"bench: {name} {c2[name]['value'] / 1e9:.3f} G cell-updates/s")
            del g64
        log("bench: host-resident pipeline (N_s streams) on the 256^3 level")
        c2["host_pipeline"] = run_host_pipeline_bench(ctx, grid2)
        del g2_32
        out["lognormal_256cube"] = c2
        torch.cuda.empty_cache()

    if args.extras and not args.headline_only:
        grid2 = make_ic()
        log("bench: coarse-fine ghost fill")
        out["amr_ghost_fill"] = run_amr_fill(ctx)
        from paper_0907_3390_amd import workloads as wl
        log("bench: building the multi-level hierarchy")
        ml = wl.multilevel()
        log("bench: multi-level batch")
        torch.cuda.empty_cache()
        out["multilevel_batch"] = run_multilevel(ctx, ml)
        log("bench: closing step on the multi-level hierarchy")
        torch.cuda.empty_cache()
        out["closing_step"] = run_closing(ctx, ml)
        log("bench: nested sub-cycled step on the multi-level hierarchy")
        torch.cuda.empty_cache()
        out["nested_subcycled_step"] = run_nested(ctx, ml, n=16, gather=True)
        out["nested_subcycled_step"]["groups_ghosted_copies"] = run_nested(ctx, ml, n=16)
        # each level on its own stream, a level's first sub-step beside its
        # parent's advance (eager steps only: this driver is not captured)
        out["nested_subcycled_step"]["groups_overlapped_levels"] = run_nested(
            ctx, ml, n=16, gather=True, overlap=True)
        # levels 0-2 by the streamed advance with flux records, chains of 2
        # blocks (slower here: few chains per level, see the design notes)
        out["nested_subcycled_step"]["groups_streamed_levels"] = run_nested(
            ctx, ml, n=16, gather=True, stream_min_blocks=512, stream_chain_len=2)
        out["nested_subcycled_step"]["patches_8cube"] = run_nested(ctx, ml, n=8, gather=True)
        log("bench: Poisson SOR on patch groups")
        torch.cuda.empty_cache()
        out["poisson_sor"] = run_poisson(ctx)
        out["gravity_operator"] = run_gravity(ctx, grid2.astype(np.float32))
        log("bench: uneven batch of 4000 boxes")
        torch.cuda.empty_cache()
        out["uneven_batch"] = run_uneven(ctx)
    out["gpu_wall_s"] = time.perf_counter() - t_start

    if not args.no_cpu_baseline and not args.headline_only:
        log("bench: FP64 oracle on the host cores (bounded sample of the 512^3 blast)")
        out["cpu_baseline"] = cpu_baseline(grid5, P_FLOOR_BLAST)
        cb = out["cpu_baseline"]
        log(f"bench: oracle {cb['value'] / 1e6:.2f} M cell-updates/s on {cb['cores']} threads, "
            f"{cb['single_thread']['value'] / 1e6:.2f} M on one")
        out["paper_context"] = {
            "note": "context only: the paper's GPU/CPU ratios on its own hardware and workloads",
            "paper": {"whole_code_1gpu_vs_1cpu_max_sustained": 12.19,
                      "whole_code_setting": "purely-baryonic cosmological run, 128^3 root, 5 levels "
                                            "(4096^3 effective), GeForce 8800 GTX vs one core of an "
                                            "AMD Athlon 64 X2 3800 (GraCCA); 10.78 and 10.07 on Tesla "
                                            "T10 vs Xeon E5520 / E5462 (NCHC, CQSE)",
                      "hydro_solver_1gpu_vs_1cpu": {"GraCCA": 14.6, "NCHC": 13.4, "CQSE": 15.3}},
            "here": {"fp32_batched_vs_oracle_one_thread": value / cb["single_thread"]["value"],
                     "fp32_batched_vs_oracle_all_threads": value / cb["value"],
                     "note": "MI355X hot path only (device-resident, no host preparation), against "
                             "the plain FP64 oracle, not a tuned CPU code"}}
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
