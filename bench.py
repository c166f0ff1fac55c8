#!/usr/bin/env python3
"""Throughput of the relaxing-TVD patch advance on one MI355X.

Workload: a periodic 256^3 grid, i.e. 32768 octree patches of 8^3 cells,
lognormal density (sigma_ln = 1), Gaussian velocities (sigma = 0.3 c_s),
uniform pressure P = 1, gamma = 5/3, CFL 0.5, seeded.  A step is one pass of
the whole hot path on the device: the Eq. (CFL) signal speed and the time
step on even steps (fused into the previous odd step's advance), the
sibling ghost-zone fill, and one triple of 1-D sweeps (xyz on even steps,
zyx on odd steps).

Reported (one JSON line on stdout):
* value: cell-updates/s of the FP32 batched kernel on 2^3 patch groups
  (4096 blocks of 16^3 interior cells), inputs resident in HBM;
* fp64_plain: the same steps with the plain FP64 per-patch kernel
  (32768 blocks of 8^3) on the same FP32-rounded initial state;
* fp64_batched, fp32_batched_edge8: the batched kernel in FP64 on 8^3
  patches (with its largest difference from fp64_plain) and in FP32 on
  single 8^3 patches instead of 2^3 patch groups;
* l1_vs_fp64: relative L1 error per variable of the FP32 result against
  the FP64 result after the same steps;
* roofline: the advance kernel's algorithmic HBM bytes per launch over its
  average duration (HIP events on the launch stream) against 8 TB/s;
* cpu_baseline: the FP64 oracle on the host cores over a bounded sample;
* uneven_batch: cell-updates/s of 4000 periodic boxes of mixed sizes in one
  persistent launch per step, 50-step HIP graphs, block edge tuned;
* amr_ghost_fill: the coarse-fine ghost fill (sibling copy, else Min-Mod
  limited interpolation from the coarser level) of 8^3 patches and 16^3
  groups covering a refined 256^3-cell box;
* multilevel_batch: one step of a 4-level patch hierarchy (18 152 patches,
  per-block dt and dh) as one persistent FP32 launch on patches and on 2^3
  patch groups, and as plain FP64 launches level by level;
* closing_step: on the same hierarchy with one dt, the advance writing
  patch-boundary flux records, and the restriction and coarse-fine flux
  correction of every level pair;
* poisson_sor: red-black SOR for the Poisson equation on 4096 patch groups,
  50 fixed iterations and solves to the stopping rule, FP32 and FP64;
* gravity_operator: the self-gravity source operator on the 256^3 state.
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
GAMMA = 5.0 / 3.0
CFL = 0.5
HBM_PEAK_GBS = 8000.0
# FP32 vector peak without packed FP32 (turned off in this build):
# 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
FP32_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_batched_fp32_edge16_gather_256cube_traffic.txt")
KERNEL_SOURCES = ["paper_0907_3390_amd/csrc/tvd_kernels.hip", "paper_0907_3390_amd/csrc/tvd_device.hpp"]
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


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(variant):
    """HBM bytes per launch of the advance from the committed rocprofv3 counter
    summary, only if it was taken on the current kernel sources and on a
    launch variant with the same HBM access pattern: the block edge, the
    workgroup size and whether the third sweep runs in half pencils (split
    bit 1) fix which addresses are read and written; the LDS padding and the
    second sweep's split only move work inside the workgroup."""
    if not os.path.exists(TRAFFIC_FILE):
        return None, "no counter summary"
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_source_hash():
        return None, "kernel changed since the counters were taken"
    if variant is not None:
        got = [int(x) for x in kv.get("variant", "0,0,0,0").split(",")]
        want = [variant[k] for k in ("edge", "threads", "lds_pad", "split")]
        if got[:2] != want[:2] or (got[3] & 2) != (want[3] & 2):
            return None, f"counters were taken on variant {got}, not {want}"
    return float(kv["hbm_bytes_per_launch_mean"]), ("rocprofv3 FETCH_SIZE x2 + WRITE_SIZE, "
                                                    + os.path.relpath(TRAFFIC_FILE, ROOT))


def make_ic():
    from paper_0907_3390_amd import workloads as wl
    g = wl.lognormal(N_GRID, seed=SEED, sigma_ln=1.0, vel_sigma_rel=0.3, P0=1.0, gamma=GAMMA)
    return g.astype(np.float32)  # FP32-rounded; the FP64 runs start from the same values


def run_gpu(ctx, grid32, n, dtype, kernel, steps, warmup, gather=False, tune=False):
    """Warm up, then time `steps` steps twice: eagerly with HIP events around
    every advance launch (for the kernel's average duration), and as replays
    of a HIP graph holding one xyz/zyx pair (for the step rate)."""
    import torch
    from paper_0907_3390_amd import layout, tvd
    from paper_0907_3390_amd.driver import DeviceBlocks
    # blocks numbered along a Morton curve: each XCD's contiguous share of the
    # blocks is a compact brick, so neighbours' ghost data meet in its L2
    bs = layout.periodic_grid_blockset(N_GRID, n, curve="morton")
    dev = DeviceBlocks(ctx, bs, dtype=dtype, gamma=GAMMA, cfl=CFL, kernel=kernel, gather=gather)
    dev.upload(layout.grid_to_blocks(grid32.astype(np.float64), n, bs.perm))
    info = {"blocks": bs.n_blocks, "edge": n}
    if tune:
        # pick the launch variant on the real data (scratch output), untimed
        dev.dt.fill_(CFL / N_GRID / 4.0)
        scratch = dev.spare if gather else dev.interior.clone()
        src = dev.interior if gather else dev.ghosted
        if not gather:
            dev.fill_ghosts()
        idx, ms = ctx.tvd_autotune(dev.batch, dev.nbr if gather else None, src, scratch, GAMMA,
                                   reps=3)
        info["variant"] = dict(zip(("index", "edge", "threads", "lds_pad", "split"),
                                   tvd.variants()[idx]))
        info["variant"]["tuned_ms_per_pair"] = ms
        log(f"bench: tuned variant {info['variant']}")
    for _ in range(max(warmup, 2)):
        dev.step()
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
        dev.advance(s % 2, fuse_speed=(s % 2 == 1))
        adv_ev[k][1].record(stream)
        dev.step_index += 1
    torch.cuda.synchronize()
    info["adv_ms"] = [a.elapsed_time(b) for a, b in adv_ev]
    # graph-captured pair, replayed steps/2 times
    side = torch.cuda.Stream()
    graph = dev.capture(2, stream=side)
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
    from paper_0907_3390_amd import tvd, tuning, workloads as wl
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


def run_nested(ctx, ml, reps=4):
    """The multi-level hierarchy advanced with every level sub-cycled (FP32,
    8^3 patches): one root step is one step of level 0, two of level 1, four
    of level 2 and eight of level 3, each level closed with the next finer
    one after each of its steps (amr.NestedDevice).  Timed with HIP events
    over `reps` root steps run eagerly, and as replays of a HIP graph of two
    root steps (xyz, zyx).  Also reports the drift of the leaf totals over
    the timed steps (host sums of the downloaded state)."""
    import torch
    from paper_0907_3390_amd import amr, layout, tvd
    refined = layout.NestedLevels.refined_from_patches(ml.base, ml.patches)
    top = len(refined)
    dev = amr.NestedDevice(ctx, ml.base, refined, dtype=torch.float32)
    L = dev.L
    interior = ml.ghosted[:, :, 3:11, 3:11, 3:11]
    per = [np.zeros((n, 5, 8, 8, 8), dtype=np.float32) for n in dev.nb]
    for i, (l, px, py, pz) in enumerate(ml.patches):
        per[l][L.locate(l, px, py, pz)[0]] = interior[i]
    dev.upload(per)
    leaf = [np.ones(n, dtype=bool) for n in dev.nb]
    for l in range(top):
        for (lev, px, py, pz) in L.patches:
            if lev == l and refined[l][pz, py, px]:
                leaf[l][L.locate(l, px, py, pz)[0]] = False

    def leaf_sums(blocks):
        return sum(blocks[l][leaf[l]].astype(np.float64).sum(axis=(0, 2, 3, 4)) * 8.0 ** -l
                   for l in range(len(blocks)))
    before = leaf_sums(per)
    scale = sum(np.abs(per[l][leaf[l]]).astype(np.float64).sum(axis=(0, 2, 3, 4)) * 8.0 ** -l
                for l in range(len(per)))
    sm = torch.zeros(1, dtype=torch.float64, device="cuda")
    u_in = torch.from_numpy(np.ascontiguousarray(ml.ghosted)).float().cuda().reshape(-1)
    d_dh = torch.from_numpy(np.ascontiguousarray(ml.dh)).cuda()
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
    after = leaf_sums(dev.download())
    steps = 2 + reps + 2 + 2 * (reps // 2)
    updates = sum((1 << l) * n * 512 for l, n in enumerate(dev.nb))
    # the gas starts at rest: momentum is measured against mass times the
    # largest signal speed
    scale[1:4] = scale[0] * float(sm.item())
    drift = float(np.max(np.abs(after - before) / scale))
    res = {"workload": "multi-level hierarchy (128^3 base, levels 1-3, 18 152 patches of 8^3), "
                       "FP32, every level sub-cycled, every pair closed",
           "patches_per_level": dev.nb, "cell_updates_per_root_step": updates,
           "root_step_ms_eager": ms_eager, "root_step_ms_graph": ms_graph,
           "value": updates / (ms_graph * 1e-3), "unit": "cell-updates/s",
           "root_steps_run": steps, "leaf_total_drift": drift}
    log(f"bench: nested sub-cycled step: {ms_eager:.3f} ms eager, {ms_graph:.3f} ms as graph replay "
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
        coarse_bs, fine_bs, cnbr, corigin = layout.two_level(Nc, origin, shape, n)
        m = n + 6
        nb = fine_bs.n_blocks
        f_in = torch.from_numpy(layout.grid_to_blocks(fine, n)).cuda().reshape(-1)
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
        res[f"edge{n}"] = {"blocks": nb, "ms": ms, "ghosted_cells_per_s": nb * m ** 3 / (ms * 1e-3),
                           "ghost_cells": ghost_cells,
                           "algorithmic_GBs": bytes_alg / (ms * 1e-3) / 1e9,
                           "hbm_frac": bytes_alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        log(f"bench: coarse-fine ghost fill, edge {n}: {ms:.3f} ms, "
            f"{res[f'edge{n}']['algorithmic_GBs']:.0f} GB/s algorithmic")
        del f_in, f_gh
        torch.cuda.empty_cache()
    st, fl, bad = ctx.tvd_read_flags()
    res["health"] = {"nonphysical": bad}
    return res


def cpu_baseline(grid32, budget_s=15.0):
    """The FP64 oracle (as it stands) on the host cores over a bounded sample
    of the same workload: whole steps of the 256^3 grid as 32768 patches of
    8^3 (periodic ghost fill in numpy, then the C advance), repeated until the
    time budget is used; only the advance is timed, like the GPU's kernel."""
    import oracle
    g = grid32.astype(np.float64)
    dh = 1.0 / N_GRID
    steps, adv, threads, t_all = 0, 0.0, 1, time.perf_counter()
    dt = None
    while adv < budget_s and steps < 20:
        if steps % 2 == 0:
            dt = CFL * dh / oracle.max_signal_speed(g, GAMMA)
        blocks = oracle.periodic_ghosted_blocks(g, 8)
        c = oracle.Counts()
        t = time.perf_counter()
        out = oracle.advance_blocks(blocks, steps % 2, dt, dh, GAMMA, counts=c)
        adv += time.perf_counter() - t
        threads = c.threads
        g = oracle.assemble_blocks(out, g.shape)
        steps += 1
    # one host thread (the paper compares one GPU with one CPU core): one step
    # of a 4096-patch slice of the same state
    blocks = oracle.periodic_ghosted_blocks(g, 8)[:4096]
    oracle.set_threads(1)
    c = oracle.Counts()
    t = time.perf_counter()
    oracle.advance_blocks(blocks, 0, dt, dh, GAMMA, counts=c)
    t1 = time.perf_counter() - t
    oracle.set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    return {"value": steps * N_GRID ** 3 / adv, "unit": "cell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{steps} steps of the full 256^3 workload (32768 8^3 patches), FP64, "
                      f"advance {adv:.1f} s timed of {time.perf_counter() - t_all:.1f} s "
                      f"(ghost fill and CFL speed in numpy not timed)",
            "single_thread": {"value": 4096 * 512 / t1, "unit": "cell-updates/s", "cores": c.threads,
                              "sample": "one step of 4096 of the 32768 patches, FP64"}}


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 plain comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-variant tuner")
    ap.add_argument("--no-amr-fill", action="store_true",
                    help="skip the coarse-fine ghost-fill throughput")
    ap.add_argument("--no-multilevel", action="store_true",
                    help="skip the multi-level (18 152 patches) throughput")
    ap.add_argument("--no-closing", action="store_true",
                    help="skip the closing step (flux records, restriction, flux correction)")
    ap.add_argument("--no-poisson", action="store_true",
                    help="skip the red-black SOR Poisson solver on patch groups")
    ap.add_argument("--no-uneven", action="store_true",
                    help="skip the uneven-batch (4000 mixed boxes) throughput")
    ap.add_argument("--edge", type=int, default=16, help="block edge of the FP32 batched run")
    ap.add_argument("--no-gather", action="store_true",
                    help="headline run with a separate ghost fill instead of the gathering advance")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.steps % 2 or args.warmup % 2:
        sys.exit("--steps and --warmup must be even (steps come in xyz/zyx pairs)")

    import torch
    from paper_0907_3390_amd import tvd
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    log(f"bench: building the 256^3 initial state (seed {SEED})")
    grid32 = make_ic()
    ctx = tvd.Context(0)
    cells = N_GRID ** 3

    gather = not args.no_gather
    log(f"bench: FP32 batched, edge {args.edge}, gather={gather}, {args.warmup}+{args.steps} steps")
    dev32, r32 = run_gpu(ctx, grid32, args.edge, torch.float32, tvd.TVD_KERNEL_AUTO,
                         args.steps, args.warmup, gather=gather, tune=not args.no_tune)
    ms_step = r32["total_ms"] / args.steps
    value = cells * args.steps / (r32["total_ms"] * 1e-3)
    n = args.edge
    nb = r32["blocks"]
    # algorithmic bytes of one launch: the ghosted block in (gathered from the
    # neighbours' interiors, or read from a ghosted copy) and the interior out
    bytes_launch = nb * ((n + 6) ** 3 + n ** 3) * 5 * 4
    adv_avg_ms = float(np.mean(r32["adv_ms"]))
    achieved = bytes_launch / (adv_avg_ms * 1e-3) / 1e9
    flops_launch = nb * flops_per_block(n)
    tflops = flops_launch / (adv_avg_ms * 1e-3) / 1e12
    traffic, traffic_note = (measured_traffic(r32.get("variant")) if (n == 16 and gather)
                             else (None, "not profiled"))
    out = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "256^3 periodic grid = 32768 patches of 8^3 (run as 4096 "
                               "2^3 patch groups of 16^3), lognormal rho sigma_ln=1, Gaussian "
                               "v sigma=0.3 c_s, P=1, gamma=5/3, CFL 0.5, seed 2024"
                               if n == 16 else
                               "256^3 periodic grid = 32768 patches of 8^3, lognormal rho "
                               "sigma_ln=1, Gaussian v sigma=0.3 c_s, P=1, gamma=5/3, CFL 0.5, "
                               "seed 2024",
                   "cells": cells, "blocks": nb, "block_edge": n, "precision": "fp32",
                   "ghost_zones": "gathered inside the advance" if gather else "separate fill",
                   "block_order": "Morton curve"},
        "roofline": {"bound": "alu", "achieved": tflops, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": tflops / FP32_PEAK_TFLOPS, "traffic": traffic,
                     "traffic_source": traffic_note,
                     "kernel": f"k_batched<float,{n}>" + (" gather" if gather else ""),
                     "avg_launch_ms": adv_avg_ms,
                     "algorithmic_flops_per_launch": flops_launch,
                     "hbm": {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": achieved / HBM_PEAK_GBS,
                             "algorithmic_bytes_per_launch": bytes_launch}},
        "advance_cell_updates_per_s": cells / (adv_avg_ms * 1e-3),
        "timing": "steps replayed as a HIP graph of one xyz/zyx pair; advance duration from "
                  "HIP events around eager launches of the same steps",
        "variant": r32.get("variant"),
        "health": {"floored": r32["floored"], "nonphysical": r32["nonphysical"]},
    }
    log(f"bench: FP32 {value / 1e9:.2f} G cell-updates/s, advance {adv_avg_ms:.3f} ms "
        f"({achieved:.0f} GB/s, {tflops:.1f} TFLOP/s)")
    out["hbm_copy_measured"] = copy_bandwidth()
    out["roofline"]["hbm"]["frac_of_measured_copy"] = (
        achieved / out["hbm_copy_measured"]["read_plus_write_GBs"])
    log(f"bench: plain 1 GiB copy {out['hbm_copy_measured']['read_plus_write_GBs']:.0f} GB/s")

    if not args.no_fp64:
        log(f"bench: FP64 plain, edge 8, {args.warmup}+{args.steps} steps")
        s32 = np.stack(dev32.download()).astype(np.float64)
        dev32_perm = dev32.bs.perm
        del dev32
        torch.cuda.empty_cache()
        dev64, r64 = run_gpu(ctx, grid32, 8, torch.float64, tvd.TVD_KERNEL_PLAIN, args.steps,
                             args.warmup)
        v64 = cells * args.steps / (r64["total_ms"] * 1e-3)
        a64 = float(np.mean(r64["adv_ms"]))
        from paper_0907_3390_amd import layout
        s64 = np.stack(dev64.download())
        g32 = layout.blocks_to_grid(s32, (5, N_GRID, N_GRID, N_GRID), dev32_perm)
        g64 = layout.blocks_to_grid(s64, (5, N_GRID, N_GRID, N_GRID), dev64.bs.perm)
        del dev64, s64
        nrm = {}
        for k, nm in enumerate(["rho", "m_x", "m_y", "m_z", "e"]):
            d = np.abs(g32[k] - g64[k]).sum()
            nrm[nm] = d / np.abs(g64[k]).sum()
        rho = g64[0]
        kin = 0.5 * (g64[1] ** 2 + g64[2] ** 2 + g64[3] ** 2) / rho
        cs = np.sqrt(GAMMA * np.maximum((GAMMA - 1) * (g64[4] - kin), 0) / rho)
        scale = (rho * cs).sum()
        for k, nm in enumerate(["m_x", "m_y", "m_z"]):
            nrm[nm + "_scale"] = np.abs(g32[k + 1] - g64[k + 1]).sum() / scale
        out["fp64_plain"] = {"value": v64, "unit": "cell-updates/s", "ms_per_step": r64["total_ms"] / args.steps,
                             "avg_launch_ms": a64, "blocks": r64["blocks"], "block_edge": 8}
        out["speedup_fp32_batched_vs_fp64_plain"] = value / v64
        out["l1_vs_fp64"] = {k: float(v) for k, v in nrm.items()}
        out["l1_vs_fp64"]["after_steps"] = max(args.warmup, 2) + 2 * args.steps
        log(f"bench: FP64 plain {v64 / 1e9:.3f} G cell-updates/s; relL1 {nrm}")
        # the other two points of the comparison: the batched kernel in FP64
        # (8^3 patches, gathering) and in FP32 on single 8^3 patches
        torch.cuda.empty_cache()
        others = {}
        for name, dtype, n in (("fp64_batched", torch.float64, 8), ("fp32_batched_edge8", torch.float32, 8)):
            log(f"bench: {name}, edge {n}, {args.warmup}+{args.steps} steps")
            dv, rr = run_gpu(ctx, grid32, n, dtype, tvd.TVD_KERNEL_AUTO, args.steps, args.warmup,
                             gather=True, tune=not args.no_tune)
            vv = cells * args.steps / (rr["total_ms"] * 1e-3)
            others[name] = {"value": vv, "unit": "cell-updates/s",
                            "ms_per_step": rr["total_ms"] / args.steps,
                            "avg_launch_ms": float(np.mean(rr["adv_ms"])), "blocks": rr["blocks"],
                            "block_edge": n, "variant": rr.get("variant")}
            if dtype == torch.float64:
                gb = layout.blocks_to_grid(np.stack(dv.download()), (5, N_GRID, N_GRID, N_GRID),
                                           dv.bs.perm)
                others[name]["max_rel_diff_vs_fp64_plain"] = float(
                    max(np.abs(gb[k] - g64[k]).max() / np.abs(g64[k]).max() for k in range(5)))
            del dv
            torch.cuda.empty_cache()
            log(f"bench: {name} {vv / 1e9:.3f} G cell-updates/s")
        out.update(others)
    if not args.no_amr_fill:
        log("bench: coarse-fine ghost fill")
        torch.cuda.empty_cache()
        out["amr_ghost_fill"] = run_amr_fill(ctx)
    if not args.no_multilevel or not args.no_closing:
        from paper_0907_3390_amd import workloads as wl
        log("bench: building the multi-level hierarchy")
        ml = wl.multilevel()
    if not args.no_multilevel:
        log("bench: multi-level batch")
        torch.cuda.empty_cache()
        out["multilevel_batch"] = run_multilevel(ctx, ml)
    if not args.no_closing:
        log("bench: closing step on the multi-level hierarchy")
        torch.cuda.empty_cache()
        out["closing_step"] = run_closing(ctx, ml)
        log("bench: nested sub-cycled step on the multi-level hierarchy")
        torch.cuda.empty_cache()
        out["nested_subcycled_step"] = run_nested(ctx, ml)
    if not args.no_poisson:
        log("bench: Poisson SOR on patch groups")
        torch.cuda.empty_cache()
        out["poisson_sor"] = run_poisson(ctx)
        out["gravity_operator"] = run_gravity(ctx, grid32)
    if not args.no_uneven:
        log("bench: uneven batch of 4000 boxes")
        torch.cuda.empty_cache()
        out["uneven_batch"] = run_uneven(ctx)
    if not args.no_cpu_baseline:
        log("bench: FP64 oracle on the host cores (bounded sample)")
        out["cpu_baseline"] = cpu_baseline(grid32)
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
