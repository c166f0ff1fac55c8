"""Closing step of a coarse-fine pair of levels, for the oracle (test
infrastructure only; nothing on the product path imports it).

Sec. 2.1, step 3 of a level's update: once the finer level has been
advanced, the coarse level is corrected with its results.
  * Restriction: a coarse cell overlaid by fine cells takes the spatial
    average of its eight children.
  * Flux correction: a coarse cell next to a coarse-fine interface gets the
    difference between the coarse flux and the fine flux through that
    interface, so that what leaves the coarse cell is what enters the fine
    cells (conservation).
Sec. 3.1 describes the GPU side of it: the advance outputs the fluxes across
every patch boundary, and the closing step routes them to the coarse patch of
each coarse-fine interface.  Here everything is numpy on whole periodic grids,
with FP64 inputs (or FP32 ones, to mirror a lower-precision run operation by
operation).

Readings (the paper names the operations, not their arithmetic):
  * The fine flux through a coarse face is the mean of the 2 x 2 fine face
    fluxes covering it, summed ((f00 + f01) + f10) + f11 over (a, b) = the
    face's two axes, the higher-numbered first, then times 1/4, of the fine
    records over the coarse step: the fluxes themselves with one dt on both
    levels (the paper's uniform time step), or, with the fine level
    sub-cycled in two steps of dt/2, 1/2 H of the first plus 1/2 H of the
    second (``two_level_step_subcycled``).
  * Sub-cycling: the second fine step takes its ghost zones from the coarse
    level half-way through its step, the mean of its old and advanced states
    (linear interpolation in time), and sweeps in the other order.
  * A coarse cell whose + face along d is a coarse-fine interface gets
    u + lam (H_c - H_f); one whose - face is gets u - lam (H_c - H_f), with
    lam = dt / dh_c: the coarse flux H_c is replaced by H_f in the cell's
    full step (Eq. FullstepValue).
  * A cell on several interfaces takes the corrections in the order
    x-, x+, y-, y+, z-, z+ (of its own faces).
  * Restriction: the children summed in the order (dz, dy, dx) = 000, 001,
    010, 011, 100, 101, 110, 111, then times 1/8.
  * The refined region is a union of whole coarse 8^3 patches (a patch is
    refined into its eight children, Sec. 2.1); proper nesting is assumed.

Grids: a coarse state (5, N, N, N) with patches of 8^3, periodic; the refined
patches as a boolean array (N/8, N/8, N/8) indexed [pz, py, px]; a fine state
(5, 2N, 2N, 2N) whose values matter only inside refined patches.
"""
from __future__ import annotations

import numpy as np

from . import NVAR, GHOST, advance_ragged, periodic_ghosted_blocks
from .ghosts import coarse_to_fine

PATCH = 8


def restrict(fine):
    """Average of the eight children of every coarse cell: fine (5, 2a, 2b, 2c)
    -> coarse (5, a, b, c), in the dtype of ``fine``."""
    f = np.asarray(fine)
    s = f[:, 0::2, 0::2, 0::2]
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                if dz or dy or dx:
                    s = s + f[:, dz::2, dy::2, dx::2]
    return s * f.dtype.type(0.125)


def refined_patches(refined):
    """Coarse patch coordinates (pz, py, px) of the refined patches, z slowest."""
    return [tuple(int(v) for v in p) for p in np.argwhere(np.asarray(refined))]


def fine_block_origins(refined, n_f: int):
    """Fine-cell origins (z, y, x) of the fine blocks of edge n_f (8: patches,
    16: 2^3 patch groups) covering the refined patches: patch by patch in
    (pz, py, px) order, then the blocks of a patch in (z, y, x) order."""
    k = 2 * PATCH // n_f
    out = []
    for pz, py, px in refined_patches(refined):
        for bz in range(k):
            for by in range(k):
                for bx in range(k):
                    out.append((2 * PATCH * pz + n_f * bz, 2 * PATCH * py + n_f * by,
                                2 * PATCH * px + n_f * bx))
    return out


def _in_refined(refined, fz, fy, fx):
    """Whether fine cells (periodic indices) lie in a refined coarse patch."""
    r = np.asarray(refined)
    P = r.shape[0]
    s = 2 * PATCH
    return r[(fz // s) % P, (fy // s) % P, (fx // s) % P]


def ghosted_fine_blocks(coarse, fine, refined, n_f: int):
    """Ghosted fine blocks (B, 5, n_f+6, n_f+6, n_f+6) in ``fine_block_origins``
    order (Sec. 2.2): a ghost cell inside a refined patch is the fine value
    (sibling copy), any other is interpolated from ``coarse``."""
    fine = np.asarray(fine)
    Nf = fine.shape[1]
    m = n_f + 2 * GHOST
    r = np.arange(m) - GHOST
    out = []
    for oz, oy, ox in fine_block_origins(refined, n_f):
        kz, ky, kx = np.meshgrid(oz + r, oy + r, ox + r, indexing="ij")
        inside = _in_refined(refined, kz, ky, kx)
        blk = np.empty((NVAR, m, m, m), dtype=fine.dtype)
        blk[:, inside] = fine[:, kz[inside] % Nf, ky[inside] % Nf, kx[inside] % Nf]
        o = ~inside
        blk[:, o] = coarse_to_fine(coarse, kz[o] % Nf, ky[o] % Nf, kx[o] % Nf)
        out.append(blk)
    return np.stack(out)


def fine_face_fluxes(records, refined, n_f: int, Nf: int):
    """Fine fluxes on the fine grid's faces from the fine blocks' flux records
    (``advance_ragged(..., fluxes=True)`` layout, blocks in
    ``fine_block_origins`` order): for each axis d an array (5, Nf, Nf, Nf)
    indexed [k, f, A, B], the flux through the face between fine cells f-1
    and f along d at transverse fine coordinates (A, B), higher-numbered axis
    first.  Faces no block reports are NaN."""
    dtype = np.asarray(records[0]).dtype if len(records) else np.float64
    out = [np.full((NVAR, Nf, Nf, Nf), np.nan, dtype=dtype) for _ in range(3)]
    for rec, (oz, oy, ox) in zip(records, fine_block_origins(refined, n_f)):
        o = {0: ox, 1: oy, 2: oz}
        for d in range(3):
            hi, lo = (2, 1) if d == 0 else (2, 0) if d == 1 else (1, 0)
            for q in range(n_f // PATCH + 1):
                f = (o[d] + PATCH * q) % Nf
                out[d][:, f, o[hi]:o[hi] + n_f, o[lo]:o[lo] + n_f] = rec[d, q]
    return out


def flux_correct(coarse, refined, coarse_records, fine_faces, lam):
    """Coarse-fine flux correction (Sec. 2.1) of the coarse state, returned as
    a new array.  coarse_records[pz, py, px] is the flux record (3, 2, 5, 8, 8)
    of each coarse patch; fine_faces the per-axis fine face fluxes
    (``fine_face_fluxes``); lam = dt / dh_c as a scalar of the state's dtype.
    Only unrefined patches are corrected, on the faces they share with a
    refined patch."""
    u = np.array(coarse, copy=True)
    ref = np.asarray(refined)
    P = ref.shape[0]
    lam = u.dtype.type(lam)
    q4 = u.dtype.type(0.25)
    for d in range(3):
        hi, lo = (2, 1) if d == 0 else (2, 0) if d == 1 else (1, 0)
        for s in (0, 1):
            for pz, py, px in np.argwhere(~ref):
                p = {0: int(px), 1: int(py), 2: int(pz)}
                nb = dict(p)
                nb[d] = (p[d] + (1 if s else -1)) % P
                if not ref[nb[2], nb[1], nb[0]]:
                    continue
                # the interface: coarse face index along d, fine face twice it
                fc = (PATCH * p[d] + (PATCH if s else 0)) % (P * PATCH)
                A = 2 * (PATCH * p[hi] + np.arange(PATCH))
                B = 2 * (PATCH * p[lo] + np.arange(PATCH))
                F = fine_faces[d][:, 2 * fc]
                f00 = F[:, A[:, None], B[None, :]]
                f01 = F[:, A[:, None], B[None, :] + 1]
                f10 = F[:, A[:, None] + 1, B[None, :]]
                f11 = F[:, A[:, None] + 1, B[None, :] + 1]
                Hf = (((f00 + f01) + f10) + f11) * q4
                Hc = coarse_records[pz, py, px][d, s]
                t = Hc - Hf
                # the corrected cells: index 7 (s = 1) or 0 (s = 0) along d
                c = {a: slice(PATCH * p[a], PATCH * p[a] + PATCH) for a in range(3)}
                c[d] = PATCH * p[d] + (PATCH - 1 if s else 0)
                # cells [k, z, y, x] of that face, viewed as [k, a, b]
                view = u[:, c[2], c[1], c[0]]
                new = view + lam * t if s else view - lam * t
                u[:, c[2], c[1], c[0]] = new
    return u


def two_level_step(coarse, fine, refined, n_f: int, dt: float, order: int, gamma: float,
                   p_floor: float = 0.0, correct: bool = True, restrict_fine: bool = True):
    """One step of a two-level periodic hierarchy with one dt on both levels
    (FP64): the coarse patches (8^3, ghost zones by periodic copy) and the
    fine blocks (edge n_f, ghost zones by sibling copy or coarse-fine
    interpolation from the coarse level at the old time) are advanced with
    the oracle's step, then the coarse level is restricted from the fine one
    and flux-corrected.  Returns (coarse, fine) after the step; fine is
    unchanged outside the refined patches."""
    coarse = np.asarray(coarse, dtype=np.float64)
    fine = np.asarray(fine, dtype=np.float64)
    N = coarse.shape[1]
    Nf = 2 * N
    P = N // PATCH
    dh_c = 1.0 / N
    dh_f = 0.5 / N
    # coarse level
    cb = periodic_ghosted_blocks(coarse, PATCH)
    c_out, c_rec = advance_ragged(list(cb), order, dt, dh_c, gamma, p_floor, fluxes=True)
    new_c = np.empty_like(coarse)
    recs = np.empty((P, P, P) + c_rec[0].shape)
    i = 0
    for pz in range(P):
        for py in range(P):
            for px in range(P):
                new_c[:, PATCH * pz:PATCH * pz + PATCH, PATCH * py:PATCH * py + PATCH,
                      PATCH * px:PATCH * px + PATCH] = c_out[i]
                recs[pz, py, px] = c_rec[i]
                i += 1
    # fine level, ghost zones from the coarse level at the old time
    fb = ghosted_fine_blocks(coarse, fine, refined, n_f)
    f_out, f_rec = advance_ragged(list(fb), order, dt, dh_f, gamma, p_floor, fluxes=True)
    new_f = fine.copy()
    for blk, (oz, oy, ox) in zip(f_out, fine_block_origins(refined, n_f)):
        new_f[:, oz:oz + n_f, oy:oy + n_f, ox:ox + n_f] = blk
    # closing: restriction of refined patches, then the flux correction
    if restrict_fine:
        for pz, py, px in refined_patches(refined):
            s = 2 * PATCH
            new_c[:, PATCH * pz:PATCH * pz + PATCH, PATCH * py:PATCH * py + PATCH,
                  PATCH * px:PATCH * px + PATCH] = restrict(
                new_f[:, s * pz:s * pz + s, s * py:s * py + s, s * px:s * px + s])
    if correct:
        faces = fine_face_fluxes(f_rec, refined, n_f, Nf)
        new_c = flux_correct(new_c, refined, recs, faces, dt / dh_c)
    return new_c, new_f


def lerp(a, b, w: float):
    """a + w (b - a) in the dtype of a, w rounded to it: linear interpolation
    in time between two states of a level."""
    a = np.asarray(a)
    return a + a.dtype.type(w) * (np.asarray(b) - a)


def _advance_grid_fine(coarse, fine, refined, n_f, dt, order, gamma, p_floor):
    fb = ghosted_fine_blocks(coarse, fine, refined, n_f)
    f_out, f_rec = advance_ragged(list(fb), order, dt, 0.5 / coarse.shape[1], gamma, p_floor,
                                  fluxes=True)
    new_f = fine.copy()
    for blk, (oz, oy, ox) in zip(f_out, fine_block_origins(refined, n_f)):
        new_f[:, oz:oz + n_f, oy:oy + n_f, ox:ox + n_f] = blk
    return new_f, f_rec


def two_level_step_subcycled(coarse, fine, refined, n_f: int, dt: float, order: int,
                             gamma: float, p_floor: float = 0.0, correct: bool = True):
    """One coarse step of dt with the fine level sub-cycled (Sec. 2.1: the
    step of level l may be half that of level l-1), FP64.  The coarse level
    advances by dt (sweep order `order`); the fine level advances twice by
    dt/2 (orders `order`, then the other), the first time with ghost zones
    from the coarse level at the old time, the second from the coarse level
    half-way through its step (the mean of the old and the advanced coarse
    states, linear in time) and its own siblings after the first sub-step.
    The fine flux records of the two sub-steps are summed with weight 1/2
    each (the first written as 1/2 H, the second added as 1/2 H), which makes
    them the fine fluxes over the coarse step; then restriction and the flux
    correction as in ``two_level_step``.  Returns (coarse, fine)."""
    coarse = np.asarray(coarse, dtype=np.float64)
    fine = np.asarray(fine, dtype=np.float64)
    N = coarse.shape[1]
    P = N // PATCH
    dh_c = 1.0 / N
    cb = periodic_ghosted_blocks(coarse, PATCH)
    c_out, c_rec = advance_ragged(list(cb), order, dt, dh_c, gamma, p_floor, fluxes=True)
    new_c = np.empty_like(coarse)
    recs = np.empty((P, P, P) + c_rec[0].shape)
    i = 0
    for pz in range(P):
        for py in range(P):
            for px in range(P):
                new_c[:, PATCH * pz:PATCH * pz + PATCH, PATCH * py:PATCH * py + PATCH,
                      PATCH * px:PATCH * px + PATCH] = c_out[i]
                recs[pz, py, px] = c_rec[i]
                i += 1
    half = 0.5
    f1, r1 = _advance_grid_fine(coarse, fine, refined, n_f, dt * half, order, gamma, p_floor)
    c_half = lerp(coarse, new_c, half)
    f2, r2 = _advance_grid_fine(c_half, f1, refined, n_f, dt * half, 1 - order, gamma, p_floor)
    f_rec = [half * a + half * b for a, b in zip(r1, r2)]
    for pz, py, px in refined_patches(refined):
        s = 2 * PATCH
        new_c[:, PATCH * pz:PATCH * pz + PATCH, PATCH * py:PATCH * py + PATCH,
              PATCH * px:PATCH * px + PATCH] = restrict(
            f2[:, s * pz:s * pz + s, s * py:s * py + s, s * px:s * px + s])
    if correct:
        faces = fine_face_fluxes(f_rec, refined, n_f, 2 * N)
        new_c = flux_correct(new_c, refined, recs, faces, dt / dh_c)
    return new_c, f2


def leaf_sums(coarse, fine, refined):
    """Totals of the five conserved variables over the leaf cells (coarse cells
    of unrefined patches, fine cells of refined ones), in units of the coarse
    cell volume, summed exactly (math.fsum)."""
    import math
    ref = np.asarray(refined)
    cm = np.repeat(np.repeat(np.repeat(~ref, PATCH, 0), PATCH, 1), PATCH, 2)
    fm = np.repeat(np.repeat(np.repeat(ref, 2 * PATCH, 0), 2 * PATCH, 1), 2 * PATCH, 2)
    return np.array([math.fsum(np.asarray(coarse[k], dtype=np.float64)[cm].tolist()) +
                     math.fsum((np.asarray(fine[k], dtype=np.float64)[fm] / 8.0).tolist())
                     for k in range(NVAR)])


def _dense_records(recs, refined, n_f: int = PATCH):
    """Flux records of the blocks over ``refined`` (``fine_block_origins``
    order, 8^3 patches) scattered to a [pz, py, px] array over the fine
    level's patch grid; patches that do not exist hold NaN."""
    P = 2 * np.asarray(refined).shape[0]
    out = np.full((P, P, P) + np.asarray(recs[0]).shape, np.nan)
    for rec, (oz, oy, ox) in zip(recs, fine_block_origins(refined, n_f)):
        out[oz // PATCH, oy // PATCH, ox // PATCH] = rec
    return out


def _close(coarse, fine, refined, coarse_recs, fine_recs, lam, correct):
    """Restriction of the refined patches from ``fine``, then the flux
    correction of the coarse level with the fine records (Sec. 2.1, step 3)."""
    new_c = np.array(coarse, copy=True)
    s = 2 * PATCH
    for pz, py, px in refined_patches(refined):
        new_c[:, PATCH * pz:PATCH * pz + PATCH, PATCH * py:PATCH * py + PATCH,
              PATCH * px:PATCH * px + PATCH] = restrict(
            fine[:, s * pz:s * pz + s, s * py:s * py + s, s * px:s * px + s])
    if correct:
        faces = fine_face_fluxes(fine_recs, refined, PATCH, fine.shape[1])
        new_c = flux_correct(new_c, refined, coarse_recs, faces, lam)
    return new_c


def _subcycle(states, refined, lev, c_old, c_new, dt, order, gamma, p_floor, correct):
    """Level ``lev`` (>= 1) takes two steps of dt/2 inside its parent's step
    of dt, whose level went from c_old to c_new (before its closing step):
    the first with ghost zones from c_old, the second from lerp(c_old, c_new,
    1/2), in sweep orders ``order`` and 1 - order.  After each sub-step the
    next finer level, if any, does the same inside it and then closes into
    this one.  Returns this level's records over dt: lerp of the two
    sub-steps' records at 1/2 (their mean)."""
    half = 0.5
    c_half = lerp(c_old, c_new, half)
    recs = []
    for k in (0, 1):
        o = order if k == 0 else 1 - order
        old = states[lev]
        new, rec = _advance_grid_fine(c_old if k == 0 else c_half, old, refined[lev - 1], PATCH,
                                      dt * half, o, gamma, p_floor)
        if lev + 1 < len(states):
            fine_recs = _subcycle(states, refined, lev + 1, old, new, dt * half, o, gamma,
                                  p_floor, correct)
            new = _close(new, states[lev + 1], refined[lev],
                         _dense_records(rec, refined[lev - 1]), fine_recs,
                         dt * half * new.shape[1], correct)
        states[lev] = new
        recs.append(rec)
    return [lerp(a, b, half) for a, b in zip(*recs)]


def nested_step_subcycled(states, refined, dt: float, order: int, gamma: float,
                          p_floor: float = 0.0, correct: bool = True):
    """One root step of dt on a periodic hierarchy of any depth, every level
    sub-cycled (Sec. 2.1: the step of level l is half that of level l-1, and
    a level's update is: advance, let the finer level catch up, correct with
    it), FP64, 8^3 patches on every level.

    states[l] is level l's state on its whole periodic grid (5, N 2^l, ...),
    meaningful inside its patches; refined[l] (over level l's patch grid)
    marks the patches refined into level l+1 (proper nesting assumed).  The
    root level advances by dt with periodic ghost zones; each finer level as
    in ``_subcycle`` (recursively); each level is then closed with the next
    finer one (restriction, then the flux correction with the finer level's
    records averaged over the step), finest pair first.  Returns the new
    states."""
    states = [np.array(s, dtype=np.float64) for s in states]
    c0 = states[0]
    N = c0.shape[1]
    P = N // PATCH
    cb = periodic_ghosted_blocks(c0, PATCH)
    c_out, c_rec = advance_ragged(list(cb), order, dt, 1.0 / N, gamma, p_floor, fluxes=True)
    new0 = np.empty_like(c0)
    recs0 = np.empty((P, P, P) + c_rec[0].shape)
    i = 0
    for pz in range(P):
        for py in range(P):
            for px in range(P):
                new0[:, PATCH * pz:PATCH * pz + PATCH, PATCH * py:PATCH * py + PATCH,
                     PATCH * px:PATCH * px + PATCH] = c_out[i]
                recs0[pz, py, px] = c_rec[i]
                i += 1
    if len(states) > 1:
        fine_recs = _subcycle(states, refined, 1, c0, new0, dt, order, gamma, p_floor, correct)
        new0 = _close(new0, states[1], refined[0], recs0, fine_recs, dt * N, correct)
    states[0] = new0
    return states


def nested_leaf_sums(states, refined):
    """Totals of the conserved variables over the leaf cells of a nested
    hierarchy (cells of existing patches that are not refined; level l's
    cells weigh 8^-l), summed exactly."""
    import math
    L = len(states)
    exist = np.ones((states[0].shape[1] // PATCH,) * 3, dtype=bool)
    tot = np.zeros(NVAR)
    for lev in range(L):
        leaf = exist & ~refined[lev] if lev + 1 < L else exist
        m = np.repeat(np.repeat(np.repeat(leaf, PATCH, 0), PATCH, 1), PATCH, 2)
        w = 8.0 ** -lev
        for k in range(NVAR):
            tot[k] += math.fsum((np.asarray(states[lev][k], dtype=np.float64)[m] * w).tolist())
        if lev + 1 < L:
            exist = np.repeat(np.repeat(np.repeat(refined[lev], 2, 0), 2, 1), 2, 2)
    return tot
