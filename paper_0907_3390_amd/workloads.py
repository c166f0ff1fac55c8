"""Seeded synthetic inputs for the relaxing-TVD patch advance.

This module only builds initial states: it holds none of the scheme's
arithmetic, so that the oracle and the HIP path can both be fed from it
without sharing solver code.  Every generator returns conserved variables
(rho, m_x, m_y, m_z, e) in FP64 as an array of shape (5, Nz, Ny, Nx), x
fastest, built from primitive variables with the ideal-gas relations of
Eqs. (ThermalEnergy) and (EOS) of Schive, Tsai & Chiueh (GAMER, 2010).

The shapes and value distributions stand in for the paper's workloads: its
test problems (Sec. 4: sound wave, Sod shock tube, Sedov-Taylor blast) and,
for throughput, its cosmological runs (Sec. 5), whose initial conditions are
not available; those are replaced by lognormal densities with Gaussian
velocities on the paper's patch geometry (8^3 patches, 2^3 patch families).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GAMMA = 5.0 / 3.0


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def conserved(rho, vx, vy, vz, P, gamma: float = GAMMA):
    """Stack primitive fields into conserved variables (5, ...) in FP64."""
    rho = np.asarray(rho, dtype=np.float64)
    shape = rho.shape
    vx = np.broadcast_to(np.asarray(vx, dtype=np.float64), shape)
    vy = np.broadcast_to(np.asarray(vy, dtype=np.float64), shape)
    vz = np.broadcast_to(np.asarray(vz, dtype=np.float64), shape)
    P = np.broadcast_to(np.asarray(P, dtype=np.float64), shape)
    if gamma == 1.0:
        if np.any(P != 0.0):
            raise ValueError("gamma = 1 describes pressureless gas only")
        eint = np.zeros(shape)
    else:
        eint = P / (gamma - 1.0)
    e = eint + 0.5 * rho * (vx * vx + vy * vy + vz * vz)
    return np.stack([rho, rho * vx, rho * vy, rho * vz, e]).astype(np.float64)


def uniform(N, rho=1.0, v=(0.0, 0.0, 0.0), P=1.0, gamma: float = GAMMA):
    Nz, Ny, Nx = (N, N, N) if np.isscalar(N) else N
    ones = np.ones((Nz, Ny, Nx))
    return conserved(rho * ones, v[0], v[1], v[2], P * ones, gamma)


def sod_x(N: int = 32, gamma: float = GAMMA, split: int | None = None,
          left=(1.0, 1.0), right=(0.125, 0.1), ny: int | None = None, nz: int | None = None):
    """Sod shock tube along x (Sec. 4.2 states): cells with x index < split take
    the left state (rho, P), the others the right state; gas at rest."""
    ny = N if ny is None else ny
    nz = N if nz is None else nz
    split = N // 2 if split is None else split
    x = np.arange(N)
    rho1 = np.where(x < split, left[0], right[0])
    P1 = np.where(x < split, left[1], right[1])
    rho = np.broadcast_to(rho1, (nz, ny, N)).copy()
    P = np.broadcast_to(P1, (nz, ny, N)).copy()
    return conserved(rho, 0.0, 0.0, 0.0, P, gamma)


def acoustic(N: int, amplitude: float = 1e-6, k=(1, 0, 0), rho0: float = 1.0,
             P0: float = 0.6, gamma: float = GAMMA, shape=None):
    """Standing sound wave at rest (Sec. 4.1 background: rho0 = 1, P0 = 3/5, so
    c_s = 1): rho = rho0 (1 + A sin(2 pi k.x / L)), adiabatic pressure
    perturbation dP = c_s^2 drho, zero velocity; cell centres at (i + 1/2)/N.
    ``shape`` = (Nz, Ny, Nx) overrides the cubic N^3 box (unit cell size)."""
    Nz, Ny, Nx = (N, N, N) if shape is None else shape
    cs2 = gamma * P0 / rho0
    z, y, x = np.meshgrid((np.arange(Nz) + 0.5) / Nz, (np.arange(Ny) + 0.5) / Ny,
                          (np.arange(Nx) + 0.5) / Nx, indexing="ij")
    phase = 2.0 * np.pi * (k[0] * x + k[1] * y + k[2] * z)
    drho = rho0 * amplitude * np.sin(phase)
    return conserved(rho0 + drho, 0.0, 0.0, 0.0, P0 + cs2 * drho, gamma)


def lognormal(N: int, seed: int, sigma_ln: float = 1.0, vel_sigma_rel: float = 0.3,
              P0: float = 1.0, gamma: float = GAMMA):
    """Rough synthetic state: mean-one lognormal density rho = exp(s g - s^2/2)
    with g ~ N(0, 1) iid per cell, Gaussian velocity components with standard
    deviation vel_sigma_rel * sqrt(gamma P0 / 1), uniform pressure P0."""
    r = rng(seed)
    g = r.standard_normal((N, N, N))
    rho = np.exp(sigma_ln * g - 0.5 * sigma_ln * sigma_ln)
    cs0 = math.sqrt(gamma * P0)
    v = r.standard_normal((3, N, N, N)) * (vel_sigma_rel * cs0)
    return conserved(rho, v[0], v[1], v[2], P0, gamma)


def smooth_random(N: int, seed: int, amplitude: float = 0.2, modes: int = 4,
                  rho0: float = 1.0, P0: float = 1.0, vel: float = 0.3,
                  gamma: float = GAMMA):
    """Smooth periodic state: a few random-phase Fourier modes with integer
    wavevectors (|k_i| <= 2) in density, pressure and all three velocities."""
    r = rng(seed)
    z, y, x = np.meshgrid((np.arange(N) + 0.5) / N, (np.arange(N) + 0.5) / N,
                          (np.arange(N) + 0.5) / N, indexing="ij")

    def field_():
        f = np.zeros((N, N, N))
        for _ in range(modes):
            k = r.integers(-2, 3, size=3)
            ph = r.uniform(0, 2 * np.pi)
            a = r.uniform(-1, 1)
            f += a * np.sin(2 * np.pi * (k[0] * x + k[1] * y + k[2] * z) + ph)
        return f / modes

    rho = rho0 * (1.0 + amplitude * field_())
    P = P0 * (1.0 + amplitude * field_())
    vx, vy, vz = (vel * field_() for _ in range(3))
    return conserved(rho, vx, vy, vz, P, gamma)


def sedov_lognormal(N: int, seed: int, sigma_ln: float = 0.5, E: float = 1.0,
                    P_bg: float = 1e-5, gamma: float = GAMMA):
    """Point blast on a lognormal background (Sec. 4.3 set-up, scaled): the
    energy E is deposited as thermal energy in the central 2^3 cells (indices
    N/2-1 and N/2 on every axis), background pressure P_bg, gas at rest, unit
    box so dh = 1/N."""
    r = rng(seed)
    g = r.standard_normal((N, N, N))
    rho = np.exp(sigma_ln * g - 0.5 * sigma_ln * sigma_ln)
    u = conserved(rho, 0.0, 0.0, 0.0, P_bg, gamma)
    dh = 1.0 / N
    c = slice(N // 2 - 1, N // 2 + 1)
    u[4, c, c, c] = E / (8.0 * dh ** 3)
    return u


# ---------------------------------------------------------------------------
# uneven batch of independent periodic boxes
# ---------------------------------------------------------------------------

@dataclass
class BoxSet:
    """Independent periodic boxes of mixed edge, each with its own zone size."""
    grids: list = field(default_factory=list)   # each (5, n, n, n) FP64
    dh: list = field(default_factory=list)


def sound_wave_boxes(counts=(2286, 1143, 571), edges=(8, 16, 32), seed: int = 4,
                     amplitude: float = 1e-3, rho0: float = 1.0, P0: float = 0.6,
                     gamma: float = GAMMA, modes: int = 4) -> BoxSet:
    """Independent unit periodic boxes of mixed sizes (counts per edge), each
    holding one traveling fundamental sound wave plus ``modes`` random-phase
    traveling modes with integer wavevectors |k_i| <= 2, normalised to a total
    relative density amplitude ``amplitude``; adiabatic dP = c_s^2 drho and
    velocity c_s (drho / rho0) k_hat per mode (Sec. 4.1 background)."""
    r = rng(seed)
    cs = math.sqrt(gamma * P0 / rho0)
    out = BoxSet()
    order = []
    for e, c in zip(edges, counts):
        order += [e] * c
    for n in order:
        z, y, x = np.meshgrid((np.arange(n) + 0.5) / n, (np.arange(n) + 0.5) / n,
                              (np.arange(n) + 0.5) / n, indexing="ij")
        ks = [np.array([1, 0, 0])]
        amps = [1.0]
        phs = [0.0]
        for _ in range(modes):
            k = r.integers(-2, 3, size=3)
            while not k.any():
                k = r.integers(-2, 3, size=3)
            ks.append(k)
            amps.append(r.uniform(0.2, 1.0))
            phs.append(r.uniform(0, 2 * np.pi))
        norm = amplitude / sum(amps)
        drho = np.zeros((n, n, n))
        v = np.zeros((3, n, n, n))
        for k, a, ph in zip(ks, amps, phs):
            w = norm * a * np.sin(2 * np.pi * (k[0] * x + k[1] * y + k[2] * z) + ph)
            drho += rho0 * w
            kh = k / np.linalg.norm(k)
            for ax in range(3):
                v[ax] += cs * w * kh[ax]
        out.grids.append(conserved(rho0 + drho, v[0], v[1], v[2], P0 + cs * cs * drho, gamma))
        out.dh.append(1.0 / n)
    return out


# ---------------------------------------------------------------------------
# multi-level patch hierarchy (static), ghost zones pre-filled
# ---------------------------------------------------------------------------

@dataclass
class MultiLevel:
    """A static octree of 8^3 patches over the periodic unit box.

    ``patches`` lists (level, px, py, pz) patch coordinates; ``ghosted`` holds
    the (5, 14, 14, 14) FP64 ghosted block of every patch; ``dh`` the zone
    size of each patch (1 / (base * 2^level)).  ``group_blocks()`` gives the
    same hierarchy as 2^3 patch groups (16^3 blocks, 22^3 ghosted)."""
    base: int
    patches: list = field(default_factory=list)
    ghosted: np.ndarray | None = None
    dh: np.ndarray | None = None
    rho_f: object = None
    P0: float = 1.0
    gamma: float = GAMMA

    @property
    def levels(self):
        return np.array([p[0] for p in self.patches])

    def closing(self, edge: int = 8):
        """Closing-step rows of every level pair (layout.closing_tables) for
        the hierarchy as 8^3 patches (edge 8, blocks in ``patches`` order) or
        as 2^3 patch groups (edge 16, blocks in ``group_blocks`` order)."""
        from . import layout
        if edge == 8:
            idx = {p: i for i, p in enumerate(self.patches)}
            locate = lambda l, x, y, z: (idx[(l, x, y, z)], (0, 0, 0))
        else:
            groups = self._group_list()
            gidx = {g: i for i, g in enumerate(groups)}
            locate = lambda l, x, y, z: (gidx[(l, x // 2, y // 2, z // 2)],
                                         (8 * (x & 1), 8 * (y & 1), 8 * (z & 1)))
        return layout.closing_tables(self.patches, self.base // 8, locate)

    def _group_list(self):
        by_lev = {}
        for lev, px, py, pz in self.patches:
            by_lev.setdefault(lev, set()).add((px // 2, py // 2, pz // 2))
        return [(lev, *g) for lev in sorted(by_lev)
                for g in sorted(by_lev[lev], key=lambda t: (t[2], t[1], t[0]))]

    def group_blocks(self):
        """The patches as 2^3 patch groups (Sec. 3.1): every family of eight
        siblings (level >= 1), and every aligned 2^3 set of root patches,
        becomes one 16^3 block with three ghost zones, filled by the same
        rule as the patches' (sibling copy where a same-level patch exists,
        else trilinear from the next coarser level).  Returns (groups
        [(level, gx, gy, gz)], ghosted (G, 5, 22, 22, 22), dh (G,)), groups
        ordered by level; the cells of group (l, g) are those of patches
        (l, 2g + c), c in {0, 1}^3."""
        groups = self._group_list()
        by_lev = {}
        for g in groups:
            by_lev.setdefault(g[0], []).append(g)
        for lev, gx, gy, gz in groups:
            for c in range(8):
                if (lev, 2 * gx + (c & 1), 2 * gy + (c >> 1 & 1), 2 * gz + (c >> 2)) not in self._present:
                    raise ValueError("a patch group is incomplete")
        levels = [np.array([g[1:] for g in groups if g[0] == lev], dtype=np.int64).reshape(-1, 3)
                  for lev in range(max(by_lev) + 1)]
        g, dh = _ghosted_blocks(self, levels, 16)
        return groups, g, dh


def _ghosted_blocks(ml, levels, e):
    """Ghosted blocks of edge e (8: patches, 16: 2^3 patch groups) at the block
    coordinates levels[l] (array [P, 3]) of each level: cells take the field
    at their centres where a same-level patch covers them, else the trilinear
    interpolant of the next coarser level's cell centres (conserved
    variables; gas at rest, P = P0)."""
    n = 8
    m = e + 6
    total = sum(len(b) for b in levels)
    g = np.empty((total, 5, m, m, m))
    dh = np.empty(total)
    off = np.arange(m) - 3 + 0.5  # ghosted cell centres in units of h, relative to the block
    # patch index (relative to the block's first patch, +1) of each ghosted cell
    reg = (np.arange(m) - 3) // n + 1
    nr = e // n + 2
    base_i = 0
    for lev, bcs in enumerate(levels):
        if len(bcs) == 0:
            continue
        h = 1.0 / (ml.base * 2 ** lev)
        xs, ys, zs = [(bcs[:, a, None] * e + off[None, :]) * h for a in range(3)]
        fine = ml.rho_f(xs % 1.0, ys % 1.0, zs % 1.0)
        if lev > 0:
            # cells whose same-level patch does not exist: interpolate from the
            # coarser level's cell centres (trilinear, periodic)
            npl = ml.base * 2 ** lev // n
            q = e // n
            have = np.array([[((lev, (q * bx + rx - 1) % npl, (q * by + ry - 1) % npl,
                                (q * bz + rz - 1) % npl) in ml._present)
                              for rz in range(nr) for ry in range(nr) for rx in range(nr)]
                             for bx, by, bz in bcs]).reshape(-1, nr, nr, nr)
            cover = have[:, reg[:, None, None], reg[None, :, None], reg[None, None, :]]
            need = np.nonzero(~cover.reshape(len(bcs), -1).all(axis=1))[0]
            if need.size:
                H = 2.0 * h
                # per axis: coarse cell below each fine centre and the weight
                f_ = [a[need] / H - 0.5 for a in (xs, ys, zs)]
                i_ = [np.floor(a) for a in f_]
                t_ = [a - b for a, b in zip(f_, i_)]
                interp = np.zeros((need.size, m, m, m))
                for dz_ in (0, 1):
                    for dy_ in (0, 1):
                        for dx_ in (0, 1):
                            w = [t if d else 1 - t for t, d in zip(t_, (dx_, dy_, dz_))]
                            wgt = w[2][:, :, None, None] * w[1][:, None, :, None] * w[0][:, None, None, :]
                            interp += wgt * ml.rho_f(((i_[0] + dx_ + 0.5) * H) % 1.0,
                                                     ((i_[1] + dy_ + 0.5) * H) % 1.0,
                                                     ((i_[2] + dz_ + 0.5) * H) % 1.0)
                fine[need] = np.where(cover[need], fine[need], interp)
        k = len(bcs)
        g[base_i:base_i + k] = np.moveaxis(
            conserved(fine, 0.0, 0.0, 0.0, np.full(fine.shape, ml.P0), ml.gamma), 0, 1)
        dh[base_i:base_i + k] = h
        base_i += k
    return g, dh


def _gaussian_field(centres, amps, radii):
    """rho on tensor-product point sets: rho(xs, ys, zs) with per-block axis
    coordinates of shape (P, k) returns (P, k, k, k) values (z, y, x order) of
    1 + sum_k A_k exp(-d^2 / 2 r_k^2), d the periodic distance in the unit box.
    Each Gaussian factorises into three 1-D factors, and a factor is cut to 0
    where that axis' distance exceeds 8 r_k (below exp(-32) relative): a
    rule per cell, so the value of a cell does not depend on which block it
    is evaluated in.  Blocks with no cell inside the cut skip the Gaussian."""
    def rho(xs, ys, zs):
        P, k = xs.shape
        out = np.ones((P, k, k, k))
        for (cx, cy, cz), amp, r in zip(centres, amps, radii):
            d = [(a - c + 0.5) % 1.0 - 0.5 for a, c in ((xs, cx), (ys, cy), (zs, cz))]
            inside = [np.abs(x) <= 8.0 * r for x in d]
            sel = np.nonzero(inside[0].any(axis=1) & inside[1].any(axis=1) & inside[2].any(axis=1))[0]
            if sel.size == 0:
                continue
            f = [np.where(ins[sel], np.exp(-(x[sel] ** 2) / (2.0 * r * r)), 0.0)
                 for x, ins in zip(d, inside)]
            out[sel] += amp * (f[2][:, :, None, None] * f[1][:, None, :, None] *
                               f[0][:, None, None, :])
        return out
    return rho


def multilevel(base: int = 128, n_over: int = 32, seed: int = 3, max_level: int = 3,
               radius: float = 0.032, P0: float = 1.0, gamma: float = GAMMA) -> MultiLevel:
    """Base grid of base^3 cells (8^3 patches) with up to ``max_level`` refined
    levels around ``n_over`` Gaussian overdensities rho = 1 + sum A_k
    exp(-r^2 / 2 r_k^2): centres uniform, A_k log-uniform in [10, 1e3], r_k =
    radius * U(0.5, 1.5).  A patch of level l is refined into its 2^3
    children when its densest cell reaches 8^(l+1) (the paper's cosmological
    criterion rho_l >= 8^(l+1) rho_b, Sec. 5) and its 26 neighbours exist on
    level l (proper nesting, Sec. 2.1).  Gas at rest, P = P0.

    Cells take the density at their centres on every level.  Ghost cells
    covered by a patch of the same level are copied from it (sibling copy);
    the others are trilinearly interpolated from the cell centres of the next
    coarser level (conserved variables).  Ghost values therefore equal the
    analytic field sampled at same-level centres, or its trilinear
    interpolant one level down."""
    r = rng(seed)
    centres = r.uniform(0, 1, size=(n_over, 3))
    amps = 10.0 ** r.uniform(1, 3, size=n_over)
    radii = radius * r.uniform(0.5, 1.5, size=n_over)
    rho_f = _gaussian_field(centres, amps, radii)
    n = 8
    ml = MultiLevel(base=base)

    def axes_of(pc, h, offs):
        # per-axis cell-centre coordinates of the patches pc [P, 3] (px, py,
        # pz) at offsets offs (in cells) from each patch corner: 3 x [P, k]
        return [(pc[:, a, None] * n + offs[None, :]) * h for a in range(3)]

    # level 0: every patch; refine level by level
    npb = base // n
    cur = np.array([(px, py, pz) for pz in range(npb) for py in range(npb) for px in range(npb)],
                   dtype=np.int64)
    levels = [cur]
    for lev in range(max_level):
        h = 1.0 / (base * 2 ** lev)
        xs, ys, zs = axes_of(cur, h, np.arange(n) + 0.5)
        hot = cur[rho_f(xs, ys, zs).reshape(len(cur), -1).max(axis=1) >= 8.0 ** (lev + 1)]
        # proper nesting (Sec. 2.1): a patch is refined only if its 26
        # neighbours exist on its level, so that refinement never jumps more
        # than one level across adjacent patches
        have = set(map(tuple, cur.tolist()))
        npl = npb << lev
        nest = [all(((p[0] + rx) % npl, (p[1] + ry) % npl, (p[2] + rz) % npl) in have
                    for rz in (-1, 0, 1) for ry in (-1, 0, 1) for rx in (-1, 0, 1))
                for p in hot.tolist()]
        hot = hot[np.array(nest, dtype=bool)] if len(hot) else hot
        kids = np.array([(cx, cy, cz) for cz in range(2) for cy in range(2) for cx in range(2)],
                        dtype=np.int64)
        cur = (2 * hot[:, None, :] + kids[None, :, :]).reshape(-1, 3)
        levels.append(cur)
        if len(cur) == 0:
            break
    allp = [(lev, int(p[0]), int(p[1]), int(p[2])) for lev, pcs in enumerate(levels) for p in pcs]
    ml.patches = allp
    ml._present = set(allp)
    ml.rho_f, ml.P0, ml.gamma = rho_f, P0, gamma
    g, dh = _ghosted_blocks(ml, levels, n)
    ml.ghosted = g
    ml.dh = dh
    return ml
