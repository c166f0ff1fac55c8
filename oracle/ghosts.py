"""Coarse-fine ghost zones for the oracle (test infrastructure only).

Sec. 2.2: a patch's ghost cells come from the sibling patch by direct copy
when that sibling exists, otherwise by linear interpolation with the Min-Mod
limiter from the patches one level coarser (proper nesting guarantees that
level exists there).  Written with numpy in FP64 (or in the dtype of the
inputs, to mirror a lower-precision run operation by operation).

Reading of the interpolation (the paper names only the method): for each
conserved variable separately, a fine cell lying in coarse cell c takes

    u_c + dx s_x + dy s_y + dz s_z,   s_d = minmod(u_{c+e_d} - u_c, u_c - u_{c-e_d})

summed in the order x, y, z, with d_ = -1/4 for the lower and +1/4 for the
upper of the two fine cells along that axis (the fine centres sit a quarter
of a coarse cell from the coarse centre).  minmod(a, b) is 0 unless a and b
are both positive or both negative, then the one of smaller magnitude (b on
a tie).  The eight fine cells of a coarse cell average to u_c.
"""
from __future__ import annotations

import numpy as np

NVAR = 5
GHOST = 3


def minmod(a, b):
    """Min-Mod limiter, elementwise (Sec. 2.2)."""
    a = np.asarray(a)
    b = np.asarray(b)
    same = ((a > 0) & (b > 0)) | ((a < 0) & (b < 0))
    return np.where(same, np.where(np.abs(a) < np.abs(b), a, b), np.zeros_like(a))


def coarse_to_fine(coarse, fz, fy, fx):
    """Values of fine cells with fine-level indices (fz, fy, fx) (integer
    arrays of one shape) interpolated from the periodic coarse level
    ``coarse`` (5, Nz, Ny, Nx): coarse cell c = floor(f / 2), position
    -1/4 (f even) or +1/4 (f odd) of a coarse cell from its centre."""
    coarse = np.asarray(coarse)
    _, Nz, Ny, Nx = coarse.shape
    cz, cy, cx = fz // 2, fy // 2, fx // 2
    q = np.array(0.25, dtype=coarse.dtype)
    dz = np.where(fz % 2 == 1, q, -q)
    dy = np.where(fy % 2 == 1, q, -q)
    dx = np.where(fx % 2 == 1, q, -q)

    def at(z, y, x):
        return coarse[:, z % Nz, y % Ny, x % Nx]

    u = at(cz, cy, cx)
    sx = minmod(at(cz, cy, cx + 1) - u, u - at(cz, cy, cx - 1))
    sy = minmod(at(cz, cy + 1, cx) - u, u - at(cz, cy - 1, cx))
    sz = minmod(at(cz + 1, cy, cx) - u, u - at(cz - 1, cy, cx))
    return ((u + dx * sx) + dy * sy) + dz * sz


def two_level_ghosted_blocks(coarse, fine_box, origin, n: int):
    """Ghosted blocks of a fine region: ``fine_box`` (5, Lz, Ly, Lx) holds the
    fine level (twice the coarse resolution, periodic with 2 N per axis) on
    the box of fine cells starting at ``origin`` (oz, oy, ox); the box is cut
    into n^3 blocks (x fastest).  A ghost cell inside the box is copied (the
    sibling exists), one outside is interpolated from ``coarse``.  Returns
    (B, 5, n+6, n+6, n+6)."""
    coarse = np.asarray(coarse)
    fine_box = np.asarray(fine_box)
    _, Lz, Ly, Lx = fine_box.shape
    oz, oy, ox = origin
    m = n + 2 * GHOST
    r = np.arange(m) - GHOST
    out = []
    for bz in range(Lz // n):
        for by in range(Ly // n):
            for bx in range(Lx // n):
                # box-relative indices of the ghosted block's cells
                kz, ky, kx = np.meshgrid(bz * n + r, by * n + r, bx * n + r, indexing="ij")
                inside = (kz >= 0) & (kz < Lz) & (ky >= 0) & (ky < Ly) & (kx >= 0) & (kx < Lx)
                blk = np.empty((NVAR, m, m, m), dtype=fine_box.dtype)
                blk[:, inside] = fine_box[:, kz[inside], ky[inside], kx[inside]]
                out_ = ~inside
                blk[:, out_] = coarse_to_fine(coarse, oz + kz[out_], oy + ky[out_], ox + kx[out_])
                out.append(blk)
    return np.stack(out)
