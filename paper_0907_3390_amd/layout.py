"""Host-side block bookkeeping: block grids, neighbour tables, offsets.

Pure integer bookkeeping and array reshapes (no arithmetic of the scheme):
a periodic domain, or a set of independent periodic boxes, is cut into cubic
blocks of edge 8 or 16 (one 8^3 patch, or a 2^3 patch group as in the
paper's Sec. 3.1); every block gets the 27-entry table of the blocks that
cover its neighbourhood, which the device ghost fill reads.  Blocks are
numbered x fastest, then y, then z, box after box, or, for a periodic grid,
optionally along a Morton (Z-order) curve, so that blocks with nearby numbers
are nearby in space.
"""
from __future__ import annotations

import numpy as np

NVAR = 5
GHOST = 3


def periodic_neighbors(nbx: int, nby: int, nbz: int, base: int = 0) -> np.ndarray:
    """[nb, 27] int32 table for an nbx x nby x nbz periodic block grid.
    Entry r = (rx+1) + 3(ry+1) + 9(rz+1) names the block at offset (rx, ry, rz)."""
    bx, by, bz = np.meshgrid(np.arange(nbx), np.arange(nby), np.arange(nbz), indexing="ij")
    bx, by, bz = bx.transpose(2, 1, 0).ravel(), by.transpose(2, 1, 0).ravel(), bz.transpose(2, 1, 0).ravel()
    nb = nbx * nby * nbz
    out = np.empty((nb, 27), dtype=np.int32)
    for rz in (-1, 0, 1):
        for ry in (-1, 0, 1):
            for rx in (-1, 0, 1):
                r = (rx + 1) + 3 * (ry + 1) + 9 * (rz + 1)
                out[:, r] = base + ((bx + rx) % nbx) + nbx * (((by + ry) % nby) + nby * ((bz + rz) % nbz))
    return out


def morton_perm(nbx: int, nby: int, nbz: int) -> np.ndarray:
    """perm[k] = x-fastest linear index of the k-th block along the Morton
    curve (bits of bx, by, bz interleaved, x lowest) of an nbx x nby x nbz grid."""
    lin = np.arange(nbx * nby * nbz, dtype=np.int64)
    b = [lin % nbx, (lin // nbx) % nby, lin // (nbx * nby)]
    key = np.zeros_like(lin)
    for bit in range(21):
        for a in range(3):
            key |= ((b[a] >> bit) & 1) << (3 * bit + a)
    return np.argsort(key, kind="stable")


def grid_to_blocks(grid: np.ndarray, n: int, perm=None) -> np.ndarray:
    """(5, Nz, Ny, Nx) -> (B, 5, n, n, n) interiors, blocks x fastest (or in
    the order perm, block k being linear block perm[k])."""
    _, Nz, Ny, Nx = grid.shape
    nbz, nby, nbx = Nz // n, Ny // n, Nx // n
    if nbz * n != Nz or nby * n != Ny or nbx * n != Nx:
        raise ValueError("grid extents must be multiples of the block edge")
    g = grid.reshape(NVAR, nbz, n, nby, n, nbx, n)
    out = g.transpose(1, 3, 5, 0, 2, 4, 6).reshape(nbz * nby * nbx, NVAR, n, n, n)
    return np.ascontiguousarray(out if perm is None else out[perm])


def blocks_to_grid(blocks: np.ndarray, shape, perm=None) -> np.ndarray:
    """(B, 5, n, n, n) -> (5, Nz, Ny, Nx), the inverse of grid_to_blocks."""
    _, Nz, Ny, Nx = shape
    n = blocks.shape[2]
    nbz, nby, nbx = Nz // n, Ny // n, Nx // n
    if perm is not None:
        lin = np.empty_like(blocks)
        lin[perm] = blocks
        blocks = lin
    g = blocks.reshape(nbz, nby, nbx, NVAR, n, n, n).transpose(3, 0, 4, 1, 5, 2, 6)
    return np.ascontiguousarray(g.reshape(NVAR, Nz, Ny, Nx))


class BlockSet:
    """Layout of a ragged set of blocks: edges, offsets, zone sizes, neighbours.

    ``in_off`` and ``out_off`` are element offsets of each block's ghosted
    (5 (e+6)^3) and interior (5 e^3) data in two flat buffers, blocks packed
    in order.  ``dh`` is the zone size of each block.
    """

    def __init__(self, edges, dh, nbr):
        self.perm = None  # block k is linear block perm[k] (periodic grids)
        self.edges = np.asarray(edges, dtype=np.int32)
        self.dh = np.asarray(dh, dtype=np.float64)
        self.nbr = np.ascontiguousarray(nbr, dtype=np.int32)
        n = self.edges.astype(np.int64)
        in_sizes = NVAR * (n + 2 * GHOST) ** 3
        out_sizes = NVAR * n ** 3
        self.in_off = np.concatenate([[0], np.cumsum(in_sizes)[:-1]]).astype(np.int64)
        self.out_off = np.concatenate([[0], np.cumsum(out_sizes)[:-1]]).astype(np.int64)
        self.in_total = int(in_sizes.sum())
        self.out_total = int(out_sizes.sum())

    @property
    def n_blocks(self) -> int:
        return int(self.edges.size)

    @property
    def uniform_edge(self):
        e = np.unique(self.edges)
        return int(e[0]) if e.size == 1 else None

    @property
    def cells(self) -> int:
        return int((self.edges.astype(np.int64) ** 3).sum())

    def pack_interior(self, blocks) -> np.ndarray:
        """List of (5, e, e, e) interiors -> flat buffer."""
        return np.concatenate([np.ascontiguousarray(b).ravel() for b in blocks])

    def unpack_interior(self, flat) -> list:
        out = []
        for b in range(self.n_blocks):
            e = int(self.edges[b])
            o = int(self.out_off[b])
            out.append(flat[o:o + NVAR * e ** 3].reshape(NVAR, e, e, e))
        return out


def periodic_grid_blockset(N, n: int, dh: float | None = None, curve: str = "linear") -> BlockSet:
    """A periodic box of N^3 (or (Nz, Ny, Nx)) cells cut into n^3 blocks,
    numbered x fastest (curve "linear") or along the Morton curve ("morton";
    bs.perm then maps block k to linear block perm[k], for grid_to_blocks and
    blocks_to_grid)."""
    Nz, Ny, Nx = (N, N, N) if np.isscalar(N) else N
    nbx, nby, nbz = Nx // n, Ny // n, Nz // n
    nbr = periodic_neighbors(nbx, nby, nbz)
    nb = nbx * nby * nbz
    perm = None
    if curve == "morton":
        perm = morton_perm(nbx, nby, nbz)
        inv = np.empty_like(perm)
        inv[perm] = np.arange(nb)
        nbr = inv[nbr[perm]].astype(np.int32)
    elif curve != "linear":
        raise ValueError(f"unknown curve {curve!r}")
    bs = BlockSet(np.full(nb, n), np.full(nb, 1.0 / Nx if dh is None else dh), nbr)
    bs.perm = perm
    return bs


def boxes_blockset(box_edges, block_edge_for, dhs) -> BlockSet:
    """Independent periodic boxes; box i of edge L_i is cut into blocks of
    edge block_edge_for(L_i), each box periodic on itself."""
    edges, dh, nbrs = [], [], []
    base = 0
    for L, h in zip(box_edges, dhs):
        e = block_edge_for(int(L))
        k = int(L) // e
        nbrs.append(periodic_neighbors(k, k, k, base))
        edges += [e] * k ** 3
        dh += [h] * k ** 3
        base += k ** 3
    return BlockSet(edges, dh, np.concatenate(nbrs))


def boxes_to_blocks(grids, block_edge_for) -> list:
    """Interiors of every box cut into blocks, in BlockSet order."""
    out = []
    for g in grids:
        L = g.shape[1]
        e = block_edge_for(L)
        out += list(grid_to_blocks(g, e))
    return out


def blocks_to_boxes(blocks, box_edges, block_edge_for) -> list:
    out = []
    i = 0
    for L in box_edges:
        e = block_edge_for(int(L))
        k = int(L) // e
        out.append(blocks_to_grid(np.stack(blocks[i:i + k ** 3]), (NVAR, L, L, L)))
        i += k ** 3
    return out


def two_level(Nc: int, origin, shape, n: int, curve: str = "linear"):
    """A coarse-fine configuration: the periodic coarse level of Nc^3 cells as
    8^3 patches (x fastest), and a box of fine cells (the level one finer, 2 Nc
    cells per axis) of shape (Lz, Ly, Lx) at fine-cell origin (oz, oy, ox), cut
    into n^3 blocks (x fastest).  The origin and shape must be multiples of n,
    so that blocks are aligned like octree patches (n = 8) or patch groups
    (n = 16), and the box must not wrap around the domain.

    Returns (coarse BlockSet, fine BlockSet whose sibling table is -1 outside
    the box, cnbr [B, 27] coarse patches around each fine block's parent,
    corigin [B, 3] the fine block's corner in coarse cells relative to its
    parent's corner, x first).  curve "morton" numbers the fine blocks along
    the Morton curve instead (fine.perm then maps block k to the x-fastest
    block perm[k] of the box, for grid_to_blocks)."""
    Lz, Ly, Lx = shape
    oz, oy, ox = origin
    if any(v % n for v in (Lz, Ly, Lx, oz, oy, ox)) or Nc % 8:
        raise ValueError("box origin and shape must be multiples of the block edge")
    if any(o < 0 or o + L > 2 * Nc for o, L in ((oz, Lz), (oy, Ly), (ox, Lx))):
        raise ValueError("the box must lie inside the domain")
    coarse = periodic_grid_blockset(Nc, 8, dh=1.0 / Nc)
    npc = Nc // 8
    nbx, nby, nbz = Lx // n, Ly // n, Lz // n
    nb = nbx * nby * nbz
    nbr = np.full((nb, 27), -1, dtype=np.int32)
    cnbr = np.empty((nb, 27), dtype=np.int32)
    corigin = np.empty((nb, 3), dtype=np.int32)
    for b in range(nb):
        bx, by, bz = b % nbx, (b // nbx) % nby, b // (nbx * nby)
        corner = [(ox + bx * n) // 2, (oy + by * n) // 2, (oz + bz * n) // 2]  # coarse cells
        parent = [c // 8 for c in corner]
        corigin[b] = [c - 8 * p for c, p in zip(corner, parent)]
        for rz in (-1, 0, 1):
            for ry in (-1, 0, 1):
                for rx in (-1, 0, 1):
                    r = (rx + 1) + 3 * (ry + 1) + 9 * (rz + 1)
                    sx, sy, sz = bx + rx, by + ry, bz + rz
                    if 0 <= sx < nbx and 0 <= sy < nby and 0 <= sz < nbz:
                        nbr[b, r] = sx + nbx * (sy + nby * sz)
                    px, py, pz = ((parent[0] + rx) % npc, (parent[1] + ry) % npc,
                                  (parent[2] + rz) % npc)
                    cnbr[b, r] = px + npc * (py + npc * pz)
    perm = None
    if curve == "morton":
        perm = morton_perm(nbx, nby, nbz)
        inv = np.empty_like(perm)
        inv[perm] = np.arange(nb)
        nbr = np.where(nbr[perm] >= 0, inv[np.maximum(nbr[perm], 0)], -1).astype(np.int32)
        cnbr, corigin = cnbr[perm], corigin[perm]
    elif curve != "linear":
        raise ValueError(f"unknown curve {curve!r}")
    fine = BlockSet(np.full(nb, n), np.full(nb, 0.5 / Nc), nbr)
    fine.perm = perm
    return coarse, fine, cnbr, corigin


# ---------------------------------------------------------------------------
# closing step of a level pair (Sec. 2.1 step 3, Sec. 3.1): patch-boundary
# flux records, restriction rows and coarse-fine face rows
# ---------------------------------------------------------------------------

PATCH = 8
# columns of a face row (see closing_tables)
FACE_COLS = ("c", "d", "s", "qc", "oa", "ob", "f", "qf")


def flux_record_size(edge: int) -> int:
    """Values in one block's patch-boundary flux record: 3 axes x (edge/8 + 1)
    planes x 5 variables x edge^2 face cells."""
    return 3 * (edge // PATCH + 1) * NVAR * edge * edge


def flux_offsets(edges) -> np.ndarray:
    """Element offsets of the blocks' flux records packed in block order."""
    sizes = np.array([flux_record_size(int(e)) for e in edges], dtype=np.int64)
    return np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)


def _face_axes(d: int):
    """The two axes of a face normal to d, higher-numbered first."""
    return {0: (2, 1), 1: (2, 0), 2: (1, 0)}[d]


def closing_tables(patches, base: int, locate):
    """Restriction and flux-correction rows of every level pair of a static
    octree of 8^3 patches over a periodic box of ``base`` root patches per
    axis.

    patches: iterable of (level, px, py, pz); a patch of level l > 0 is a
    child of (l-1, px//2, py//2, pz//2), and children come in complete
    families of eight.  locate(level, px, py, pz) -> (block, (ox, oy, oz))
    names the block holding the patch and the patch's cell offset in it (a
    patch is its own block, offset 0; or one octant of a 16^3 patch group).

    Returns {level l: (restrict_rows, face_rows, pass_count)} for every l
    with a finer level:
      restrict_rows int32 [R, 5] (f, c, ox, oy, oz): fine block f (level
        l+1) averages into coarse block c (level l) at coarse-cell offset
        (ox, oy, oz); one row per fine block.
      face_rows int32 [F, 8] (c, d, s, qc, oa, ob, f, qf): coarse block c
        holds an unrefined patch whose face along axis d (s = 1: its + face,
        s = 0: its - face) is a coarse-fine interface at plane qc of c's flux
        record; the face cells [oa, oa + e_f/2) x [ob, ob + e_f/2) of that
        plane (face axes higher-numbered first) are covered by plane qf of
        fine block f (edge e_f).  Rows are sorted by pass 2d + s, then c, f.
      pass_count int32 [6]: rows of each pass.
    """
    present = set(tuple(int(v) for v in p) for p in patches)
    levels = sorted(set(p[0] for p in present))
    out = {}
    for lev in levels:
        if lev + 1 not in levels:
            continue
        n_l = base << lev

        def refined(px, py, pz):
            return (lev + 1, 2 * px, 2 * py, 2 * pz) in present

        rrows, seen = [], set()
        for (l1, cx, cy, cz) in sorted(p for p in present if p[0] == lev + 1):
            fb, fo = locate(l1, cx, cy, cz)
            if any(fo) or fb in seen:
                continue  # one row per fine block, from its corner child
            seen.add(fb)
            cb, co = locate(lev, cx // 2, cy // 2, cz // 2)
            bits = (cx & 1, cy & 1, cz & 1)
            rrows.append((fb, cb) + tuple(co[a] + 4 * bits[a] for a in range(3)))
        frows = []
        for (l0, px, py, pz) in sorted(p for p in present if p[0] == lev):
            if refined(px, py, pz):
                continue
            P = (px, py, pz)
            cb, co = locate(lev, px, py, pz)
            for d in range(3):
                hi, lo = _face_axes(d)
                for s in (0, 1):
                    Q = list(P)
                    Q[d] = (P[d] + (1 if s else -1)) % n_l
                    if (lev, *Q) not in present or not refined(*Q):
                        continue
                    done = set()
                    for c in range(8):
                        bit = (c & 1, (c >> 1) & 1, c >> 2)
                        if bit[d] != (0 if s else 1):
                            continue  # children of Q that touch P
                        C = tuple(2 * Q[a] + bit[a] for a in range(3))
                        fb, fo = locate(lev + 1, *C)
                        if fb in done:
                            continue
                        done.add(fb)
                        qc = (co[d] + (PATCH if s else 0)) // PATCH
                        qf = (fo[d] + (0 if s else PATCH)) // PATCH
                        # the fine block's face corner, in coarse cells of P's face
                        oa = co[hi] + (PATCH * bit[hi] - fo[hi]) // 2
                        ob = co[lo] + (PATCH * bit[lo] - fo[lo]) // 2
                        frows.append((cb, d, s, qc, oa, ob, fb, qf))
        frows.sort(key=lambda r: (2 * r[1] + r[2], r[0], r[6]))
        count = np.zeros(6, dtype=np.int32)
        for r in frows:
            count[2 * r[1] + r[2]] += 1
        out[lev] = (np.array(rrows, dtype=np.int32).reshape(-1, 5),
                    np.array(frows, dtype=np.int32).reshape(-1, 8), count)
    return out


def group_face_rows(face_rows):
    """Face rows regrouped for tvd_close_level: sorted by coarse block, then
    pass 2d + s, then fine block; returns (rows int32 [F, 8], start int32
    [G + 1]) with group g = rows[start[g]:start[g+1]] naming one coarse
    block."""
    fr = np.asarray(face_rows, dtype=np.int32).reshape(-1, 8)
    if len(fr) == 0:
        return fr.copy(), np.zeros(1, dtype=np.int32)
    order = np.lexsort((fr[:, 6], 2 * fr[:, 1] + fr[:, 2], fr[:, 0]))
    rows = np.ascontiguousarray(fr[order])
    cut = np.nonzero(np.diff(rows[:, 0]))[0] + 1
    start = np.concatenate([[0], cut, [len(rows)]]).astype(np.int32)
    return rows, start


class RefinedLevels:
    """A two-level periodic hierarchy: the coarse level of Nc^3 cells as 8^3
    patches numbered x fastest, and the refined patches ``refined[pz, py, px]``
    (a boolean array of Nc/8 per axis) replaced on the next level by fine
    blocks of edge n (8: the eight child patches, 16: one 2^3 patch group),
    numbered refined patch by refined patch (pz slowest, px fastest), then
    block by block inside the patch (z slowest, x fastest).

    Attributes: coarse, fine (BlockSets; the fine sibling table is -1 where
    the neighbouring region is not refined), cnbr [B, 27] and corigin [B, 3]
    (for the coarse-fine ghost fill: the coarse patches around each fine
    block's parent and the block's corner in coarse cells inside its parent,
    x first), origins [B, 3] fine-cell corners (z, y, x), patches (the
    octree, for closing_tables), locate."""

    def __init__(self, Nc: int, refined, n: int):
        refined = np.asarray(refined, dtype=bool)
        npc = Nc // PATCH
        if Nc % PATCH or refined.shape != (npc, npc, npc) or n not in (8, 16):
            raise ValueError("refined must be (Nc/8,)*3 and the fine edge 8 or 16")
        self.Nc, self.n, self.refined = Nc, n, refined
        self.coarse = periodic_grid_blockset(Nc, PATCH, dh=1.0 / Nc)
        k = 2 * PATCH // n              # fine blocks per refined patch and axis
        nfb = 2 * Nc // n               # fine block grid per axis (periodic)
        ref = [tuple(int(v) for v in p) for p in np.argwhere(refined)]   # (pz, py, px)
        index, origins = {}, []
        for pz, py, px in ref:
            for bz in range(k):
                for by in range(k):
                    for bx in range(k):
                        g = (k * px + bx, k * py + by, k * pz + bz)
                        index[g] = len(origins)
                        origins.append((n * g[2], n * g[1], n * g[0]))
        nb = len(origins)
        nbr = np.full((nb, 27), -1, dtype=np.int32)
        cnbr = np.empty((nb, 27), dtype=np.int32)
        corigin = np.empty((nb, 3), dtype=np.int32)
        for g, b in index.items():
            corner = [n * g[a] // 2 for a in range(3)]       # coarse cells, x first
            parent = [c // PATCH for c in corner]
            corigin[b] = [c - PATCH * p for c, p in zip(corner, parent)]
            for rz in (-1, 0, 1):
                for ry in (-1, 0, 1):
                    for rx in (-1, 0, 1):
                        r = (rx + 1) + 3 * (ry + 1) + 9 * (rz + 1)
                        s = ((g[0] + rx) % nfb, (g[1] + ry) % nfb, (g[2] + rz) % nfb)
                        nbr[b, r] = index.get(s, -1)
                        q = ((parent[0] + rx) % npc, (parent[1] + ry) % npc, (parent[2] + rz) % npc)
                        cnbr[b, r] = q[0] + npc * (q[1] + npc * q[2])
        self.fine = BlockSet(np.full(nb, n), np.full(nb, 0.5 / Nc), nbr)
        self.cnbr, self.corigin = cnbr, corigin
        self.origins = np.array(origins, dtype=np.int64).reshape(-1, 3)
        self._index = index
        self.patches = [(0, px, py, pz) for pz in range(npc) for py in range(npc) for px in range(npc)]
        self.patches += [(1, 2 * px + (c & 1), 2 * py + (c >> 1 & 1), 2 * pz + (c >> 2))
                         for pz, py, px in ref for c in range(8)]

    def locate(self, level, px, py, pz):
        npc = self.Nc // PATCH
        if level == 0:
            return px + npc * (py + npc * pz), (0, 0, 0)
        k = 2 * PATCH // self.n
        per = self.n // PATCH           # patches per fine block and axis
        g = (px // per, py // per, pz // per)
        return self._index[g], tuple(PATCH * (v % per) for v in (px, py, pz))

    def tables(self):
        """(restrict_rows, face_rows, pass_count) of the level pair."""
        return closing_tables(self.patches, self.Nc // PATCH, self.locate)[0]


class NestedLevels:
    """A periodic hierarchy of 8^3 patches on any number of levels: level 0
    is the Nc^3 root grid, numbered x fastest; ``refined[l]`` (a boolean
    array over level l's patch grid, Nc/8 * 2^l per axis, indexed [pz, py,
    px]) marks the level-l patches refined into eight children on level l+1.
    Level l+1 numbers its patches refined parent by refined parent (pz
    slowest, px fastest), then child by child (z slowest, x fastest).

    Proper nesting (Sec. 2.1) is checked: a refined patch must exist on its
    level and so must its 26 neighbours (periodic), so that every coarse-fine
    ghost zone and flux interface has its coarse patches.

    Per level l: blocks[l] (a BlockSet; the sibling table is -1 where the
    neighbouring patch does not exist on level l), origins[l] [B, 3]
    (cell corners z, y, x on level l's grid); for l >= 1 also cnbr[l] [B, 27]
    and corigin[l] [B, 3] for the coarse-fine ghost fill (the level-(l-1)
    patches around each patch's parent, and the patch's corner in coarse
    cells inside its parent, x first).  patches and locate describe the
    octree for closing_tables.

    With n = 16 every level is held as 2^3 patch groups of 16^3 cells
    instead (Sec. 3.1): level 0 as the (Nc/16)^3 groups of the root grid, x
    fastest, and level l >= 1 as one group per refined patch of level l-1
    (its eight children), in the order of the refined patches.  blocks,
    origins, cnbr and corigin then describe the groups: cnbr names the 27
    level-(l-1) groups around the group holding the parent patch, corigin
    is the group's corner in coarse cells inside that group (0 or 8), and
    locate returns a patch's group and its cell offset in it."""

    def __init__(self, Nc: int, refined, n: int = PATCH):
        npc = Nc // PATCH
        if Nc % PATCH:
            raise ValueError("Nc must be a multiple of 8")
        if n not in (PATCH, 2 * PATCH) or (n == 2 * PATCH and Nc % n):
            raise ValueError("blocks are 8^3 patches or 16^3 patch groups (then Nc % 16 == 0)")
        self.Nc, self.n = Nc, n
        self.refined = [np.asarray(r, dtype=bool) for r in refined]
        self.n_levels = len(self.refined) + 1
        index = {(px, py, pz): px + npc * (py + npc * pz)
                 for pz in range(npc) for py in range(npc) for px in range(npc)}
        self._index = [index]
        coords = [sorted(index, key=index.get)]
        for lev, r in enumerate(self.refined):
            n_l = npc << lev
            if r.shape != (n_l, n_l, n_l):
                raise ValueError(f"refined[{lev}] must be ({n_l},)*3")
            prev = self._index[lev]
            nxt, cl = {}, []
            for pz, py, px in (tuple(int(v) for v in q) for q in np.argwhere(r)):
                if (px, py, pz) not in prev:
                    raise ValueError(f"level {lev} patch {(px, py, pz)} is refined but does not exist")
                for rz in (-1, 0, 1):
                    for ry in (-1, 0, 1):
                        for rx in (-1, 0, 1):
                            q = ((px + rx) % n_l, (py + ry) % n_l, (pz + rz) % n_l)
                            if q not in prev:
                                raise ValueError(f"level {lev} patch {(px, py, pz)} is refined "
                                                 f"but its neighbour {q} does not exist "
                                                 "(proper nesting)")
                for c in range(8):
                    ch = (2 * px + (c & 1), 2 * py + (c >> 1 & 1), 2 * pz + (c >> 2))
                    nxt[ch] = len(cl)
                    cl.append(ch)
            self._index.append(nxt)
            coords.append(cl)
        self.blocks, self.origins, self.cnbr, self.corigin = [], [], [None], [None]
        for lev, cl in enumerate(coords):
            n_l = npc << lev
            idx = self._index[lev]
            nbr = np.full((len(cl), 27), -1, dtype=np.int32)
            for b, (px, py, pz) in enumerate(cl):
                for rz in (-1, 0, 1):
                    for ry in (-1, 0, 1):
                        for rx in (-1, 0, 1):
                            q = ((px + rx) % n_l, (py + ry) % n_l, (pz + rz) % n_l)
                            nbr[b, (rx + 1) + 3 * (ry + 1) + 9 * (rz + 1)] = idx.get(q, -1)
            self.blocks.append(BlockSet(np.full(len(cl), PATCH),
                                        np.full(len(cl), 1.0 / (Nc << lev)), nbr))
            self.origins.append(np.array([(PATCH * pz, PATCH * py, PATCH * px)
                                          for px, py, pz in cl], dtype=np.int64).reshape(-1, 3))
            if lev == 0:
                continue
            n_p = npc << (lev - 1)
            prev = self._index[lev - 1]
            cnbr = np.empty((len(cl), 27), dtype=np.int32)
            corigin = np.empty((len(cl), 3), dtype=np.int32)
            for b, (px, py, pz) in enumerate(cl):
                par = (px // 2, py // 2, pz // 2)
                corigin[b] = [PATCH // 2 * (px % 2), PATCH // 2 * (py % 2), PATCH // 2 * (pz % 2)]
                for rz in (-1, 0, 1):
                    for ry in (-1, 0, 1):
                        for rx in (-1, 0, 1):
                            q = ((par[0] + rx) % n_p, (par[1] + ry) % n_p, (par[2] + rz) % n_p)
                            cnbr[b, (rx + 1) + 3 * (ry + 1) + 9 * (rz + 1)] = prev[q]
            self.cnbr.append(cnbr)
            self.corigin.append(corigin)
        self.patches = [(lev, px, py, pz) for lev, cl in enumerate(coords) for px, py, pz in cl]
        if n == 2 * PATCH:
            self._groups(coords)

    def _groups(self, coords):
        """Replace the per-patch tables by those of 2^3 patch groups."""
        Nc, n = self.Nc, self.n
        self._gindex, gcoords = [], []
        for lev, cl in enumerate(coords):
            # a group at position G holds the patches 2G + (0|1) of the level
            gl = sorted({(px // 2, py // 2, pz // 2) for px, py, pz in cl},
                        key=lambda g: (g[2], g[1], g[0]))
            self._gindex.append({g: i for i, g in enumerate(gl)})
            gcoords.append(gl)
        self.blocks, self.origins, self.cnbr, self.corigin = [], [], [None], [None]
        for lev, gl in enumerate(gcoords):
            ng = (Nc << lev) // n
            idx = self._gindex[lev]
            nbr = np.full((len(gl), 27), -1, dtype=np.int32)
            for b, (gx, gy, gz) in enumerate(gl):
                for rz in (-1, 0, 1):
                    for ry in (-1, 0, 1):
                        for rx in (-1, 0, 1):
                            q = ((gx + rx) % ng, (gy + ry) % ng, (gz + rz) % ng)
                            nbr[b, (rx + 1) + 3 * (ry + 1) + 9 * (rz + 1)] = idx.get(q, -1)
            self.blocks.append(BlockSet(np.full(len(gl), n), np.full(len(gl), 1.0 / (Nc << lev)),
                                        nbr))
            self.origins.append(np.array([(n * gz, n * gy, n * gx) for gx, gy, gz in gl],
                                         dtype=np.int64).reshape(-1, 3))
            if lev == 0:
                continue
            # group G of level lev holds the children of patch G of level lev-1,
            # which sits in group G // 2 of that level at octant G % 2
            ngp = (Nc << (lev - 1)) // n
            prev = self._gindex[lev - 1]
            cnbr = np.empty((len(gl), 27), dtype=np.int32)
            corigin = np.empty((len(gl), 3), dtype=np.int32)
            for b, (gx, gy, gz) in enumerate(gl):
                par = (gx // 2, gy // 2, gz // 2)
                corigin[b] = [PATCH * (gx % 2), PATCH * (gy % 2), PATCH * (gz % 2)]
                for rz in (-1, 0, 1):
                    for ry in (-1, 0, 1):
                        for rx in (-1, 0, 1):
                            q = ((par[0] + rx) % ngp, (par[1] + ry) % ngp, (par[2] + rz) % ngp)
                            cnbr[b, (rx + 1) + 3 * (ry + 1) + 9 * (rz + 1)] = prev.get(q, -1)
            self.cnbr.append(cnbr)
            self.corigin.append(corigin)

    def stand_ins(self, level):
        """The source-only stand-ins for the missing siblings of level
        `level`'s blocks (tvd_fill_coarse_fine, tvd_patch_advance_flux_gather):
        returns (nbr, n_sources) where nbr is the level's sibling table with
        every -1 replaced by an index >= n_blocks, one per missing block
        position (shared by all the blocks around it, numbered in order of
        first use), and n_sources = n_blocks + the number of stand-ins."""
        bs = self.blocks[level]
        n = self.n
        ng = (self.Nc << level) // n
        nbr = bs.nbr.copy()
        pos = self.origins[level] // n          # (z, y, x) block coordinates
        index = {}
        for b in range(bs.n_blocks):
            z, y, x = (int(v) for v in pos[b])
            for r in np.nonzero(nbr[b] < 0)[0]:
                rx, ry, rz = r % 3 - 1, (r // 3) % 3 - 1, r // 9 - 1
                q = ((x + rx) % ng, (y + ry) % ng, (z + rz) % ng)
                if q not in index:
                    index[q] = bs.n_blocks + len(index)
                nbr[b, r] = index[q]
        return nbr, bs.n_blocks + len(index)

    def locate(self, level, px, py, pz):
        if self.n == PATCH:
            return self._index[level][(px, py, pz)], (0, 0, 0)
        return (self._gindex[level][(px // 2, py // 2, pz // 2)],
                (PATCH * (px % 2), PATCH * (py % 2), PATCH * (pz % 2)))

    @staticmethod
    def refined_from_patches(Nc: int, patches):
        """The ``refined`` masks of an octree given as (level, px, py, pz)
        patches over an Nc^3 root grid: a patch is refined when its first
        child is listed."""
        pset = set(tuple(int(v) for v in p) for p in patches)
        top = max(p[0] for p in pset)
        out = []
        for lev in range(top):
            n = (Nc // PATCH) << lev
            r = np.zeros((n, n, n), dtype=bool)
            for (l, px, py, pz) in pset:
                if l == lev and (lev + 1, 2 * px, 2 * py, 2 * pz) in pset:
                    r[pz, py, px] = True
            out.append(r)
        return out

    def tables(self):
        """{level l: (restrict_rows, face_rows, pass_count)} of every pair
        (l, l+1)."""
        return closing_tables(self.patches, self.Nc // PATCH, self.locate)


# ---------------------------------------------------------------------------
# chains of blocks for the streamed advance
# ---------------------------------------------------------------------------

# neighbour region of the block at +1 along x, y, z
PLUS_REGION = {0: 2 + 3 * 1 + 9 * 1, 1: 1 + 3 * 2 + 9 * 1, 2: 1 + 3 * 1 + 9 * 2}
MINUS_REGION = {0: 0 + 3 * 1 + 9 * 1, 1: 1 + 3 * 0 + 9 * 1, 2: 1 + 3 * 1 + 9 * 0}


def stream_chains(nbr: np.ndarray, axis: int, max_len: int, members=None):
    """Cut the lines of blocks along `axis` (0 x, 1 y, 2 z; block b's
    successor is nbr[b][+axis]) into chains of at most `max_len` consecutive
    blocks, as even in length as the line allows.  A line is a cycle on a
    periodic grid (it starts at its lowest block number) or a path from a
    block without a predecessor.  `members`: the blocks to chain (default:
    all); a successor outside them ends a path.  Chains are ordered by their
    first block's number, so consecutive chains lie close together when the
    blocks are numbered along a space-filling curve.  Returns (start, blocks)
    int32 arrays: chain c is blocks[start[c]:start[c+1]]."""
    nbr = np.asarray(nbr)
    nb = nbr.shape[0]
    if max_len < 1:
        raise ValueError("max_len must be >= 1")
    inset = np.zeros(nb, dtype=bool)
    inset[np.arange(nb) if members is None else np.asarray(members, dtype=np.int64)] = True
    succ = nbr[:, PLUS_REGION[axis]].astype(np.int64)
    pred = nbr[:, MINUS_REGION[axis]].astype(np.int64)
    ok_s = (succ >= 0) & (succ < nb)
    ok_p = (pred >= 0) & (pred < nb)
    has_pred = np.zeros(nb, dtype=bool)
    has_pred[ok_p] = inset[pred[ok_p]]
    has_pred &= inset
    seen = ~inset
    lines = []

    def walk(b):
        line = []
        while 0 <= b < nb and not seen[b]:
            seen[b] = True
            line.append(b)
            b = succ[b] if ok_s[b] else -1
        return line

    # paths first (from blocks without a predecessor in the set), then cycles
    for b in np.nonzero(inset & ~has_pred)[0]:
        if not seen[b]:
            lines.append(walk(int(b)))
    for b in np.nonzero(~seen)[0]:
        if not seen[b]:
            line = walk(int(b))
            k = int(np.argmin(line))
            lines.append(line[k:] + line[:k])
    chains = []
    for line in lines:
        n = len(line)
        pieces = -(-n // max_len)
        q, r = divmod(n, pieces)
        o = 0
        for i in range(pieces):
            m = q + (1 if i < r else 0)
            chains.append(line[o:o + m])
            o += m
    chains.sort(key=lambda c: c[0])
    start = np.zeros(len(chains) + 1, dtype=np.int32)
    start[1:] = np.cumsum([len(c) for c in chains])
    blocks = np.array([b for c in chains for b in c], dtype=np.int32)
    return start, blocks
