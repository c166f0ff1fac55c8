"""Host bookkeeping: block numbering, neighbour tables, block <-> grid maps.

Integer work only, checked exactly: the Morton numbering is a permutation
whose neighbour table names, for every block and region, the block that
covers that region of the periodic grid; block and grid views round-trip.
"""
import numpy as np
import pytest

from paper_0907_3390_amd import layout


def _coords(lin, nbx, nby):
    return lin % nbx, (lin // nbx) % nby, lin // (nbx * nby)


def test_morton_perm_is_a_z_curve():
    perm = layout.morton_perm(4, 4, 4)
    assert sorted(perm.tolist()) == list(range(64))
    # the first eight blocks are the 2^3 brick at the origin, x bit lowest
    x, y, z = _coords(perm[:8], 4, 4)
    assert x.tolist() == [0, 1, 0, 1, 0, 1, 0, 1]
    assert y.tolist() == [0, 0, 1, 1, 0, 0, 1, 1]
    assert z.tolist() == [0, 0, 0, 0, 1, 1, 1, 1]
    # every aligned run of 8 is a 2^3 brick
    for k in range(0, 64, 8):
        x, y, z = _coords(perm[k:k + 8], 4, 4)
        assert np.ptp(x) == 1 and np.ptp(y) == 1 and np.ptp(z) == 1


@pytest.mark.parametrize("shape", [(4, 4, 4), (2, 4, 8), (3, 5, 2)])
def test_morton_neighbour_table(shape):
    nbx, nby, nbz = shape
    n = 8
    bs = layout.periodic_grid_blockset((nbz * n, nby * n, nbx * n), n, curve="morton")
    perm = bs.perm
    for k in range(bs.n_blocks):
        bx, by, bz = _coords(perm[k], nbx, nby)
        for rz in (-1, 0, 1):
            for ry in (-1, 0, 1):
                for rx in (-1, 0, 1):
                    r = (rx + 1) + 3 * (ry + 1) + 9 * (rz + 1)
                    want = ((bx + rx) % nbx) + nbx * (((by + ry) % nby) + nby * ((bz + rz) % nbz))
                    assert perm[bs.nbr[k, r]] == want


def test_grid_blocks_round_trip_with_perm():
    rng = np.random.default_rng(0)
    g = rng.standard_normal((5, 16, 32, 24))
    bs = layout.periodic_grid_blockset((16, 32, 24), 8, curve="morton")
    blocks = layout.grid_to_blocks(g, 8, bs.perm)
    lin = layout.grid_to_blocks(g, 8)
    assert np.array_equal(blocks, lin[bs.perm])
    assert np.array_equal(layout.blocks_to_grid(blocks, g.shape, bs.perm), g)
    # block k's interior is the grid's cells of linear block perm[k]
    k = 5
    bx, by, bz = _coords(bs.perm[k], 3, 4)
    assert np.array_equal(blocks[k], g[:, 8 * bz:8 * bz + 8, 8 * by:8 * by + 8, 8 * bx:8 * bx + 8])


def test_two_level_tables():
    coarse, fine, cnbr, corigin = layout.two_level(16, (8, 0, 16), (8, 16, 8), 8)
    assert coarse.n_blocks == 8 and fine.n_blocks == 2
    # block 1 sits above block 0 in y; outside the box there are no siblings
    assert fine.nbr[0, 13] == 0 and fine.nbr[0, 1 + 3 * 2 + 9] == 1 and fine.nbr[0, 1 + 9] == -1
    assert (fine.nbr[0] >= 0).sum() == 2
    # fine block 0 corner at fine (x, y, z) = (16, 0, 8) -> coarse (8, 0, 4): parent patch (1, 0, 0)
    assert corigin[0].tolist() == [0, 0, 4] and corigin[1].tolist() == [0, 4, 4]
    assert cnbr[0, 13] == 1 and cnbr[0, 12] == 0 and cnbr[0, 14] == 0   # periodic, 2 patches per axis
    with pytest.raises(ValueError):
        layout.two_level(16, (4, 0, 0), (8, 8, 8), 8)


def _L_refined():
    r = np.zeros((4, 4, 4), dtype=bool)
    r[1, 1, 1] = r[1, 1, 2] = r[1, 2, 1] = True
    r[3, 0, 3] = True          # a refined patch at the periodic corner
    return r


@pytest.mark.parametrize("n", [8, 16])
def test_refined_levels_tables_match_geometry(n):
    """Every restriction row and face row names cells that coincide in space,
    and the face rows cover each coarse-fine interface cell face exactly once
    (checked against a brute-force scan of the refinement mask)."""
    Nc = 32
    ref = _L_refined()
    L = layout.RefinedLevels(Nc, ref, n)
    rr, fr, count = L.tables()
    corner = lambda c: np.array([8 * (c % 4), 8 * ((c // 4) % 4), 8 * (c // 16)])  # x, y, z
    fo = L.origins[:, ::-1]                                                       # x, y, z
    # restriction: fine block f is the coarse region at (c, offset)
    assert sorted(rr[:, 0].tolist()) == list(range(L.fine.n_blocks))
    for f, c, ox, oy, oz in rr:
        assert np.array_equal(fo[f] // 2, corner(c) + [ox, oy, oz])
        assert ref[(fo[f][2] // 16), (fo[f][1] // 16), (fo[f][0] // 16)]
    # faces
    assert count.sum() == len(fr) and np.all(np.diff(2 * fr[:, 1] + fr[:, 2]) >= 0)
    covered = set()
    for c, d, s, qc, oa, ob, f, qf in fr:
        hi, lo = {0: (2, 1), 1: (2, 0), 2: (1, 0)}[d]
        plane_c = corner(c)[d] + 8 * qc
        plane_f = fo[f][d] + 8 * qf
        assert (2 * plane_c - plane_f) % (2 * Nc) == 0
        assert (2 * (corner(c)[hi] + oa) - fo[f][hi]) % (2 * Nc) == 0
        assert (2 * (corner(c)[lo] + ob) - fo[f][lo]) % (2 * Nc) == 0
        for a in range(n // 2):
            for b in range(n // 2):
                cell = [0, 0, 0]
                cell[d] = (plane_c - 1 if s else plane_c) % Nc
                cell[hi], cell[lo] = corner(c)[hi] + oa + a, corner(c)[lo] + ob + b
                key = (tuple(cell), d, s)
                assert key not in covered
                covered.add(key)
    want = set()
    rc = np.repeat(np.repeat(np.repeat(ref, 8, 0), 8, 1), 8, 2)     # [z, y, x]
    for z, y, x in np.argwhere(~rc):
        for d in range(3):
            for s in (0, 1):
                q = [x, y, z]
                q[d] = (q[d] + (1 if s else -1)) % Nc
                if rc[q[2], q[1], q[0]]:
                    want.add(((x, y, z), d, s))
    assert covered == want


def test_refined_levels_sibling_table():
    ref = _L_refined()
    L = layout.RefinedLevels(32, ref, 8)
    fo = L.origins
    pos = {tuple(o): b for b, o in enumerate(fo.tolist())}
    for b in range(L.fine.n_blocks):
        for r in range(27):
            rx, ry, rz = r % 3 - 1, (r // 3) % 3 - 1, r // 9 - 1
            o = ((fo[b][0] + 8 * rz) % 64, (fo[b][1] + 8 * ry) % 64, (fo[b][2] + 8 * rx) % 64)
            assert L.fine.nbr[b, r] == pos.get(o, -1)


def test_group_face_rows():
    ref = _L_refined()
    L = layout.RefinedLevels(32, ref, 8)
    _, fr, _ = L.tables()
    rows, start = layout.group_face_rows(fr)
    assert sorted(map(tuple, rows.tolist())) == sorted(map(tuple, fr.tolist()))
    assert start[0] == 0 and start[-1] == len(rows) and np.all(np.diff(start) > 0)
    seen = set()
    for g in range(len(start) - 1):
        grp = rows[start[g]:start[g + 1]]
        assert np.all(grp[:, 0] == grp[0, 0]) and grp[0, 0] not in seen
        seen.add(grp[0, 0])
        assert np.all(np.diff(2 * grp[:, 1] + grp[:, 2]) >= 0)
    r0, s0 = layout.group_face_rows(np.zeros((0, 8), np.int32))
    assert len(r0) == 0 and s0.tolist() == [0]


def test_nested_levels_tables():
    """A three-level hierarchy: block counts, sibling tables (-1 where no
    patch exists), the coarse patches around every parent, and the closing
    rows of both level pairs; a refinement that breaks proper nesting is
    rejected."""
    r0 = np.zeros((4, 4, 4), dtype=bool)
    r0[1:3, 1:3, 1:3] = True
    r1 = np.zeros((8, 8, 8), dtype=bool)
    r1[3, 3, 3] = r1[3, 3, 4] = r1[3, 4, 3] = True
    L = layout.NestedLevels(32, [r0, r1])
    assert [b.n_blocks for b in L.blocks] == [64, 64, 24]
    assert (L.blocks[0].nbr >= 0).all()
    # level 1 is a 4^3 cube of patches: a corner patch has 7 of its 27
    # regions (itself included) on the level
    assert sorted(set((L.blocks[1].nbr >= 0).sum(1))) == [8, 12, 18, 27]
    for lev in (1, 2):
        o = L.origins[lev] // 8
        par = {tuple(v) for v in (L.origins[lev - 1] // 8)}
        for b in range(L.blocks[lev].n_blocks):
            z, y, x = o[b]
            assert L.corigin[lev][b].tolist() == [4 * (x % 2), 4 * (y % 2), 4 * (z % 2)]
            pz, py, px = L.origins[lev - 1][L.cnbr[lev][b, 13]] // 8
            assert (pz, py, px) == (z // 2, y // 2, x // 2) and (pz, py, px) in par
    t = L.tables()
    assert sorted(t) == [0, 1]
    assert t[0][0].shape[0] == 64 and t[1][0].shape[0] == 24
    # faces: the 2^3 cube shows 24 coarse faces, each covered by 4 fine patches
    assert t[0][1].shape[0] == 96 and int(sum(t[0][2])) == 96
    # the L of three patches shows 14 faces
    assert t[1][1].shape[0] == 4 * 14
    bad = r1.copy()
    bad[2, 3, 3] = True
    with pytest.raises(ValueError, match="proper nesting"):
        layout.NestedLevels(32, [r0, bad])
    with pytest.raises(ValueError, match="does not exist"):
        r2 = np.zeros((16, 16, 16), dtype=bool)
        r2[0, 0, 0] = True
        layout.NestedLevels(32, [r0, r1, r2])


def test_nested_levels_masks_round_trip():
    r0 = np.zeros((4, 4, 4), dtype=bool)
    r0[1:3, 1:3, 1:3] = True
    r1 = np.zeros((8, 8, 8), dtype=bool)
    r1[3, 3, 3] = r1[3, 4, 4] = True
    L = layout.NestedLevels(32, [r0, r1])
    back = layout.NestedLevels.refined_from_patches(32, L.patches)
    assert len(back) == 2 and all(np.array_equal(a, b) for a, b in zip(back, [r0, r1]))


def test_stream_chains_cover_and_follow_the_axis():
    """Chains for the streamed advance: every block exactly once, each block
    the +axis neighbour of the one before, lengths as even as the line
    allows (at most max_len), on periodic grids numbered linearly and along
    the Morton curve, and on independent periodic boxes (lines that are
    cycles of one block)."""
    from paper_0907_3390_amd.driver import default_chain_len
    cases = [layout.periodic_grid_blockset(96, 16), layout.periodic_grid_blockset(64, 16, curve="morton"),
             layout.boxes_blockset([32, 32, 16], lambda L: L, [1 / 32, 1 / 32, 1 / 16])]
    for bs in cases:
        for axis in (0, 1, 2):
            for L in (1, 2, 3, 4, 64):
                st, bl = layout.stream_chains(bs.nbr, axis, L)
                assert st[0] == 0 and st[-1] == bs.n_blocks
                assert sorted(bl.tolist()) == list(range(bs.n_blocks))
                lens = np.diff(st)
                assert lens.min() >= 1 and lens.max() <= L
                for c in range(len(lens)):
                    ch = bl[st[c]:st[c + 1]]
                    for a, b in zip(ch[:-1], ch[1:]):
                        assert bs.nbr[a, layout.PLUS_REGION[axis]] == b
    # a periodic line of 6 blocks cut at most 4 long: two chains of 3
    bs = layout.periodic_grid_blockset((16, 16, 96), 16)
    st, bl = layout.stream_chains(bs.nbr, 0, 4)
    assert np.diff(st).tolist() == [3, 3]
    # a subset: the successor outside the set ends a path
    st, bl = layout.stream_chains(bs.nbr, 0, 8, members=[1, 2, 3])
    assert bl.tolist() == [1, 2, 3] and st.tolist() == [0, 3]
    assert default_chain_len(32768) == 32 and default_chain_len(4096) == 4
    assert default_chain_len(10 ** 7) == 64


def test_nested_levels_as_patch_groups():
    """NestedLevels with n = 16: every patch of every level lies in one
    group at its octant (the group's origin plus the offset is the patch's
    origin in the patch view); siblings are groups at +-1; every coarse
    group that a group's coarse-fine ghost zone or stencil can reach (the
    level-(l-1) groups holding the parent patch's 26 neighbours) is named
    in cnbr; the closing tables restrict each group once into the group
    holding its parent at that patch's octant, and the face rows cover the
    same coarse faces as the patch view (same coarse cells, 8x8 instead of
    4x4 pieces)."""
    r0 = np.zeros((4, 4, 4), dtype=bool)
    r0[1:3, 1:3, 1:3] = True
    r1 = np.zeros((8, 8, 8), dtype=bool)
    r1[3, 3, 3] = r1[3, 3, 4] = r1[3, 4, 3] = True
    P = layout.NestedLevels(32, [r0, r1])
    G = layout.NestedLevels(32, [r0, r1], 16)
    assert [b.n_blocks for b in G.blocks] == [8, 8, 3]
    assert all(np.all(b.edges == 16) for b in G.blocks)
    for (l, px, py, pz) in P.patches:
        pb, _ = P.locate(l, px, py, pz)
        gb, (ox, oy, oz) = G.locate(l, px, py, pz)
        assert tuple(P.origins[l][pb]) == (G.origins[l][gb][0] + oz, G.origins[l][gb][1] + oy,
                                            G.origins[l][gb][2] + ox)
    for l in (1, 2):
        for b in range(G.blocks[l].n_blocks):
            gz, gy, gx = (G.origins[l][b] // 16).tolist()
            # the parent patch (gx, gy, gz) of level l-1 and its 26 neighbours
            # are all in groups named by cnbr, at the offsets corigin implies
            cx, cy, cz = G.corigin[l][b]
            assert (cx, cy, cz) == (8 * (gx % 2), 8 * (gy % 2), 8 * (gz % 2))
            n_p = (32 << (l - 1)) // 8
            for rz in (-1, 0, 1):
                for ry in (-1, 0, 1):
                    for rx in (-1, 0, 1):
                        q = ((gx + rx) % n_p, (gy + ry) % n_p, (gz + rz) % n_p)
                        cb, off = G.locate(l - 1, *q)
                        # the region of that patch's group around the central group
                        rel = [c // 2 - g // 2 for c, g in zip((gx + rx, gy + ry, gz + rz), (gx, gy, gz))]
                        reg = (rel[0] + 1) + 3 * (rel[1] + 1) + 9 * (rel[2] + 1)
                        assert G.cnbr[l][b][reg] == cb
    tp, tg = P.tables(), G.tables()
    for lev in tp:
        rr, fr, _ = tg[lev]
        assert len(rr) == G.blocks[lev + 1].n_blocks
        assert len(np.unique(rr[:, 0])) == len(rr)
        # normalise to absolute coarse face cells (axis, side, plane coordinate, two face coords)
        def absolute(L, rows, e_f):
            h = e_f // 2
            res = set()
            hi_lo = {0: (2, 1), 1: (2, 0), 2: (1, 0)}
            for c, d, s, qc, oa, ob, f, qf in rows:
                z, y, x = L.origins[lev][c]
                org = {0: x, 1: y, 2: z}
                hi, lo = hi_lo[int(d)]
                for a in range(oa, oa + h):
                    for b2 in range(ob, ob + h):
                        res.add((int(d), int(s), org[int(d)] + 8 * int(qc), org[hi] + a, org[lo] + b2))
            return res
        assert absolute(P, tp[lev][1], 8) == absolute(G, fr, 16)


def test_two_level_morton_numbering():
    """Morton numbering of the fine box renumbers the blocks only: the sibling
    table, the coarse tables and the cut interiors are the linear ones
    permuted, and the blocks are those of the box in that order."""
    import numpy as np
    from paper_0907_3390_amd import layout
    for n in (8, 16):
        _, f1, cn1, co1 = layout.two_level(64, (32, 32, 32), (64, 64, 64), n)
        _, f2, cn2, co2 = layout.two_level(64, (32, 32, 32), (64, 64, 64), n, curve="morton")
        p = f2.perm
        inv = np.empty_like(p)
        inv[p] = np.arange(len(p))
        want = np.where(f1.nbr[p] >= 0, inv[np.maximum(f1.nbr[p], 0)], -1)
        assert np.array_equal(f2.nbr, want)
        assert np.array_equal(cn2, cn1[p]) and np.array_equal(co2, co1[p])
        assert sorted(p.tolist()) == list(range(f1.n_blocks))
        g = np.arange(5 * 64 ** 3, dtype=np.float64).reshape(5, 64, 64, 64)
        assert np.array_equal(layout.grid_to_blocks(g, n, p), layout.grid_to_blocks(g, n)[p])
        # consecutive Morton blocks are face neighbours more often than not
        adj = sum(int(k + 1 in f2.nbr[k]) for k in range(f2.n_blocks - 1))
        assert adj > 0.5 * (f2.n_blocks - 1)
