"""Input generators: the multi-level hierarchy as 8^3 patches and as 2^3
patch groups describes the same cells, and the oracle advances both to the
same values (decomposition invariance across the two block sizes)."""
import numpy as np

import oracle
from paper_0907_3390_amd import workloads as wl

GAMMA = 5.0 / 3.0


def _ml():
    return wl.multilevel(base=32, n_over=4, seed=5, radius=0.07)


def test_group_blocks_contain_the_patch_blocks():
    ml = _ml()
    groups, G, gdh = ml.group_blocks()
    assert len(groups) * 8 == len(ml.patches)
    pidx = {p: i for i, p in enumerate(ml.patches)}
    for gi, (lev, gx, gy, gz) in enumerate(groups):
        assert gdh[gi] == 1.0 / (32 * 2 ** lev)
        for c in range(8):
            cx, cy, cz = c & 1, c >> 1 & 1, c >> 2
            P = ml.ghosted[pidx[(lev, 2 * gx + cx, 2 * gy + cy, 2 * gz + cz)]]
            # the patch's whole ghosted block is a window of the group's
            assert np.array_equal(P, G[gi][:, 8 * cz:8 * cz + 14, 8 * cy:8 * cy + 14,
                                           8 * cx:8 * cx + 14])


def test_oracle_patches_and_groups_agree():
    ml = _ml()
    groups, G, gdh = ml.group_blocks()
    dt = 0.5 * ml.dh / 40.0
    gdt = 0.5 * gdh / 40.0
    outp = oracle.advance_ragged(list(ml.ghosted), 0, dt, ml.dh, GAMMA)
    outg = oracle.advance_ragged(list(G), 0, gdt, gdh, GAMMA)
    pidx = {p: i for i, p in enumerate(ml.patches)}
    for gi, (lev, gx, gy, gz) in enumerate(groups):
        for c in range(8):
            cx, cy, cz = c & 1, c >> 1 & 1, c >> 2
            p = outp[pidx[(lev, 2 * gx + cx, 2 * gy + cy, 2 * gz + cz)]]
            assert np.array_equal(p, outg[gi][:, 8 * cz:8 * cz + 8, 8 * cy:8 * cy + 8,
                                              8 * cx:8 * cx + 8])


def test_hierarchy_is_properly_nested():
    """Sec. 2.1: refinement never jumps more than one level across adjacent
    patches, so every face of a level-l patch (l >= 1) without a same-level
    neighbour borders a level-(l-1) patch."""
    ml = _ml()
    assert set(np.unique(ml.levels)) == {0, 1, 2, 3}
    present = set(ml.patches)
    nb = ml.base // 8
    for lev, px, py, pz in ml.patches:
        for rz in (-1, 0, 1):
            for ry in (-1, 0, 1):
                for rx in (-1, 0, 1):
                    n_l = nb << lev
                    q = ((px + rx) % n_l, (py + ry) % n_l, (pz + rz) % n_l)
                    if (lev, *q) not in present:
                        assert lev > 0 and (lev - 1, q[0] // 2, q[1] // 2, q[2] // 2) in present


def test_closing_tables_cover_every_coarse_fine_face():
    """The face rows of all level pairs cover each coarse-fine interface cell
    face once, in patch and in patch-group blocks, and the restriction rows
    cover each refined patch once."""
    ml = _ml()
    nb = ml.base // 8
    present = set(ml.patches)
    want = 0
    for lev, px, py, pz in ml.patches:
        if (lev + 1, 2 * px, 2 * py, 2 * pz) in present:
            continue
        for d in range(3):
            for s in (-1, 1):
                q = [px, py, pz]
                q[d] = (q[d] + s) % (nb << lev)
                if (lev, *q) in present and (lev + 1, 2 * q[0], 2 * q[1], 2 * q[2]) in present:
                    want += 64     # an 8 x 8 coarse face
    n_refined = sum(1 for p in ml.patches if (p[0] + 1, 2 * p[1], 2 * p[2], 2 * p[3]) in present)
    for edge in (8, 16):
        tabs = ml.closing(edge)
        got = sum(int(((fr[:, 6] >= 0).sum())) * (edge // 2) ** 2 for _, fr, _ in tabs.values())
        assert got == want
        cells = sum(len(rr) * (edge // 2) ** 3 for rr, _, _ in tabs.values())
        assert cells == n_refined * 512
