"""Input generators: the multi-level hierarchy as 8^3 patches and as 2^3
patch groups describes the same cells, and the oracle advances both to the
same values (decomposition invariance across the two block sizes)."""
import numpy as np

import oracle
from paper_0907_3390_amd import workloads as wl

GAMMA = 5.0 / 3.0


def _ml():
    return wl.multilevel(base=32, n_over=4, seed=3, radius=0.05)


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
