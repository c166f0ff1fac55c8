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
