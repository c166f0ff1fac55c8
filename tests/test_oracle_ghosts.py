"""Pins of the oracle's coarse-fine ghost interpolation (Sec. 2.2: linear
interpolation with the Min-Mod limiter from one level coarser), checked
against closed forms and invariants, not against its own formula:

* a linear field is reproduced exactly (both one-sided differences equal the
  gradient, so the limiter passes it through);
* the eight fine cells of a coarse cell average to the coarse value
  (conservative interpolation);
* no new extrema: every fine value lies within the range of its coarse cell
  and the cell's six face neighbours;
* at an isolated extremum the slopes vanish (the fine cells copy the coarse
  value) and a monotone step gets no overshoot;
* in a two-level region, ghost cells inside the fine box are copies and the
  others interpolations.
Planted mistakes (wrong sign of the offset, a limiter that takes the larger
difference, a one-sided slope) each fail one of these.
"""
import numpy as np
import pytest

from oracle import ghosts


def _children(coarse):
    """All fine cells of a periodic coarse grid, as a fine grid (5, 2Nz, 2Ny, 2Nx)."""
    _, Nz, Ny, Nx = coarse.shape
    fz, fy, fx = np.meshgrid(np.arange(2 * Nz), np.arange(2 * Ny), np.arange(2 * Nx), indexing="ij")
    return ghosts.coarse_to_fine(coarse, fz, fy, fx)


def test_minmod_cases():
    a = np.array([1.0, -1.0, 2.0, -2.0, 1.0, 0.0, 3.0, -0.5])
    b = np.array([2.0, -3.0, 1.0, -1.0, -1.0, 5.0, 3.0, -0.5])
    want = np.array([1.0, -1.0, 1.0, -1.0, 0.0, 0.0, 3.0, -0.5])
    assert np.array_equal(ghosts.minmod(a, b), want)
    assert np.array_equal(ghosts.minmod(b, a), want)


def test_linear_field_is_reproduced():
    N = 8
    c = (np.arange(N) + 0.5) / N
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    coarse = np.stack([1.0 + 0.3 * x - 0.2 * y + 0.1 * z + k for k in range(5)])
    # fine cells whose coarse stencil does not wrap around the periodic box
    f = np.arange(2, 2 * N - 2)
    fz, fy, fx = np.meshgrid(f, f, f, indexing="ij")
    got = ghosts.coarse_to_fine(coarse, fz, fy, fx)
    h = 0.5 / N
    xf, yf, zf = (fx + 0.5) * h, (fy + 0.5) * h, (fz + 0.5) * h
    want = np.stack([1.0 + 0.3 * xf - 0.2 * yf + 0.1 * zf + k for k in range(5)])
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-14)


def test_children_average_to_the_coarse_cell():
    rng = np.random.default_rng(1)
    coarse = rng.lognormal(size=(5, 6, 7, 8))
    fine = _children(coarse)
    avg = fine.reshape(5, 6, 2, 7, 2, 8, 2).mean(axis=(2, 4, 6))
    np.testing.assert_allclose(avg, coarse, rtol=1e-15, atol=0)


def test_no_new_extrema():
    rng = np.random.default_rng(2)
    coarse = rng.standard_normal((5, 6, 6, 6))
    fine = _children(coarse)
    nb = [coarse] + [np.roll(coarse, s, axis=a) for a in (1, 2, 3) for s in (1, -1)]
    lo = np.min(nb, axis=0)
    hi = np.max(nb, axis=0)
    rep = lambda a: a.repeat(2, 1).repeat(2, 2).repeat(2, 3)
    assert np.all(fine >= rep(lo) - 1e-15) and np.all(fine <= rep(hi) + 1e-15)


def test_extremum_is_flat_and_step_has_no_overshoot():
    coarse = np.zeros((5, 6, 6, 6))
    coarse[:, 3, 3, 3] = 1.0
    fine = _children(coarse)
    assert np.all(fine[:, 6:8, 6:8, 6:8] == 1.0)
    step = np.zeros((5, 4, 4, 8))
    step[:, :, :, 4:] = 1.0
    f = _children(step)
    assert f.min() == 0.0 and f.max() == 1.0


def test_two_level_blocks():
    rng = np.random.default_rng(3)
    coarse = rng.lognormal(size=(5, 8, 8, 8))
    box = rng.lognormal(size=(5, 8, 16, 8))
    origin = (4, 0, 6)
    blocks = ghosts.two_level_ghosted_blocks(coarse, box, origin, 8)
    assert blocks.shape == (2, 5, 14, 14, 14)
    # interiors are the box data
    assert np.array_equal(blocks[0][:, 3:11, 3:11, 3:11], box[:, :, 0:8, :])
    assert np.array_equal(blocks[1][:, 3:11, 3:11, 3:11], box[:, :, 8:16, :])
    # the ghost rows between the two blocks are sibling copies
    assert np.array_equal(blocks[0][:, 3:11, 11:14, 3:11], box[:, :, 8:11, :])
    # a ghost cell outside the box is the interpolation at its fine index
    want = ghosts.coarse_to_fine(coarse, np.array([origin[0] - 1]), np.array([origin[1] + 2]),
                                 np.array([origin[2] + 5]))
    assert np.array_equal(blocks[0][:, 2, 5, 8], want[:, 0])


_coarse_to_fine = ghosts.coarse_to_fine


def _mutants():
    def flipped(coarse, fz, fy, fx):
        # offsets on the wrong side along z: the parity flips, the coarse cell does not
        return _coarse_to_fine(coarse, 2 * (fz // 2) + (1 - fz % 2), fy, fx)

    def maxmod(coarse, fz, fy, fx):
        orig = ghosts.minmod
        try:
            ghosts.minmod = lambda a, b: np.where(a * b > 0, np.where(np.abs(a) > np.abs(b), a, b), 0.0)
            return _coarse_to_fine(coarse, fz, fy, fx)
        finally:
            ghosts.minmod = orig

    def one_sided(coarse, fz, fy, fx):
        orig = ghosts.minmod
        try:
            ghosts.minmod = lambda a, b: a
            return _coarse_to_fine(coarse, fz, fy, fx)
        finally:
            ghosts.minmod = orig
    return {"flipped offset": flipped, "larger difference": maxmod, "one-sided slope": one_sided}


@pytest.mark.parametrize("name", list(_mutants()))
def test_planted_mistakes_are_caught(name, monkeypatch):
    bad = _mutants()[name]
    failed = []
    for test in (test_linear_field_is_reproduced, test_no_new_extrema,
                 test_extremum_is_flat_and_step_has_no_overshoot):
        with monkeypatch.context() as m:
            m.setattr(ghosts, "coarse_to_fine", bad)
            try:
                test()
            except AssertionError:
                failed.append(test.__name__)
    assert failed, f"mutant '{name}' passed every pin"
