"""Pins of the oracle's closing step (Sec. 2.1, step 3; Sec. 3.1): restriction
and coarse-fine flux correction, checked against closed forms and the
conservation law they exist for, not against their own formulas:

* restriction keeps a constant and reproduces a linear field at the coarse
  centres; eight times the coarse total is the fine total;
* the leaf cells of a two-level periodic hierarchy (coarse cells of unrefined
  patches, fine cells of refined ones) keep their totals through a step with
  the flux correction, to round-off, and visibly do not without it;
* after restriction the coarse level's total equals the leaf total;
* the correction touches exactly the coarse cells that share a face with a
  refined patch, and a uniform state is left unchanged;
* the masked ghost fill agrees with the box fill of the coarse-fine ghost
  zones where both apply;
* with the fine level sub-cycled (two steps of dt/2) and its flux records
  summed with weight 1/2, the leaf totals are again conserved to round-off;
  so they are on three levels, each sub-cycled in its parent's step, and
  with two levels that step is the two-level one.
Planted mistakes (the correction's sign, the 1/4 of the fine mean, the coarse
flux of the other face, a restriction from one child) each fail one of these.
"""
import math

import numpy as np
import pytest

from oracle import closing, ghosts
from paper_0907_3390_amd import workloads as wl

G53 = 5.0 / 3.0


def _refined_L(P=4):
    """An L of three refined patches in the plane pz = 1: the unrefined patch
    (1, 2, 2) touches refined patches across its -x and -y faces, so its
    corner cells take two corrections."""
    r = np.zeros((P, P, P), dtype=bool)
    r[1, 1, 1] = r[1, 1, 2] = r[1, 2, 1] = True
    return r


def _two_level_state(N, seed):
    coarse = wl.lognormal(N, seed=seed, sigma_ln=0.5)
    fine = ghosts.coarse_to_fine(coarse, *np.meshgrid(np.arange(2 * N), np.arange(2 * N),
                                                       np.arange(2 * N), indexing="ij"))
    # a fine level with its own structure on top of the interpolated coarse one
    fine = fine * (1.0 + 0.05 * wl.smooth_random(2 * N, seed=seed + 1, amplitude=1.0)[0:1] /
                   wl.smooth_random(2 * N, seed=seed + 1, amplitude=1.0)[0:1].max())
    return coarse, fine


def test_restrict_closed_forms():
    N = 8
    c = (np.arange(2 * N) + 0.5) / (2 * N)
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    lin = np.stack([1.0 + 0.3 * x - 0.2 * y + 0.1 * z + k for k in range(5)])
    cc = (np.arange(N) + 0.5) / N
    zc, yc, xc = np.meshgrid(cc, cc, cc, indexing="ij")
    want = np.stack([1.0 + 0.3 * xc - 0.2 * yc + 0.1 * zc + k for k in range(5)])
    np.testing.assert_allclose(closing.restrict(lin), want, rtol=0, atol=1e-15)
    const = np.full((5, 4, 6, 8), 2.5)
    assert np.array_equal(closing.restrict(const), np.full((5, 2, 3, 4), 2.5))
    r = wl.rng(7)
    f = r.lognormal(size=(5, 8, 8, 8))
    co = closing.restrict(f)
    for k in range(5):
        assert math.fsum((8 * co[k]).ravel()) == pytest.approx(math.fsum(f[k].ravel()), rel=1e-15)
    # dyadic data: the mean is exact
    fi = r.integers(-1000, 1000, size=(5, 4, 4, 4)).astype(np.float64)
    assert np.array_equal(closing.restrict(fi) * 8, fi.reshape(5, 2, 2, 2, 2, 2, 2).sum(axis=(2, 4, 6)))
    # FP32 stays FP32
    assert closing.restrict(f.astype(np.float32)).dtype == np.float32


def test_masked_ghosts_match_box_ghosts():
    N = 16
    coarse = wl.lognormal(N, seed=3, sigma_ln=0.5)
    r = np.zeros((2, 2, 2), dtype=bool)
    r[0, 1, 0] = True
    fine = wl.smooth_random(2 * N, seed=4, amplitude=0.3)
    # the box of that refined patch: fine cells z 0..15, y 16..31, x 0..15
    box = fine[:, 0:16, 16:32, 0:16]
    for n_f in (8, 16):
        a = closing.ghosted_fine_blocks(coarse, fine, r, n_f)
        b = ghosts.two_level_ghosted_blocks(coarse, box, (0, 16, 0), n_f)
        assert np.array_equal(a, b)


@pytest.mark.parametrize("n_f", [8, 16])
@pytest.mark.parametrize("order", [0, 1])
def test_two_level_step_conserves_leaf_totals(n_f, order):
    N = 32
    coarse, fine = _two_level_state(N, seed=30 + n_f + order)
    refined = _refined_L()
    dt = 0.25 / N
    before = closing.leaf_sums(coarse, fine, refined)
    scale = closing.leaf_sums(np.abs(coarse), np.abs(fine), refined)
    c1, f1 = closing.two_level_step(coarse, fine, refined, n_f, dt, order, G53)
    after = closing.leaf_sums(c1, f1, refined)
    assert np.all(np.abs(after - before) <= 1e-13 * scale), (after - before) / scale
    # without the correction the coarse-fine faces leak
    c0, f0 = closing.two_level_step(coarse, fine, refined, n_f, dt, order, G53, correct=False)
    leak = np.abs(closing.leaf_sums(c0, f0, refined) - before) / scale
    assert leak[0] > 1e-9 and leak[4] > 1e-9, leak
    # restriction: the coarse total is the leaf total
    for k in range(5):
        tot = math.fsum(c1[k].ravel())
        assert abs(tot - after[k]) <= 1e-13 * scale[k]


@pytest.mark.parametrize("n_f", [8, 16])
def test_subcycled_step_conserves_leaf_totals(n_f):
    """With the fine level sub-cycled (two steps of dt/2, ghosts from the
    coarse level at the old time and half-way), the time-weighted fine flux
    records make the correction exactly conservative again; without it the
    coarse-fine faces leak.  The result differs from the one-dt step."""
    N = 32
    coarse, fine = _two_level_state(N, seed=60 + n_f)
    refined = _refined_L()
    dt = 0.25 / N
    before = closing.leaf_sums(coarse, fine, refined)
    scale = closing.leaf_sums(np.abs(coarse), np.abs(fine), refined)
    c1, f1 = closing.two_level_step_subcycled(coarse, fine, refined, n_f, dt, 0, G53)
    after = closing.leaf_sums(c1, f1, refined)
    assert np.all(np.abs(after - before) <= 1e-13 * scale), (after - before) / scale
    c0, f0 = closing.two_level_step_subcycled(coarse, fine, refined, n_f, dt, 0, G53, correct=False)
    leak = np.abs(closing.leaf_sums(c0, f0, refined) - before) / scale
    assert leak[0] > 1e-9 and leak[4] > 1e-9, leak
    cu, fu = closing.two_level_step(coarse, fine, refined, n_f, dt, 0, G53)
    assert not np.allclose(fu, f1, rtol=1e-9, atol=0)


def test_lerp():
    a = np.array([1.0, 2.0, -3.0])
    b = np.array([3.0, 2.0, 5.0])
    assert np.array_equal(closing.lerp(a, b, 0.5), [2.0, 2.0, 1.0])
    assert np.array_equal(closing.lerp(a, b, 0.0), a) and np.array_equal(closing.lerp(a, b, 1.0), b)
    assert closing.lerp(a.astype(np.float32), b.astype(np.float32), 0.5).dtype == np.float32


def test_correction_touches_only_interface_cells():
    N = 32
    coarse, fine = _two_level_state(N, seed=40)
    refined = _refined_L()
    dt = 0.25 / N
    c1, _ = closing.two_level_step(coarse, fine, refined, 8, dt, 0, G53)
    c0, _ = closing.two_level_step(coarse, fine, refined, 8, dt, 0, G53, correct=False)
    changed = np.any(c1 != c0, axis=0)
    want = np.zeros((N, N, N), dtype=bool)
    # unrefined cells sharing a face with a refined patch's cell
    ref_cells = np.repeat(np.repeat(np.repeat(refined, 8, 0), 8, 1), 8, 2)
    for ax in (0, 1, 2):
        for sh in (1, -1):
            want |= np.roll(ref_cells, sh, axis=ax)
    want &= ~ref_cells
    assert np.array_equal(changed, want)
    # the corner cells of patch (1, 2, 2) next to both -x and -y neighbours
    assert changed[8:16, 16, 16].all()


def test_uniform_state_is_unchanged():
    N = 32
    u = wl.uniform(N, rho=1.2, v=(0.3, -0.1, 0.2), P=0.9, gamma=G53)
    uf = wl.uniform(2 * N, rho=1.2, v=(0.3, -0.1, 0.2), P=0.9, gamma=G53)
    c1, f1 = closing.two_level_step(u, uf, _refined_L(), 16, 0.25 / N, 1, G53)
    np.testing.assert_allclose(c1, u, rtol=1e-15, atol=0)
    np.testing.assert_allclose(f1, uf, rtol=1e-15, atol=0)


_flux_correct = closing.flux_correct
_restrict = closing.restrict


def _mutants():
    def sign_flipped(coarse, refined, recs, faces, lam):
        return _flux_correct(coarse, refined, recs, faces, -lam)

    def sum_not_mean(coarse, refined, recs, faces, lam):
        return _flux_correct(coarse, refined, recs, [4 * f for f in faces], lam)

    def other_face(coarse, refined, recs, faces, lam):
        return _flux_correct(coarse, refined, recs[:, :, :, :, ::-1], faces, lam)

    def one_child(fine):
        f = np.asarray(fine)
        return f[:, 0::2, 0::2, 0::2].copy()
    return {"correction sign flipped": ("flux_correct", sign_flipped),
            "fine fluxes summed, not averaged": ("flux_correct", sum_not_mean),
            "coarse flux of the opposite face": ("flux_correct", other_face),
            "restriction from one child": ("restrict", one_child)}


@pytest.mark.parametrize("name", list(_mutants()))
def test_planted_mistakes_are_caught(name, monkeypatch):
    attr, bad = _mutants()[name]
    failed = []
    for test, kw in ((test_two_level_step_conserves_leaf_totals, dict(n_f=8, order=0)),
                     (test_restrict_closed_forms, {}), (test_uniform_state_is_unchanged, {})):
        with monkeypatch.context() as m:
            m.setattr(closing, attr, bad)
            try:
                test(**kw)
            except AssertionError:
                failed.append(test.__name__)
    assert failed, f"mutant '{name}' passed every pin"


def _three_levels():
    """Level 0: 32^3; a 2^3 cube of refined root patches; on level 1 an L of
    three refined patches inside it (their 26 neighbours exist: proper
    nesting)."""
    r0 = np.zeros((4, 4, 4), dtype=bool)
    r0[1:3, 1:3, 1:3] = True
    r1 = np.zeros((8, 8, 8), dtype=bool)
    r1[3, 3, 3] = r1[3, 3, 4] = r1[3, 4, 3] = True
    return [r0, r1]


def _three_level_states(seed):
    N = 32
    s0 = wl.lognormal(N, seed=seed, sigma_ln=0.5)
    out = [s0]
    for lev in (1, 2):
        M = N << lev
        g = np.meshgrid(np.arange(M), np.arange(M), np.arange(M), indexing="ij")
        f = ghosts.coarse_to_fine(out[-1], *g)
        bump = wl.smooth_random(M, seed=seed + lev, amplitude=1.0)[0:1]
        out.append(f * (1.0 + 0.05 * bump / np.abs(bump).max()))
    return out


@pytest.mark.parametrize("order", [0, 1])
def test_nested_subcycled_step_conserves_leaf_totals(order):
    """Three levels, each sub-cycled in its parent's step (four level-2 steps
    per root step): with the time-averaged records of every finer level the
    leaf totals are conserved to round-off, and visibly not without the
    correction; after the closing chain the root total is the leaf total."""
    refined = _three_levels()
    states = _three_level_states(80 + order)
    dt = 0.25 / 32
    before = closing.nested_leaf_sums(states, refined)
    scale = closing.nested_leaf_sums([np.abs(s) for s in states], refined)
    new = closing.nested_step_subcycled(states, refined, dt, order, G53)
    after = closing.nested_leaf_sums(new, refined)
    assert np.all(np.abs(after - before) <= 1e-13 * scale), (after - before) / scale
    for k in range(5):
        assert abs(math.fsum(new[0][k].ravel()) - after[k]) <= 1e-13 * scale[k]
    leaky = closing.nested_step_subcycled(states, refined, dt, order, G53, correct=False)
    leak = np.abs(closing.nested_leaf_sums(leaky, refined) - before) / scale
    assert leak[0] > 1e-9 and leak[4] > 1e-9, leak


def test_nested_two_levels_is_the_two_level_step():
    """With two levels the nested step is the two-level sub-cycled step (the
    fine records averaged as a lerp instead of 1/2 H1 + 1/2 H2: equal to
    round-off)."""
    coarse, fine = _two_level_state(32, seed=90)
    refined = _refined_L()
    dt = 0.25 / 32
    c1, f1 = closing.two_level_step_subcycled(coarse, fine, refined, 8, dt, 1, G53)
    c2, f2 = closing.nested_step_subcycled([coarse, fine], [refined], dt, 1, G53)
    np.testing.assert_allclose(c2, c1, rtol=1e-14, atol=0)
    m = np.repeat(np.repeat(np.repeat(refined, 16, 0), 16, 1), 16, 2)
    np.testing.assert_allclose(f2[:, m], f1[:, m], rtol=1e-14, atol=0)


def test_nested_uniform_state_is_unchanged():
    refined = _three_levels()
    states = [wl.uniform(32 << l, rho=1.2, v=(0.3, -0.1, 0.2), P=0.9, gamma=G53) for l in range(3)]
    new = closing.nested_step_subcycled(states, refined, 0.25 / 32, 0, G53)
    for a, b in zip(new, states):
        np.testing.assert_allclose(a, b, rtol=1e-15, atol=0)


def test_nested_planted_mistake_is_caught(monkeypatch):
    """The sub-steps' records summed instead of averaged."""
    orig = closing._subcycle

    def summed(states, refined, lev, *a):
        return [2 * r for r in orig(states, refined, lev, *a)]
    monkeypatch.setattr(closing, "_subcycle", summed)
    with pytest.raises(AssertionError):
        test_nested_subcycled_step_conserves_leaf_totals(0)
