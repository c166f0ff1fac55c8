"""Pins of the oracle's self-gravity operator (Sec. 2.3; Eqs. MomConserve
and EnergyConserve without their flux terms) against closed forms:

* a linear potential is a uniform field, and a quadratic one a linear field,
  both differenced exactly by 3-point central differences: the momentum
  gains dt rho g with g = -grad phi at the cell centres;
* the density never changes, and the internal energy e - |m|^2/(2 rho) is
  unchanged to round-off (the energy gains exactly the kinetic energy the
  momentum update adds);
* a potential constant along an axis leaves that momentum unchanged.
Planted mistakes (a one-sided difference, the wrong sign, the energy from the
old momentum only) each fail one of these.
"""
import numpy as np
import pytest

from oracle import gravity
from paper_0907_3390_amd import workloads as wl

N = 8


def _state(seed):
    g = wl.lognormal(N, seed=seed, sigma_ln=0.5)
    return g[None]


def _phi(fn, n=N, h=1.0 / N):
    c = (np.arange(-1, n + 1) + 0.5) * h
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    return fn(x, y, z)[None], (x[1:-1, 1:-1, 1:-1], y[1:-1, 1:-1, 1:-1], z[1:-1, 1:-1, 1:-1])


def test_uniform_and_linear_fields():
    u = _state(1)
    dt, h = 0.01, 1.0 / N
    for fn, grad in ((lambda x, y, z: 2.0 * x - 3.0 * y + 0.5 * z, lambda x, y, z: (2.0, -3.0, 0.5)),
                     (lambda x, y, z: x * x + 2 * y * y - z * z + x * y,
                      lambda x, y, z: (2 * x + y, 4 * y + x, -2 * z))):
        phi, (x, y, z) = _phi(fn)
        out = gravity.apply(u, phi, dt, h)
        gx, gy, gz = grad(x, y, z)
        for d, gd in enumerate((gx, gy, gz)):
            want = u[0, 1 + d] - dt * u[0, 0] * np.asarray(gd)
            np.testing.assert_allclose(out[0, 1 + d], want, rtol=1e-12, atol=1e-13)
        assert np.array_equal(out[0, 0], u[0, 0])


def test_internal_energy_unchanged():
    u = _state(2)
    r = np.random.default_rng(3)
    phi = r.standard_normal((1, N + 2, N + 2, N + 2))
    out = gravity.apply(u, phi, 0.02, 1.0 / N)
    ein = lambda v: v[0, 4] - 0.5 * (v[0, 1] ** 2 + v[0, 2] ** 2 + v[0, 3] ** 2) / v[0, 0]
    assert np.abs(out[0, 1:4] - u[0, 1:4]).max() > 1e-3
    np.testing.assert_allclose(ein(out), ein(u), rtol=1e-12, atol=1e-12 * np.abs(u[0, 4]).max())


def test_axis_without_gradient():
    u = _state(4)
    phi, _ = _phi(lambda x, y, z: np.sin(3 * x) + 0 * y + 0 * z)
    out = gravity.apply(u, phi, 0.02, 1.0 / N)
    assert np.array_equal(out[0, 2], u[0, 2]) and np.array_equal(out[0, 3], u[0, 3])
    assert not np.array_equal(out[0, 1], u[0, 1])


_apply = gravity.apply


def _mutants():
    def one_sided(u, phi, dt, dh):
        # forward differences: phi at the cell instead of phi_{-d}
        p = np.array(phi, copy=True)
        p[:, :, :, :-1] = phi[:, :, :, 1:]
        return _apply(u, p, dt, dh)

    def wrong_sign(u, phi, dt, dh):
        return _apply(u, -np.asarray(phi), dt, dh)

    def old_momentum_energy(u, phi, dt, dh):
        out = _apply(u, phi, dt, dh)
        # energy gain with the old momentum only: 2 m . g dt / 2
        du = out[:, 1:4] - np.asarray(u)[:, 1:4]
        out[:, 4] = np.asarray(u)[:, 4] + (np.asarray(u)[:, 1:4] * du).sum(axis=1) / np.asarray(u)[:, 0]
        return out
    return {"one-sided difference": one_sided, "wrong sign": wrong_sign,
            "energy from the old momentum": old_momentum_energy}


@pytest.mark.parametrize("name", list(_mutants()))
def test_planted_mistakes_are_caught(name, monkeypatch):
    bad = _mutants()[name]
    failed = []
    for test in (test_uniform_and_linear_fields, test_internal_energy_unchanged, test_axis_without_gradient):
        with monkeypatch.context() as m:
            m.setattr(gravity, "apply", bad)
            try:
                test()
            except AssertionError:
                failed.append(test.__name__)
    assert failed, f"mutant '{name}' passed every pin"
