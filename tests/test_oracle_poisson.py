"""Pins of the oracle's red-black SOR Poisson solver (Sec. 2.3, Eqs.
DiscretePoisson, Residual, SOR; Sec. 3.2 patch groups) against what the
mathematics fixes, not against its own formulas:

* a quadratic potential is an exact solution of the 7-point equation, and a
  product of discrete sine modes (zero on the ghost layer) an exact
  eigenfunction with eigenvalue sum_a 2 (cos theta_a - 1): SOR converges to
  both to round-off, with per-axis mode numbers that tell the axes apart;
* with omega = 1, after an iteration the cells updated last (the odd ones)
  have zero residual, checked with an independent 7-point convolution
  (scipy.ndimage), which pins the update factor and the odd-even order;
* the asymptotic error reduction per iteration is the closed form of red-
  black SOR on the Dirichlet box: cos^2(pi / (n + 1)) for omega = 1 (the
  square of the Jacobi spectral radius) and omega - 1 at the optimum;
* the stopping rule ends the iteration at the first iteration whose residual
  norm is within 16 unit roundoffs of the size of the residual's terms, and
  the solution is then exact to round-off.
Planted mistakes (a dropped neighbour, the wrong update factor, the odd cells
first, the source with the wrong sign) each fail one of these.
"""
import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import poisson

N = 16


def _centres(n=N, h=1.0 / N):
    c = (np.arange(-1, n + 1) + 0.5) * h
    return np.meshgrid(c, c, c, indexing="ij")   # z, y, x of ghosted cells


def _laplacian7(phi):
    """sum of the six neighbours minus 6 phi on the interior of ghosted arrays,
    by an independent convolution."""
    k = np.zeros((3, 3, 3))
    k[1, 1, 0] = k[1, 1, 2] = k[1, 0, 1] = k[1, 2, 1] = k[0, 1, 1] = k[2, 1, 1] = 1.0
    k[1, 1, 1] = -6.0
    out = np.stack([ndimage.convolve(p, k, mode="constant") for p in phi])
    return out[:, 1:-1, 1:-1, 1:-1]


def test_quadratic_is_exact():
    h = 1.0 / N
    z, y, x = _centres()
    a, b, c = 0.7, -0.4, 1.3
    exact = a * x * x + b * y * y + c * z * z + 0.2 * x - 0.5 * z + 1.0
    G = 1.0
    rho = np.full((N, N, N), (2 * a + 2 * b + 2 * c) / (4 * math.pi * G))
    phi0 = exact.copy()
    phi0[1:-1, 1:-1, 1:-1] = 0.0
    src = poisson.source(rho[None], G, h)
    phi, it, norm = poisson.sor(phi0[None], src, max_iter=2000)
    assert it[0] < 2000
    np.testing.assert_allclose(phi[0], exact, rtol=0, atol=1e-12 * np.abs(exact).max())


@pytest.mark.parametrize("modes", [(1, 2, 3), (3, 1, 2)])
def test_discrete_sine_eigenmode(modes):
    n = N
    idx = np.arange(-1, n + 1) + 1                     # 0 and n+1 on the ghost layer
    th = [k * math.pi / (n + 1) for k in modes]        # x, y, z
    sx, sy, sz = (np.sin(t * idx) for t in th)
    exact = sz[:, None, None] * sy[None, :, None] * sx[None, None, :]
    lam = sum(2.0 * (math.cos(t) - 1.0) for t in th)
    src = (lam * exact[1:-1, 1:-1, 1:-1])[None]
    phi0 = np.zeros_like(exact)
    phi, it, _ = poisson.sor(phi0[None], src, max_iter=3000)
    np.testing.assert_allclose(phi[0], exact, rtol=0, atol=1e-12)


def test_gauss_seidel_odd_cells_have_zero_residual():
    r = np.random.default_rng(3)
    phi0 = r.standard_normal((2, N + 2, N + 2, N + 2))
    src = r.standard_normal((2, N, N, N)) * 0.1
    phi, _, _ = poisson.sor(phi0, src, omega=1.0, max_iter=1)
    R = _laplacian7(phi) - src
    zz, yy, xx = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    odd = (xx + yy + zz) % 2 == 1
    assert np.abs(R[:, odd]).max() <= 1e-14
    assert np.abs(R[:, ~odd]).max() > 1e-3
    # the ghost layer is never touched
    assert np.array_equal(phi[:, 0], phi0[:, 0]) and np.array_equal(phi[:, :, :, -1], phi0[:, :, :, -1])


def _rate(omega, it0, it1):
    r = np.random.default_rng(4)
    phi = np.zeros((1, N + 2, N + 2, N + 2))
    phi[0, 1:-1, 1:-1, 1:-1] = r.standard_normal((N, N, N))
    src = np.zeros((1, N, N, N))
    phi, _, _ = poisson.sor(phi, src, omega=omega, min_iter=it0, max_iter=it0)
    e0 = np.abs(phi).sum()
    phi, _, _ = poisson.sor(phi, src, omega=omega, min_iter=it1 - it0, max_iter=it1 - it0)
    e1 = np.abs(phi).sum()
    return (e1 / e0) ** (1.0 / (it1 - it0))


def test_convergence_rate_closed_form():
    rho_j = math.cos(math.pi / (N + 1))
    assert _rate(1.0, 150, 250) == pytest.approx(rho_j ** 2, rel=2e-3)
    w = poisson.omega_opt(N)
    assert w == pytest.approx(2.0 / (1.0 + math.sqrt(1.0 - rho_j ** 2)), rel=1e-15)
    # at the optimum the iteration matrix has a double eigenvalue w - 1, so
    # the asymptotic rate is approached slowly (a factor k per k iterations)
    assert _rate(w, 200, 300) == pytest.approx(w - 1.0, rel=3e-2)


def test_stopping_rule():
    h = 1.0 / N
    z, y, x = _centres()
    exact = x * x - y * y + 0.5 * z * z
    rho = np.full((1, N, N, N), 1.0 / (4 * math.pi) * (2 - 2 + 1) / 1.0)
    phi0 = exact.copy()[None]
    phi0[:, 1:-1, 1:-1, 1:-1] = 0.0
    src = poisson.source(rho, 1.0, h)
    phi, it, norm = poisson.sor(phi0, src, max_iter=5000)
    bound = lambda p, dt: poisson.default_tol(dt) * (np.abs(src).sum() + 6 * np.abs(p[0, 1:-1, 1:-1, 1:-1]).sum())
    assert 10 < it[0] < 5000 and norm[0] <= bound(phi, np.float64)
    # one iteration fewer had not yet met the rule
    p2, it2, norm2 = poisson.sor(phi0, src, min_iter=it[0] - 1, max_iter=it[0] - 1)
    assert norm2[0] > bound(p2, np.float64)
    # the solution is then exact to round-off
    np.testing.assert_allclose(phi[0], exact, rtol=0, atol=1e-13 * np.abs(exact).max())
    # FP32 stops at its own precision, in fewer iterations
    p32, it32, n32 = poisson.sor(phi0.astype(np.float32), src.astype(np.float32), max_iter=5000)
    assert it32[0] < it[0] and n32[0] <= bound(p32, np.float32)


_residual = poisson._residual
_masks = poisson._parity_masks
_sor = poisson.sor


def _mutants():
    def dropped_neighbour(phi, src):
        c = phi[:, 1:-1, 1:-1, 1:-1]
        s = phi[:, 1:-1, 1:-1, 2:] + phi[:, 1:-1, 2:, 1:-1] + phi[:, 2:, 1:-1, 1:-1]
        s = s + phi[:, 1:-1, 1:-1, 2:] + phi[:, 1:-1, :-2, 1:-1] + phi[:, :-2, 1:-1, 1:-1]
        return (s - 6 * c) - src

    def flipped_source(phi, src):
        return _residual(phi, -src)

    def odd_first(n):
        e, o = _masks(n)
        return o, e

    def wrong_factor(phi, src, omega=None, **kw):
        w = poisson.omega_opt(phi.shape[1] - 2) if omega is None else omega
        return _sor(phi, src, omega=w * 6.0 / 5.0 if w * 6.0 / 5.0 < 2 else w * 0.8, **kw)
    return {"x-1 neighbour replaced by x+1": ("_residual", dropped_neighbour),
            "source with the wrong sign": ("_residual", flipped_source),
            "odd cells first": ("_parity_masks", odd_first),
            "update factor omega/5": ("sor", wrong_factor)}


@pytest.mark.parametrize("name", list(_mutants()))
def test_planted_mistakes_are_caught(name, monkeypatch):
    attr, bad = _mutants()[name]
    failed = []
    for test, kw in ((test_quadratic_is_exact, {}), (test_discrete_sine_eigenmode, {"modes": (1, 2, 3)}),
                     (test_gauss_seidel_odd_cells_have_zero_residual, {}),
                     (test_convergence_rate_closed_form, {})):
        with monkeypatch.context() as m:
            m.setattr(poisson, attr, bad)
            try:
                test(**kw)
            except AssertionError:
                failed.append(test.__name__)
    assert failed, f"mutant '{name}' passed every pin"
