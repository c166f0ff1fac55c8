"""An independent 50-digit reference of one 1-D update of the relaxing TVD
scheme, for pinning the FP64 oracle on tiny inputs.

Written from the equations of Sec. 2.2 and the per-thread steps of the GPU
solver in Sec. 3.1, not from the oracle's source.  It works on whole
pencils with mpmath numbers and dictionaries keyed by cell index, and takes
the paper's forms literally where they are well defined:

* Eqs. (ThermalEnergy), (EOS): v = m / rho, epsilon = e - rho |v|^2 / 2,
  P = (gamma - 1) epsilon (with the pressure floor P* = max(P, p_floor));
* Sec. 2.2: freezing speed c = |v_d| + c_s, c_s = sqrt(gamma P* / rho);
* Eq. (LRFlux): w = F / c, F^R = c (u + w) / 2, F^L = c (u - w) / 2 (the
  limit (c u +- F) / 2 where c = 0);
* first-order upwind fluxes: F^R at n+1/2 from cell n, F^L at n+1/2 from
  cell n+1 (it moves left), Eq. (MidpointValue) for the half step;
* Sec. 3.1 step 5: freezing speed and auxiliary vector recomputed from the
  midpoint values;
* Eqs. (2ndTVDFluxCorr)-(2ndRFlux) with the van Leer limiter of Eq.
  (vanLeer) on the halved differences for F^R, and the same construction
  reflected about the interface for F^L (upwind cell n+1);
* Eq. (FullstepValue) from u^t with the midpoint fluxes.

Variables are in the global order (rho, m_x, m_y, m_z, e); the sweep axis
d picks the normal momentum.
"""
from __future__ import annotations

import mpmath

DIGITS = 50


def _mpf(x):
    return mpmath.mpf(x)


def primitive_flux(u, d, gamma, p_floor):
    """(c, F): freezing speed and flux vector along axis d of one cell."""
    rho, e = u[0], u[4]
    v = [u[1 + a] / rho for a in range(3)]
    eps = e - rho * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2) / 2
    P = (gamma - 1) * eps
    if P < p_floor:
        P = p_floor
    cs = mpmath.sqrt(gamma * P / rho)
    c = abs(v[d]) + cs
    F = [rho * v[d]]
    F += [rho * v[a] * v[d] + (P if a == d else 0) for a in range(3)]
    F += [(e + P) * v[d]]
    return c, F


def lr_fluxes(u, d, gamma, p_floor):
    """Eq. (LRFlux) of one cell: (F^R, F^L)."""
    c, F = primitive_flux(u, d, gamma, p_floor)
    if c == 0:
        return [f / 2 for f in F], [-f / 2 for f in F]
    w = [f / c for f in F]
    FR = [c * (u[k] + w[k]) / 2 for k in range(5)]
    FL = [c * (u[k] - w[k]) / 2 for k in range(5)]
    return FR, FL


def vanleer(a, b):
    """Eq. (vanLeer)."""
    if a * b > 0:
        return 2 * a * b / (a + b)
    return mpmath.mpf(0)


def update(pencil, d, dt, dh, gamma, p_floor=0.0):
    """One 1-D update of a pencil of n+6 cells (rows of 5 numbers, cells
    -3 .. n+2); returns the n updated interior cells as lists of mpf."""
    with mpmath.workdps(DIGITS):
        gamma, p_floor = _mpf(gamma), _mpf(p_floor)
        dt, dh = _mpf(dt), _mpf(dh)
        M = len(pencil)
        n = M - 6
        # cells indexed by their position i = -3 .. n+2
        u = {i - 3: [_mpf(x) for x in pencil[i]] for i in range(M)}
        # time t: split fluxes of every cell
        FR, FL = {}, {}
        for i, ui in u.items():
            FR[i], FL[i] = lr_fluxes(ui, d, gamma, p_floor)

        # first-order upwind flux through i+1/2
        def F1(i):
            return [FR[i][k] - FL[i + 1][k] for k in range(5)]

        # Eq. (MidpointValue) for cells -2 .. n+1
        half = {}
        for i in range(-2, n + 2):
            Fp, Fm = F1(i), F1(i - 1)
            half[i] = [u[i][k] - (Fp[k] - Fm[k]) / dh * (dt / 2) for k in range(5)]
        # midpoint split fluxes (freezing speed recomputed from the midpoint)
        HR, HL = {}, {}
        for i, hi in half.items():
            HR[i], HL[i] = lr_fluxes(hi, d, gamma, p_floor)

        # second-order fluxes through i+1/2 for i = -1 .. n-1
        def F2(i):
            out = []
            for k in range(5):
                R = HR[i][k] + vanleer((HR[i][k] - HR[i - 1][k]) / 2,
                                       (HR[i + 1][k] - HR[i][k]) / 2)
                L = HL[i + 1][k] + vanleer((HL[i + 1][k] - HL[i + 2][k]) / 2,
                                           (HL[i][k] - HL[i + 1][k]) / 2)
                out.append(R - L)
            return out

        flux = {i: F2(i) for i in range(-1, n)}
        # Eq. (FullstepValue) from u^t
        return [[u[i][k] - (flux[i][k] - flux[i - 1][k]) / dh * dt for k in range(5)]
                for i in range(n)]
