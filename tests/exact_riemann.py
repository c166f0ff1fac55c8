"""Exact solution of the 1-D Riemann problem for an ideal gas.

Independent of the oracle: a textbook construction (Godunov's exact solver
as presented in Toro, "Riemann Solvers and Numerical Methods for Fluid
Dynamics", Ch. 4).  The star pressure solves f_L(p) + f_R(p) + (u_R - u_L) = 0
where f_K is the shock (Rankine-Hugoniot) branch for p > p_K and the
rarefaction (isentropic) branch otherwise; the self-similar solution is then
sampled at x/t.  Used to pin the oracle on the paper's Sod problem (Sec. 4.2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class StarState:
    p: float
    u: float
    rho_L: float
    rho_R: float
    shock_speed_R: float | None
    shock_speed_L: float | None
    head_L: float | None
    tail_L: float | None


def _fK(p, rho, pK, gamma):
    aK = math.sqrt(gamma * pK / rho)
    if p > pK:
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pK
        f = (p - pK) * math.sqrt(A / (p + B))
        df = math.sqrt(A / (B + p)) * (1.0 - 0.5 * (p - pK) / (B + p))
    else:
        f = 2.0 * aK / (gamma - 1.0) * ((p / pK) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)
        df = 1.0 / (rho * aK) * (p / pK) ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


def star_state(rhoL, uL, pL, rhoR, uR, pR, gamma) -> StarState:
    aL = math.sqrt(gamma * pL / rhoL)
    aR = math.sqrt(gamma * pR / rhoR)
    # two-rarefaction guess, then Newton
    z = (gamma - 1.0) / (2.0 * gamma)
    p = ((aL + aR - 0.5 * (gamma - 1.0) * (uR - uL)) /
         (aL / pL ** z + aR / pR ** z)) ** (1.0 / z)
    for _ in range(100):
        fL, dfL = _fK(p, rhoL, pL, gamma)
        fR, dfR = _fK(p, rhoR, pR, gamma)
        dp = (fL + fR + uR - uL) / (dfL + dfR)
        p_new = max(p - dp, 1e-14)
        if abs(p_new - p) < 1e-15 * (p_new + p):
            p = p_new
            break
        p = p_new
    fL, _ = _fK(p, rhoL, pL, gamma)
    fR, _ = _fK(p, rhoR, pR, gamma)
    u = 0.5 * (uL + uR) + 0.5 * (fR - fL)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    # left wave
    if p > pL:
        rho_sL = rhoL * ((p / pL + g1) / (g1 * p / pL + 1.0))
        sL = uL - aL * math.sqrt((gamma + 1.0) / (2 * gamma) * p / pL + (gamma - 1.0) / (2 * gamma))
        headL = tailL = None
    else:
        rho_sL = rhoL * (p / pL) ** (1.0 / gamma)
        sL = None
        headL = uL - aL
        tailL = u - aL * (p / pL) ** ((gamma - 1.0) / (2.0 * gamma))
    # right wave
    if p > pR:
        rho_sR = rhoR * ((p / pR + g1) / (g1 * p / pR + 1.0))
        sR = uR + aR * math.sqrt((gamma + 1.0) / (2 * gamma) * p / pR + (gamma - 1.0) / (2 * gamma))
    else:
        rho_sR = rhoR * (p / pR) ** (1.0 / gamma)
        sR = None
    return StarState(p, u, rho_sL, rho_sR, sR, sL, headL, tailL)


def sample(xi, rhoL, uL, pL, rhoR, uR, pR, gamma):
    """Density, velocity and pressure at similarity coordinates xi = x / t.
    Covers left rarefaction / right shock configurations (Sod-type)."""
    st = star_state(rhoL, uL, pL, rhoR, uR, pR, gamma)
    aL = math.sqrt(gamma * pL / rhoL)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    if st.head_L is None or st.shock_speed_R is None:
        raise NotImplementedError("only left-rarefaction / right-shock problems")
    for i, s in enumerate(xi.ravel()):
        if s <= st.head_L:
            r, v, pp = rhoL, uL, pL
        elif s <= st.tail_L:
            v = 2.0 / (gamma + 1.0) * (aL + 0.5 * (gamma - 1.0) * uL + s)
            c = 2.0 / (gamma + 1.0) * (aL + 0.5 * (gamma - 1.0) * (uL - s))
            r = rhoL * (c / aL) ** (2.0 / (gamma - 1.0))
            pp = pL * (c / aL) ** (2.0 * gamma / (gamma - 1.0))
        elif s <= st.u:
            r, v, pp = st.rho_L, st.u, st.p
        elif s <= st.shock_speed_R:
            r, v, pp = st.rho_R, st.u, st.p
        else:
            r, v, pp = rhoR, uR, pR
        rho.ravel()[i] = r
        u.ravel()[i] = v
        p.ravel()[i] = pp
    return rho, u, p
