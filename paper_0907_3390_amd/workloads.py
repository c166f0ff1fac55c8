"""Seeded synthetic inputs for the relaxing-TVD patch advance.

This module only builds initial states: it holds none of the scheme's
arithmetic, so that the oracle and the HIP path can both be fed from it
without sharing solver code.  Every generator returns conserved variables
(rho, m_x, m_y, m_z, e) in FP64 as an array of shape (5, Nz, Ny, Nx), x
fastest, built from primitive variables with the ideal-gas relations of
Eqs. (ThermalEnergy) and (EOS) of Schive, Tsai & Chiueh (GAMER, 2010).

The shapes and value distributions stand in for the paper's workloads: its
test problems (Sec. 4: sound wave, Sod shock tube, Sedov-Taylor blast) and,
for throughput, its cosmological runs (Sec. 5), whose initial conditions are
not available; those are replaced by lognormal densities with Gaussian
velocities on the paper's patch geometry (8^3 patches, 2^3 patch families).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GAMMA = 5.0 / 3.0


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def conserved(rho, vx, vy, vz, P, gamma: float = GAMMA):
    """Stack primitive fields into conserved variables (5, ...) in FP64."""
    rho = np.asarray(rho, dtype=np.float64)
    shape = rho.shape
    vx = np.broadcast_to(np.asarray(vx, dtype=np.float64), shape)
    vy = np.broadcast_to(np.asarray(vy, dtype=np.float64), shape)
    vz = np.broadcast_to(np.asarray(vz, dtype=np.float64), shape)
    P = np.broadcast_to(np.asarray(P, dtype=np.float64), shape)
    if gamma == 1.0:
        if np.any(P != 0.0):
            raise ValueError("gamma = 1 describes pressureless gas only")
        eint = np.zeros(shape)
    else:
        eint = P / (gamma - 1.0)
    e = eint + 0.5 * rho * (vx * vx + vy * vy + vz * vz)
    return np.stack([rho, rho * vx, rho * vy, rho * vz, e]).astype(np.float64)


def uniform(N, rho=1.0, v=(0.0, 0.0, 0.0), P=1.0, gamma: float = GAMMA):
    Nz, Ny, Nx = (N, N, N) if np.isscalar(N) else N
    ones = np.ones((Nz, Ny, Nx))
    return conserved(rho * ones, v[0], v[1], v[2], P * ones, gamma)


def sod_x(N: int = 32, gamma: float = GAMMA, split: int | None = None,
          left=(1.0, 1.0), right=(0.125, 0.1), ny: int | None = None, nz: int | None = None):
    """Sod shock tube along x (Sec. 4.2 states): cells with x index < split take
    the left state (rho, P), the others the right state; gas at rest."""
    ny = N if ny is None else ny
    nz = N if nz is None else nz
    split = N // 2 if split is None else split
    x = np.arange(N)
    rho1 = np.where(x < split, left[0], right[0])
    P1 = np.where(x < split, left[1], right[1])
    rho = np.broadcast_to(rho1, (nz, ny, N)).copy()
    P = np.broadcast_to(P1, (nz, ny, N)).copy()
    return conserved(rho, 0.0, 0.0, 0.0, P, gamma)


def acoustic(N: int, amplitude: float = 1e-6, k=(1, 0, 0), rho0: float = 1.0,
             P0: float = 0.6, gamma: float = GAMMA, shape=None):
    """Standing sound wave at rest (Sec. 4.1 background: rho0 = 1, P0 = 3/5, so
    c_s = 1): rho = rho0 (1 + A sin(2 pi k.x / L)), adiabatic pressure
    perturbation dP = c_s^2 drho, zero velocity; cell centres at (i + 1/2)/N.
    ``shape`` = (Nz, Ny, Nx) overrides the cubic N^3 box (unit cell size)."""
    Nz, Ny, Nx = (N, N, N) if shape is None else shape
    cs2 = gamma * P0 / rho0
    z, y, x = np.meshgrid((np.arange(Nz) + 0.5) / Nz, (np.arange(Ny) + 0.5) / Ny,
                          (np.arange(Nx) + 0.5) / Nx, indexing="ij")
    phase = 2.0 * np.pi * (k[0] * x + k[1] * y + k[2] * z)
    drho = rho0 * amplitude * np.sin(phase)
    return conserved(rho0 + drho, 0.0, 0.0, 0.0, P0 + cs2 * drho, gamma)


def lognormal(N: int, seed: int, sigma_ln: float = 1.0, vel_sigma_rel: float = 0.3,
              P0: float = 1.0, gamma: float = GAMMA):
    """Rough synthetic state: mean-one lognormal density rho = exp(s g - s^2/2)
    with g ~ N(0, 1) iid per cell, Gaussian velocity components with standard
    deviation vel_sigma_rel * sqrt(gamma P0 / 1), uniform pressure P0."""
    r = rng(seed)
    g = r.standard_normal((N, N, N))
    rho = np.exp(sigma_ln * g - 0.5 * sigma_ln * sigma_ln)
    cs0 = math.sqrt(gamma * P0)
    v = r.standard_normal((3, N, N, N)) * (vel_sigma_rel * cs0)
    return conserved(rho, v[0], v[1], v[2], P0, gamma)


def smooth_random(N: int, seed: int, amplitude: float = 0.2, modes: int = 4,
                  rho0: float = 1.0, P0: float = 1.0, vel: float = 0.3,
                  gamma: float = GAMMA):
    """Smooth periodic state: a few random-phase Fourier modes with integer
    wavevectors (|k_i| <= 2) in density, pressure and all three velocities."""
    r = rng(seed)
    z, y, x = np.meshgrid((np.arange(N) + 0.5) / N, (np.arange(N) + 0.5) / N,
                          (np.arange(N) + 0.5) / N, indexing="ij")

    def field_():
        f = np.zeros((N, N, N))
        for _ in range(modes):
            k = r.integers(-2, 3, size=3)
            ph = r.uniform(0, 2 * np.pi)
            a = r.uniform(-1, 1)
            f += a * np.sin(2 * np.pi * (k[0] * x + k[1] * y + k[2] * z) + ph)
        return f / modes

    rho = rho0 * (1.0 + amplitude * field_())
    P = P0 * (1.0 + amplitude * field_())
    vx, vy, vz = (vel * field_() for _ in range(3))
    return conserved(rho, vx, vy, vz, P, gamma)


def sedov_lognormal(N: int, seed: int, sigma_ln: float = 0.5, E: float = 1.0,
                    P_bg: float = 1e-5, gamma: float = GAMMA):
    """Point blast on a lognormal background (Sec. 4.3 set-up, scaled): the
    energy E is deposited as thermal energy in the central 2^3 cells (indices
    N/2-1 and N/2 on every axis), background pressure P_bg, gas at rest, unit
    box so dh = 1/N."""
    r = rng(seed)
    g = r.standard_normal((N, N, N))
    rho = np.exp(sigma_ln * g - 0.5 * sigma_ln * sigma_ln)
    u = conserved(rho, 0.0, 0.0, 0.0, P_bg, gamma)
    dh = 1.0 / N
    c = slice(N // 2 - 1, N // 2 + 1)
    u[4, c, c, c] = E / (8.0 * dh ** 3)
    return u


# ---------------------------------------------------------------------------
# uneven batch of independent periodic boxes
# ---------------------------------------------------------------------------

@dataclass
class BoxSet:
    """Independent periodic boxes of mixed edge, each with its own zone size."""
    grids: list = field(default_factory=list)   # each (5, n, n, n) FP64
    dh: list = field(default_factory=list)


def sound_wave_boxes(counts=(2286, 1143, 571), edges=(8, 16, 32), seed: int = 4,
                     amplitude: float = 1e-3, rho0: float = 1.0, P0: float = 0.6,
                     gamma: float = GAMMA, modes: int = 4) -> BoxSet:
    """Independent unit periodic boxes of mixed sizes (counts per edge), each
    holding one traveling fundamental sound wave plus ``modes`` random-phase
    traveling modes with integer wavevectors |k_i| <= 2, normalised to a total
    relative density amplitude ``amplitude``; adiabatic dP = c_s^2 drho and
    velocity c_s (drho / rho0) k_hat per mode (Sec. 4.1 background)."""
    r = rng(seed)
    cs = math.sqrt(gamma * P0 / rho0)
    out = BoxSet()
    order = []
    for e, c in zip(edges, counts):
        order += [e] * c
    for n in order:
        z, y, x = np.meshgrid((np.arange(n) + 0.5) / n, (np.arange(n) + 0.5) / n,
                              (np.arange(n) + 0.5) / n, indexing="ij")
        ks = [np.array([1, 0, 0])]
        amps = [1.0]
        phs = [0.0]
        for _ in range(modes):
            k = r.integers(-2, 3, size=3)
            while not k.any():
                k = r.integers(-2, 3, size=3)
            ks.append(k)
            amps.append(r.uniform(0.2, 1.0))
            phs.append(r.uniform(0, 2 * np.pi))
        norm = amplitude / sum(amps)
        drho = np.zeros((n, n, n))
        v = np.zeros((3, n, n, n))
        for k, a, ph in zip(ks, amps, phs):
            w = norm * a * np.sin(2 * np.pi * (k[0] * x + k[1] * y + k[2] * z) + ph)
            drho += rho0 * w
            kh = k / np.linalg.norm(k)
            for ax in range(3):
                v[ax] += cs * w * kh[ax]
        out.grids.append(conserved(rho0 + drho, v[0], v[1], v[2], P0 + cs * cs * drho, gamma))
        out.dh.append(1.0 / n)
    return out
