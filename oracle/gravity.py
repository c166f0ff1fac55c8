"""The self-gravity source operator G, for the oracle (test infrastructure
only; nothing on the product path imports it).

Sec. 2.3 (last paragraphs): cell-centred accelerations g = -grad phi from
3-point central differences, and the flow variables advanced by Eqs.
(MomConserve) and (EnergyConserve) with the flux terms dropped,

    d(rho v)/dt = rho g,        de/dt = rho v . g,

the continuity equation being unchanged; with the split order xyzGGzyx the
two G operators merge into one of twice the time step.  numpy, in the dtype
of the inputs (FP64, or FP32 to mirror a lower-precision run).

Readings (the paper gives the operator, not its time discretisation):
  * momentum: m_d + (a rho) (phi_{-d} - phi_{+d}), a = dt / (2 dh) rounded
    once to the working precision;
  * energy: e + ((s_x + s_y) + s_z) b, s_d = (m_d + m_d') (phi_{-d} -
    phi_{+d}), b = dt / (4 dh) rounded once: the work of the time-centred
    momentum (m + m')/2, which changes the kinetic energy by exactly that
    much and leaves the internal energy e - |m|^2 / (2 rho) unchanged;
  * density unchanged.
"""
from __future__ import annotations

import numpy as np


def apply(u, phi, dt: float, dh):
    """G on blocks: u (B, 5, n, n, n) interiors, phi (B, n+2, n+2, n+2) the
    potential with one ghost layer; dt a scalar, dh a scalar or one value per
    block.  Returns the new u."""
    u = np.array(u, copy=True)
    phi = np.asarray(phi)
    T = u.dtype.type
    B = u.shape[0]
    dh = np.broadcast_to(np.asarray(dh, dtype=np.float64), (B,))
    a = np.array([T(dt / (2.0 * h)) for h in dh]).reshape(B, 1, 1, 1)
    b = np.array([T(dt / (4.0 * h)) for h in dh]).reshape(B, 1, 1, 1)
    # phi_{-d} - phi_{+d} at every interior cell, d = x, y, z
    dphi = [phi[:, 1:-1, 1:-1, :-2] - phi[:, 1:-1, 1:-1, 2:],
            phi[:, 1:-1, :-2, 1:-1] - phi[:, 1:-1, 2:, 1:-1],
            phi[:, :-2, 1:-1, 1:-1] - phi[:, 2:, 1:-1, 1:-1]]
    rho = u[:, 0]
    ar = a * rho
    s = []
    for d in range(3):
        m = u[:, 1 + d]
        m_new = m + ar * dphi[d]
        s.append((m + m_new) * dphi[d])
        u[:, 1 + d] = m_new
    u[:, 4] = u[:, 4] + ((s[0] + s[1]) + s[2]) * b
    return u
