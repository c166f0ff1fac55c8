"""Red-black SOR for the Poisson equation on patch groups, for the oracle
(test infrastructure only; nothing on the product path imports it).

Sec. 2.3: on refined levels the discrete Poisson equation (Eq.
DiscretePoisson, the 7-point Laplacian) is solved patch group by patch group
with Dirichlet boundary values in one ghost layer, by successive
overrelaxation: the residual of a cell (Eq. Residual)

    R = (phi_{i+1} + phi_{j+1} + phi_{k+1} + phi_{i-1} + phi_{j-1} + phi_{k-1}
         - 6 phi) - 4 pi G rho dh^2

and the update phi <- phi + omega R / 6 (Eq. SOR), first for all even cells
(i + j + k even) from the odd ones, then for all odd cells from the updated
even ones (odd-even ordering); iterations stop when the one-norm of the
residuals reaches the floating-point precision of the one-norm of the source
term.  Sec. 3.2: a patch group holds 18^3 potentials (16^3 interior and the
ghost layer) and 16^3 densities.

Written with numpy on whole arrays, in the dtype of the inputs (FP64, or FP32
to mirror a lower-precision run operation by operation).

Readings (the paper leaves them open):
  * parity of a cell: its interior indices (0 .. 15), x + y + z;
  * the six neighbours are summed in the order of Eq. (Residual): x+1, y+1,
    z+1, x-1, y-1, z-1, then 6 phi is subtracted, then the source term
    s = (4 pi G dh^2) rho, the factor rounded once to the working precision;
  * the update is phi + (omega / 6) R, the factor rounded once;
  * the residual norm of an iteration is the sum of |R| over the even cells
    (from the even step) and the odd cells (from the odd step);
  * "the floating-point precision limit compared to the source term": the
    residual of a cell is computed from terms of the size of 6 phi and s,
    so its rounding floor scales with them; stop when that norm <=
    tol * (sum |s| + 6 sum |phi|) after the iteration, tol = 16 u by default
    (u the unit roundoff of the working precision), once at least min_iter
    iterations are done, or after max_iter iterations;
  * omega defaults to the optimum for the Dirichlet box of n interior cells,
    2 / (1 + sin(pi / (n + 1))): the Jacobi iteration's spectral radius is
    cos(pi / (n + 1)) there.
"""
from __future__ import annotations

import math

import numpy as np

N = 16          # interior edge of a patch group


def omega_opt(n: int = N) -> float:
    """Optimal overrelaxation for red-black SOR on an n^3 Dirichlet box."""
    return 2.0 / (1.0 + math.sin(math.pi / (n + 1)))


def _parity_masks(n):
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    even = (x + y + z) % 2 == 0
    return even, ~even


def _residual(phi, src):
    """Eq. (Residual) for every interior cell of phi (G, n+2, n+2, n+2)."""
    c = phi[:, 1:-1, 1:-1, 1:-1]
    s = phi[:, 1:-1, 1:-1, 2:]            # x + 1
    s = s + phi[:, 1:-1, 2:, 1:-1]        # y + 1
    s = s + phi[:, 2:, 1:-1, 1:-1]        # z + 1
    s = s + phi[:, 1:-1, 1:-1, :-2]       # x - 1
    s = s + phi[:, 1:-1, :-2, 1:-1]       # y - 1
    s = s + phi[:, :-2, 1:-1, 1:-1]       # z - 1
    six = phi.dtype.type(6)
    return (s - six * c) - src


def source(rho, G: float, dh):
    """The source term 4 pi G dh^2 rho, with (4 pi G dh^2) rounded once to the
    dtype of rho; dh a scalar or one value per group."""
    rho = np.asarray(rho)
    fac = np.asarray(4.0 * math.pi * G * np.asarray(dh, dtype=np.float64) ** 2)
    fac = fac.astype(rho.dtype).reshape((-1,) + (1,) * (rho.ndim - 1) if fac.ndim else ())
    return fac * rho


def default_tol(dtype) -> float:
    """16 unit roundoffs of the working precision."""
    return 16.0 * float(np.finfo(dtype).eps) / 2.0


def sor(phi, src, omega: float | None = None, min_iter: int = 0, max_iter: int = 1000,
        tol: float | None = None):
    """Red-black SOR on patch groups: phi (G, n+2, n+2, n+2) holds the initial
    guess inside and the Dirichlet values in the ghost layer, src (G, n, n, n)
    the source term.  Groups iterate independently, each until its own
    stopping rule holds.  Returns (phi, iterations per group, last residual
    norm per group)."""
    phi = np.array(phi, copy=True)
    src = np.asarray(src)
    dt = phi.dtype.type
    n = phi.shape[1] - 2
    omega = omega_opt(n) if omega is None else omega
    w6 = dt(omega / 6.0)
    if tol is None:
        tol = default_tol(phi.dtype)
    src_norm = np.abs(src.astype(np.float64)).reshape(len(src), -1).sum(axis=1)
    even, odd = _parity_masks(n)
    iters = np.zeros(len(phi), dtype=np.int64)
    norm = np.full(len(phi), np.inf)
    active = np.ones(len(phi), dtype=bool)
    for it in range(max_iter):
        if not active.any():
            break
        a = np.nonzero(active)[0]
        p = phi[a]
        tot = np.zeros(len(a))
        for mask in (even, odd):
            R = _residual(p, src[a])
            inner = p[:, 1:-1, 1:-1, 1:-1]
            upd = inner + w6 * R
            inner[:, mask] = upd[:, mask]
            tot += np.abs(R[:, mask].astype(np.float64)).reshape(len(a), -1).sum(axis=1)
        phi[a] = p
        iters[a] += 1
        norm[a] = tot
        phi_norm = np.abs(p[:, 1:-1, 1:-1, 1:-1].astype(np.float64)).reshape(len(a), -1).sum(axis=1)
        done = (iters[a] >= min_iter) & (tot <= tol * (src_norm[a] + 6.0 * phi_norm))
        active[a[done]] = False
    return phi, iters, norm
