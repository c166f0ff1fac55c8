"""Plain FP64 CPU oracle for GAMER's relaxing TVD patch advance.

TEST INFRASTRUCTURE ONLY: the reference that the HIP path is checked
against.  It shares no code with the HIP path and imports nothing from it;
only the tests, the smoke check and the benchmark's CPU-baseline leg use it.

The arithmetic lives in ``tvd_oracle.c`` (plain C, FP64, compiled with gcc);
this module is the ctypes binding plus the step driver on periodic grids,
written with numpy.  Every routine cites the passage of Schive, Tsai &
Chiueh (GAMER, 2010) it follows:

* ``split_fluxes``     Eqs. (ThermalEnergy), (EOS), (LRFlux), Sec. 2.2
* ``vanleer``          Eq. (vanLeer)
* ``pencil``           Eqs. (MidpointValue)-(FullstepValue), the 1-D scheme
* ``advance_blocks``   Sec. 2.2 dimensional splitting (xyz forward, zyx
                       backward) with three ghost zones per side
* ``max_signal_speed`` Eq. (CFL)
* ``periodic_ghosted_blocks`` / ``run_periodic``: the step driver on a
                       uniform periodic grid cut into cubic blocks.
* ``oracle.ghosts``    Sec. 2.2 coarse-fine ghost zones: sibling copy, else
                       linear interpolation with the Min-Mod limiter from one
                       level coarser (numpy).
* ``oracle.closing``   Sec. 2.1 step 3 and Sec. 3.1 closing step: restriction
                       and coarse-fine flux correction (numpy).
* ``oracle.poisson``   Sec. 2.3 and Sec. 3.2: red-black SOR for the Poisson
                       equation on patch groups (numpy).
* ``oracle.gravity``   Sec. 2.3: the self-gravity source operator G (numpy).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tvd_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")
NVAR = 5
GHOST = 3

_lib = None


# ISO C99 keeps floating-point contraction off, so -O3 and -march change the
# speed, not the arithmetic.  The shipped build is portable (it may run on
# another host than the one that compiled it); CFLAGS_NATIVE is for a build
# made on the host that runs it.
CFLAGS = ["-O3", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall"]
CFLAGS_NATIVE = CFLAGS + ["-march=native"]


def build(verbose: bool = False, src: str = _SRC, out: str = _LIB, native: bool = False,
          extra=()) -> str:
    """Compile the C oracle with gcc (default: ``oracle/_build/liboracle.so``)."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp%d" % os.getpid()
    cmd = (["gcc"] + (CFLAGS_NATIVE if native else CFLAGS) + list(extra)
           + ["-o", tmp, src, "-lm"])
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def _bind(path: str):
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    llp = ctypes.POINTER(ctypes.c_longlong)
    ip = ctypes.POINTER(ctypes.c_int)
    lib.oracle_split_fluxes.restype = ctypes.c_double
    lib.oracle_split_fluxes.argtypes = [dp, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_double, dp, dp, ctypes.c_void_p]
    lib.oracle_vanleer.restype = ctypes.c_double
    lib.oracle_vanleer.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.oracle_pencil.restype = None
    lib.oracle_pencil.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                  dp, ctypes.c_void_p]
    lib.oracle_pencil_flux.restype = None
    lib.oracle_pencil_flux.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       dp, dp, ctypes.c_void_p]
    lib.oracle_advance_batch.restype = ctypes.c_int
    lib.oracle_advance_batch.argtypes = [dp, dp, ctypes.c_int, ip, llp, llp, dp, dp,
                                         ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                         dp, llp, llp, llp]
    lib.oracle_max_signal_speed.restype = ctypes.c_double
    lib.oracle_max_signal_speed.argtypes = [dp, ctypes.c_longlong, ctypes.c_longlong,
                                            ctypes.c_double, ctypes.c_double]
    lib.oracle_compensated_sum.restype = ctypes.c_double
    lib.oracle_compensated_sum.argtypes = [dp, ctypes.c_longlong, ctypes.c_double, dp]
    return lib


def _load():
    """The default library, built on first use if missing or stale."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    _lib = _bind(_LIB)
    return _lib


def use_library(path: str | None):
    """Point this module at another build of ``tvd_oracle.c`` (the tests use
    this to check that planted mistakes are caught by the pins); ``None``
    restores the default build."""
    global _lib
    _lib = None if path is None else _bind(path)


def set_threads(n: int):
    """Number of OpenMP threads the batch advance uses from now on (the
    OpenMP runtime the library links; a timing knob, no arithmetic)."""
    fn = _load().omp_set_num_threads
    fn.restype = None
    fn.argtypes = [ctypes.c_int]
    fn(int(n))


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ---------------------------------------------------------------------------
# cell, limiter and pencil level
# ---------------------------------------------------------------------------

def split_fluxes(u, d: int, gamma: float, p_floor: float = 0.0):
    """Eq. (LRFlux) for one cell swept along axis ``d``: returns (F^R, F^L, c)."""
    lib = _load()
    u = np.ascontiguousarray(u, dtype=np.float64)
    FR = np.zeros(NVAR)
    FL = np.zeros(NVAR)
    c = lib.oracle_split_fluxes(_dptr(u), d, gamma, p_floor, _dptr(FR), _dptr(FL), None)
    return FR, FL, c


def vanleer(a: float, b: float) -> float:
    """Eq. (vanLeer) applied to the two flux corrections ``a``, ``b``."""
    return _load().oracle_vanleer(float(a), float(b))


def pencil(q, d: int, dt: float, dh: float, gamma: float, p_floor: float = 0.0):
    """One 1-D update (Eqs. MidpointValue-FullstepValue) of an (n+6, 5) pencil."""
    lib = _load()
    q = np.ascontiguousarray(q, dtype=np.float64)
    n = q.shape[0] - 2 * GHOST
    out = np.zeros((n, NVAR))
    lib.oracle_pencil(_dptr(q), n, d, dt, dh, gamma, p_floor, _dptr(out), None)
    return out


def pencil_flux(q, d: int, dt: float, dh: float, gamma: float, p_floor: float = 0.0):
    """As ``pencil``, also returning the (n+1, 5) interface fluxes of the full
    step: row i is the flux through interface i-1/2 of interior cell i."""
    lib = _load()
    q = np.ascontiguousarray(q, dtype=np.float64)
    n = q.shape[0] - 2 * GHOST
    out = np.zeros((n, NVAR))
    hf = np.zeros((n + 1, NVAR))
    lib.oracle_pencil_flux(_dptr(q), n, d, dt, dh, gamma, p_floor, _dptr(out), _dptr(hf), None)
    return out, hf


# ---------------------------------------------------------------------------
# block level
# ---------------------------------------------------------------------------

@dataclass
class Counts:
    floored: int = 0
    nonphysical: int = 0
    threads: int = 1
    seconds: float = 0.0   # wall time inside the C advance (no marshalling)


PATCH = 8


def flux_record_shape(n: int):
    """Shape of one block's patch-boundary flux record (see ``advance_ragged``)."""
    return (3, n // PATCH + 1, NVAR, n, n)


def advance_ragged(blocks_in, order: int, dt, dh, gamma: float, p_floor: float = 0.0,
                   counts: Counts | None = None, fluxes: bool = False):
    """One step on a list of ghosted blocks of shape (5, n+6, n+6, n+6).

    ``dt`` and ``dh`` are scalars or per-block sequences.  ``order`` 0 is the
    forward xyz triple, 1 the backward zyx triple.  Returns the list of
    (5, n, n, n) interiors.

    With ``fluxes`` (n a multiple of 8) it returns (interiors, records): the
    record of a block, shape (3, n/8 + 1, 5, n, n), holds for each axis d and
    face plane f = 0, 8, .., n the flux through interface f-1/2 of every
    d-pencil, taken in the sweep along d, indexed [d, f/8, k, a, b] with
    (a, b) the other two axes, higher-numbered first (x: (z, y); y: (z, x);
    z: (y, x)).  These are the patch-boundary fluxes that the closing step
    (Sec. 3.1) hands to the coarse-fine flux correction (Sec. 2.1).
    """
    lib = _load()
    nb = len(blocks_in)
    if nb == 0:
        return ([], []) if fluxes else []
    edges = np.array([b.shape[1] - 2 * GHOST for b in blocks_in], dtype=np.int32)
    for b, n in zip(blocks_in, edges):
        if b.shape != (NVAR, n + 6, n + 6, n + 6):
            raise ValueError("ghosted block must have shape (5, n+6, n+6, n+6)")
    in_sizes = NVAR * (edges.astype(np.int64) + 6) ** 3
    out_sizes = NVAR * edges.astype(np.int64) ** 3
    in_off = np.concatenate([[0], np.cumsum(in_sizes)[:-1]]).astype(np.int64)
    out_off = np.concatenate([[0], np.cumsum(out_sizes)[:-1]]).astype(np.int64)
    flat_in = np.concatenate([np.ascontiguousarray(b, dtype=np.float64).ravel()
                              for b in blocks_in])
    flat_out = np.zeros(int(out_sizes.sum()))
    dt_a = np.broadcast_to(np.asarray(dt, dtype=np.float64), (nb,)).copy()
    dh_a = np.broadcast_to(np.asarray(dh, dtype=np.float64), (nb,)).copy()
    fl = ctypes.c_longlong(0)
    npy = ctypes.c_longlong(0)
    flux_p = flux_off_p = None
    if fluxes:
        if np.any(edges % PATCH):
            raise ValueError("flux records need block edges that are multiples of 8")
        f_sizes = np.array([int(np.prod(flux_record_shape(int(n)))) for n in edges], dtype=np.int64)
        flux_off = np.concatenate([[0], np.cumsum(f_sizes)[:-1]]).astype(np.int64)
        flat_flux = np.full(int(f_sizes.sum()), np.nan)
        flux_p = _dptr(flat_flux)
        flux_off_p = flux_off.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong))
    t0 = time.perf_counter()
    th = lib.oracle_advance_batch(
        _dptr(flat_in), _dptr(flat_out), nb,
        edges.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
        in_off.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
        out_off.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
        _dptr(dt_a), _dptr(dh_a), int(order), float(gamma), float(p_floor),
        flux_p, flux_off_p, ctypes.byref(fl), ctypes.byref(npy))
    t1 = time.perf_counter()
    if counts is not None:
        counts.seconds += t1 - t0
        counts.floored += fl.value
        counts.nonphysical += npy.value
        counts.threads = th
    outs = []
    for b in range(nb):
        n = int(edges[b])
        outs.append(flat_out[out_off[b]:out_off[b] + out_sizes[b]].reshape(NVAR, n, n, n))
    if not fluxes:
        return outs
    recs = [flat_flux[flux_off[b]:flux_off[b] + f_sizes[b]].reshape(flux_record_shape(int(edges[b])))
            for b in range(nb)]
    return outs, recs


def advance_blocks(blocks_in, order: int, dt, dh, gamma: float, p_floor: float = 0.0,
                   counts: Counts | None = None):
    """One step on an array of equal ghosted blocks, shape (B, 5, m, m, m)."""
    blocks_in = np.ascontiguousarray(blocks_in, dtype=np.float64)
    B = blocks_in.shape[0]
    n = blocks_in.shape[2] - 2 * GHOST
    if B == 0:
        return np.zeros((0, NVAR, n, n, n))
    outs = advance_ragged(list(blocks_in), order, dt, dh, gamma, p_floor, counts)
    return np.stack(outs)


# ---------------------------------------------------------------------------
# Eq. (CFL) and conservation sums
# ---------------------------------------------------------------------------

def max_signal_speed(u, gamma: float, p_floor: float = 0.0) -> float:
    """Max over cells of c_s + max(|v_x|, |v_y|, |v_z|) for u of shape (5, ...)."""
    lib = _load()
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(NVAR, -1)
    return lib.oracle_max_signal_speed(_dptr(u), u.shape[1], u.shape[1], gamma, p_floor)


def cons_sums(u, weight: float = 1.0):
    """Neumaier-compensated sum of each of the 5 planes of u, times ``weight``."""
    lib = _load()
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(NVAR, -1)
    out = np.zeros(NVAR)
    comp = ctypes.c_double(0.0)
    for k in range(NVAR):
        row = np.ascontiguousarray(u[k])
        out[k] = lib.oracle_compensated_sum(_dptr(row), row.size, weight, ctypes.byref(comp))
    return out


# ---------------------------------------------------------------------------
# periodic grid driver
# ---------------------------------------------------------------------------

def periodic_ghosted_blocks(grid, n: int):
    """Cut a periodic grid (5, Nz, Ny, Nx) into ghosted blocks of edge n.

    Ghost zones are filled by periodic copy.  Blocks are ordered with x
    fastest, then y, then z.  Returns an array (B, 5, n+6, n+6, n+6).
    """
    grid = np.asarray(grid, dtype=np.float64)
    _, Nz, Ny, Nx = grid.shape
    if Nx % n or Ny % n or Nz % n:
        raise ValueError("grid extents must be multiples of the block edge")
    g = GHOST
    if g > min(Nx, Ny, Nz):
        raise ValueError("ghost width exceeds the domain")
    padded = np.pad(grid, ((0, 0), (g, g), (g, g), (g, g)), mode="wrap")
    m = n + 2 * g
    out = []
    for bz in range(Nz // n):
        for by in range(Ny // n):
            for bx in range(Nx // n):
                out.append(padded[:, bz * n:bz * n + m, by * n:by * n + m, bx * n:bx * n + m])
    return np.ascontiguousarray(np.stack(out))


def assemble_blocks(blocks, shape):
    """Inverse of the block cut for interiors (B, 5, n, n, n) -> (5, Nz, Ny, Nx)."""
    _, Nz, Ny, Nx = shape
    n = blocks.shape[2]
    grid = np.zeros(shape)
    b = 0
    for bz in range(Nz // n):
        for by in range(Ny // n):
            for bx in range(Nx // n):
                grid[:, bz * n:(bz + 1) * n, by * n:(by + 1) * n, bx * n:(bx + 1) * n] = blocks[b]
                b += 1
    return grid


def step_periodic(grid, n: int, order: int, dt: float, dh: float, gamma: float,
                  p_floor: float = 0.0, counts: Counts | None = None):
    """One step (one directional triple) of a periodic grid cut into n^3 blocks."""
    blocks = periodic_ghosted_blocks(grid, n)
    out = advance_blocks(blocks, order, dt, dh, gamma, p_floor, counts)
    return assemble_blocks(out, grid.shape)


def run_periodic(grid, steps: int, cfl: float, dh: float, gamma: float, n: int = 8,
                 p_floor: float = 0.0, counts: Counts | None = None, record=None):
    """Step driver on a periodic grid.

    Step s uses the forward xyz triple when s is even and the backward zyx
    triple when s is odd (Sec. 2.2: the two sweeps of a pair share one time
    step).  The time step dt = cfl * dh / S, Eq. (CFL), is computed from the
    state before every even step and reused for the following odd step.
    ``record``, if given, is called as record(step, grid, dt) after each step.
    Returns the final grid and the list of time steps used.
    """
    dts = []
    dt = None
    for s in range(steps):
        if s % 2 == 0:
            S = max_signal_speed(grid, gamma, p_floor)
            dt = cfl * dh / S
        grid = step_periodic(grid, n, s % 2, dt, dh, gamma, p_floor, counts)
        dts.append(dt)
        if record is not None:
            record(s, grid, dt)
    return grid, dts
