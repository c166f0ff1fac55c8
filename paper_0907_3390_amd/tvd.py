"""Thin ctypes binding of libtvd (C ABI in ``include/tvd.h``).

Argument marshalling only: every step of the hot path runs in the HIP
kernels of ``libtvd.so``.  torch tensors supply device memory and streams;
their ``data_ptr()`` and the current HIP stream are passed through.  The
library is loaded on first use; if it has not been built, every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libtvd.so")

TVD_OK = 0
TVD_WARN_FLOORED = 1
TVD_ERR_INVALID_ARG = -1
TVD_ERR_UNSUPPORTED = -2
TVD_ERR_HIP = -3
TVD_ERR_NONPHYSICAL = -4
TVD_ERR_ALIAS = -5
TVD_ERR_STATE = -6
TVD_F32 = 1
TVD_F64 = 2
TVD_XYZ = 0
TVD_ZYX = 1
TVD_LAYOUT_GHOSTED = 0
TVD_LAYOUT_INTERIOR = 1
TVD_KERNEL_AUTO = 0
TVD_KERNEL_BATCHED = 1
TVD_KERNEL_PLAIN = 2
TVD_KERNEL_PERSISTENT = 3
TVD_STREAM_WHOLE_B = 16
TVD_STREAM_HALF_B = 32

EXPORTS = [
    "tvd_create", "tvd_destroy", "tvd_status_string", "tvd_last_error", "tvd_reserve",
    "tvd_patch_advance", "tvd_max_signal_speed", "tvd_dt_from_speed",
    "tvd_conservation_sums", "tvd_read_flags", "tvd_fill_ghosts",
    "tvd_variant_count", "tvd_variant_info", "tvd_set_variant", "tvd_patch_advance_gather",
    "tvd_autotune", "tvd_graph_begin", "tvd_graph_end", "tvd_graph_launch", "tvd_graph_destroy",
    "tvd_fill_ghosts_amr", "tvd_patch_advance_flux", "tvd_restrict", "tvd_flux_correct",
    "tvd_close_level", "tvd_poisson_sor", "tvd_gravity", "tvd_lerp",
    "tvd_patch_advance_stream", "tvd_patch_advance_stream_noalloc",
    "tvd_pipeline_stage_bytes", "tvd_patch_advance_host",
    "tvd_patch_advance_flux_gather", "tvd_fill_coarse_fine", "tvd_patch_advance_stream_flux",
]


class TvdError(RuntimeError):
    def __init__(self, status: int, text: str):
        super().__init__(f"libtvd status {status}: {text}")
        self.status = status


class tvd_chains(ctypes.Structure):
    _fields_ = [("n_chains", ctypes.c_int32), ("n_members", ctypes.c_int32),
                ("d_start", ctypes.c_void_p), ("d_blocks", ctypes.c_void_p)]


class tvd_host_pipeline(ctypes.Structure):
    _fields_ = [("n_streams", ctypes.c_int32), ("groups_per_stream", ctypes.c_int32),
                ("host_threads", ctypes.c_int32), ("concurrent", ctypes.c_int32),
                ("streams", ctypes.POINTER(ctypes.c_void_p)), ("h_stage", ctypes.c_void_p),
                ("d_stage", ctypes.c_void_p)]


class tvd_batch(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("n_blocks", ctypes.c_int32),
                ("edge", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("d_edge", ctypes.c_void_p), ("d_in_off", ctypes.c_void_p),
                ("d_out_off", ctypes.c_void_p), ("d_dt", ctypes.c_void_p),
                ("d_dh", ctypes.c_void_p), ("dt", ctypes.c_double), ("dh", ctypes.c_double)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libtvd.so and declare its signatures; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with `python -m paper_0907_3390_amd.build` "
            "(there is no fallback implementation)")
    lib = ctypes.CDLL(path)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    bp = ctypes.POINTER(tvd_batch)
    i64p = ctypes.POINTER(ctypes.c_int64)
    sig = {
        "tvd_create": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int]),
        "tvd_destroy": (ctypes.c_int, [vp]),
        "tvd_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "tvd_last_error": (ctypes.c_char_p, [vp]),
        "tvd_reserve": (ctypes.c_int, [vp, ctypes.c_int]),
        "tvd_patch_advance": (ctypes.c_int, [vp, bp, vp, vp, i32, dbl, dbl, i32, vp, vp, vp]),
        "tvd_patch_advance_gather": (ctypes.c_int, [vp, bp, vp, vp, vp, i32, dbl, dbl, i32, vp,
                                                    vp, vp]),
        "tvd_patch_advance_stream": (ctypes.c_int, [vp, bp, vp, ctypes.POINTER(tvd_chains), vp,
                                                    vp, i32, dbl, dbl, i32, vp, vp, vp]),
        "tvd_patch_advance_stream_noalloc": (ctypes.c_int, [vp, bp, vp,
                                                            ctypes.POINTER(tvd_chains), vp, vp,
                                                            i32, dbl, dbl, i32, vp, vp, vp]),
        "tvd_pipeline_stage_bytes": (ctypes.c_int, [i32, i32, ctypes.POINTER(tvd_host_pipeline),
                                                    i64p, i64p]),
        "tvd_patch_advance_host": (ctypes.c_int, [vp, bp, vp, vp, vp,
                                                  ctypes.POINTER(tvd_host_pipeline), i32, dbl, dbl,
                                                  ctypes.POINTER(ctypes.c_double)]),
        "tvd_max_signal_speed": (ctypes.c_int, [vp, bp, vp, i32, dbl, dbl, vp, vp]),
        "tvd_dt_from_speed": (ctypes.c_int, [vp, bp, vp, dbl, vp, vp]),
        "tvd_conservation_sums": (ctypes.c_int, [vp, bp, vp, i32, vp, vp]),
        "tvd_read_flags": (ctypes.c_int, [vp, i64p, i64p, vp]),
        "tvd_fill_ghosts": (ctypes.c_int, [vp, bp, vp, vp, vp, vp]),
        "tvd_fill_ghosts_amr": (ctypes.c_int, [vp, bp, vp, vp, vp, bp, vp, vp, vp, vp]),
        "tvd_patch_advance_flux": (ctypes.c_int, [vp, bp, vp, vp, vp, vp, dbl, i32, i32, dbl, dbl,
                                                  i32, vp, vp, vp]),
        "tvd_lerp": (ctypes.c_int, [vp, i32, ctypes.c_int64, vp, vp, vp, dbl, vp]),
        "tvd_patch_advance_flux_gather": (ctypes.c_int, [vp, bp, vp, i32, vp, vp, vp, vp, dbl,
                                                         i32, i32, dbl, dbl, i32, vp, vp, vp]),
        "tvd_fill_coarse_fine": (ctypes.c_int, [vp, bp, vp, i32, vp, bp, vp, vp, dbl, vp, vp,
                                                vp]),
        "tvd_patch_advance_stream_flux": (ctypes.c_int, [vp, bp, vp, i32, vp, vp, vp, vp, vp,
                                                         dbl, i32, i32, dbl, dbl, vp]),
        "tvd_restrict": (ctypes.c_int, [vp, bp, vp, bp, vp, vp, i32, vp]),
        "tvd_flux_correct": (ctypes.c_int, [vp, bp, vp, vp, vp, bp, vp, vp, vp,
                                            ctypes.POINTER(ctypes.c_int32), vp]),
        "tvd_close_level": (ctypes.c_int, [vp, bp, vp, vp, vp, bp, vp, vp, vp, vp, i32, vp, i32,
                                           vp, i32, vp]),
        "tvd_poisson_sor": (ctypes.c_int, [vp, i32, i32, vp, vp, vp, dbl, dbl, vp, dbl, i32, i32,
                                           dbl, vp, vp, vp]),
        "tvd_gravity": (ctypes.c_int, [vp, bp, vp, vp, vp]),
        "tvd_variant_count": (ctypes.c_int, []),
        "tvd_variant_info": (ctypes.c_int, [ctypes.c_int] + [ctypes.POINTER(ctypes.c_int32)] * 4),
        "tvd_set_variant": (ctypes.c_int, [vp, i32, i32, i32]),
        "tvd_graph_begin": (ctypes.c_int, [vp, vp]),
        "tvd_graph_end": (ctypes.c_int, [vp, vp, ctypes.POINTER(vp)]),
        "tvd_graph_launch": (ctypes.c_int, [vp, vp]),
        "tvd_graph_destroy": (ctypes.c_int, [vp]),
        "tvd_autotune": (ctypes.c_int, [vp, bp, vp, vp, vp, dbl, dbl, i32,
                                        ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_float)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return load().tvd_status_string(status).decode()


def _ptr(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Batch:
    """A tvd_batch plus the device arrays it points to (kept alive here)."""

    def __init__(self, dtype: int, n_blocks: int, edge: int = 8, dt: float = 0.0,
                 dh: float = 1.0, d_edge=None, d_in_off=None, d_out_off=None,
                 d_dt=None, d_dh=None):
        self.arrays = (d_edge, d_in_off, d_out_off, d_dt, d_dh)
        self.c = tvd_batch(dtype, n_blocks, edge if d_edge is None else 0, 0,
                           _ptr(d_edge), _ptr(d_in_off), _ptr(d_out_off), _ptr(d_dt),
                           _ptr(d_dh), dt, dh)

    @property
    def ref(self):
        return ctypes.byref(self.c)


class Chains:
    """A tvd_chains descriptor over two int32 device tensors (start, blocks)."""

    def __init__(self, start, blocks):
        self.start, self.blocks = start, blocks
        self.c = tvd_chains(int(start.numel()) - 1, int(blocks.numel()), _ptr(start),
                            _ptr(blocks))

    @property
    def ref(self):
        return ctypes.byref(self.c)


class HostPipeline:
    """A tvd_host_pipeline over caller-created streams and staging buffers
    (torch tensors: page-locked host memory and device memory), kept alive
    here."""

    def __init__(self, streams, groups_per_stream: int, host_threads: int, concurrent: bool,
                 h_stage=None, d_stage=None):
        self.streams = list(streams)
        self._sp = (ctypes.c_void_p * len(self.streams))(
            *[ctypes.c_void_p(st.cuda_stream) for st in self.streams])
        self.h_stage, self.d_stage = h_stage, d_stage
        self.c = tvd_host_pipeline(len(self.streams), groups_per_stream, host_threads,
                                   1 if concurrent else 0,
                                   ctypes.cast(self._sp, ctypes.POINTER(ctypes.c_void_p)),
                                   _host_ptr(h_stage), _ptr(d_stage))

    def stage_bytes(self, dtype: int, edge: int):
        """(host, device) staging bytes this pipeline needs for (dtype, edge)."""
        hb, db = ctypes.c_int64(), ctypes.c_int64()
        st = load().tvd_pipeline_stage_bytes(dtype, edge, ctypes.byref(self.c), ctypes.byref(hb),
                                             ctypes.byref(db))
        if st != TVD_OK:
            raise TvdError(st, "tvd_pipeline_stage_bytes: " + status_string(st))
        return hb.value, db.value

    def attach(self, h_stage, d_stage):
        self.h_stage, self.d_stage = h_stage, d_stage
        self.c.h_stage = _host_ptr(h_stage)
        self.c.d_stage = _ptr(d_stage)

    @property
    def ref(self):
        return ctypes.byref(self.c)


def _host_ptr(a):
    """Host address of a CPU torch tensor or numpy array (or None)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return ctypes.c_void_p(a.ctypes.data)
    return ctypes.c_void_p(a.data_ptr())


class Context:
    """Owns a tvd_ctx; methods carry the C entry points' names and arguments."""

    def __init__(self, device: int = 0):
        lib = load()
        h = ctypes.c_void_p()
        st = lib.tvd_create(ctypes.byref(h), device)
        if st != TVD_OK:
            raise TvdError(st, "tvd_create failed: " + status_string(st))
        self.h = h
        self.lib = lib

    def close(self):
        if self.h:
            self.lib.tvd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, allow_warn: bool = False):
        if st == TVD_OK or (allow_warn and st > 0):
            return st
        raise TvdError(st, self.lib.tvd_last_error(self.h).decode() or status_string(st))

    def last_error(self) -> str:
        return self.lib.tvd_last_error(self.h).decode()

    def tvd_reserve(self, n_blocks: int):
        return self._check(self.lib.tvd_reserve(self.h, n_blocks))

    def tvd_patch_advance(self, batch: Batch, u_in, u_out, sweep_order: int, gamma: float,
                          p_floor: float = 0.0, flags: int = TVD_KERNEL_AUTO, smax=None,
                          sums=None, stream=None, check: bool = True):
        st = self.lib.tvd_patch_advance(self.h, batch.ref, _ptr(u_in), _ptr(u_out),
                                        sweep_order, gamma, p_floor, flags, _ptr(smax),
                                        _ptr(sums), _stream(stream))
        return self._check(st) if check else st

    def tvd_patch_advance_gather(self, batch: Batch, nbr, u_in, u_out, sweep_order: int,
                                 gamma: float, p_floor: float = 0.0,
                                 flags: int = TVD_KERNEL_AUTO, smax=None, sums=None,
                                 stream=None, check: bool = True):
        st = self.lib.tvd_patch_advance_gather(self.h, batch.ref, _ptr(nbr), _ptr(u_in),
                                               _ptr(u_out), sweep_order, gamma, p_floor, flags,
                                               _ptr(smax), _ptr(sums), _stream(stream))
        return self._check(st) if check else st

    def tvd_patch_advance_stream(self, batch: Batch, nbr, chains: "Chains", u_in, u_out,
                                 sweep_order: int, gamma: float, p_floor: float = 0.0,
                                 flags: int = TVD_KERNEL_AUTO, smax=None, sums=None,
                                 stream=None, check: bool = True):
        st = self.lib.tvd_patch_advance_stream(self.h, batch.ref, _ptr(nbr), chains.ref,
                                               _ptr(u_in), _ptr(u_out), sweep_order, gamma,
                                               p_floor, flags, _ptr(smax), _ptr(sums),
                                               _stream(stream))
        return self._check(st) if check else st

    def tvd_patch_advance_stream_noalloc(self, batch: Batch, nbr, chains: "Chains", u_in, u_out,
                                         sweep_order: int, gamma: float, p_floor: float = 0.0,
                                         flags: int = TVD_KERNEL_AUTO, smax=None, sums=None,
                                         stream=None, check: bool = True):
        st = self.lib.tvd_patch_advance_stream_noalloc(self.h, batch.ref, _ptr(nbr), chains.ref,
                                                       _ptr(u_in), _ptr(u_out), sweep_order,
                                                       gamma, p_floor, flags, _ptr(smax),
                                                       _ptr(sums), _stream(stream))
        return self._check(st) if check else st

    def tvd_patch_advance_host(self, batch: Batch, nbr, u_in, u_out, pipe: HostPipeline,
                               sweep_order: int, gamma: float, p_floor: float = 0.0,
                               times: bool = False, check: bool = True):
        """Host arrays nbr (int32 [n][27]), u_in and u_out (numpy or CPU
        tensors).  Returns (status, times) with times a dict of ms or None."""
        t = (ctypes.c_double * 7)() if times else None
        st = self.lib.tvd_patch_advance_host(self.h, batch.ref, _host_ptr(nbr), _host_ptr(u_in),
                                             _host_ptr(u_out), pipe.ref, sweep_order, gamma,
                                             p_floor, t)
        if check:
            self._check(st)
        if t is None:
            return st, None
        keys = ("wall", "host_prepare", "host_close", "copy_down", "advance", "copy_up",
                "gpu_span")
        return st, {k: float(t[i]) for i, k in enumerate(keys)}

    def tvd_patch_advance_flux(self, batch: Batch, u_in, u_out, flux, flux_off, sweep_order: int,
                               gamma: float, p_floor: float = 0.0, flags: int = TVD_KERNEL_AUTO,
                               smax=None, sums=None, stream=None, check: bool = True,
                               flux_weight: float = 1.0, accumulate: int = 0):
        st = self.lib.tvd_patch_advance_flux(self.h, batch.ref, _ptr(u_in), _ptr(u_out),
                                             _ptr(flux), _ptr(flux_off), flux_weight, accumulate,
                                             sweep_order, gamma, p_floor, flags, _ptr(smax),
                                             _ptr(sums), _stream(stream))
        return self._check(st) if check else st

    def tvd_patch_advance_flux_gather(self, batch: Batch, nbr, n_sources: int, u_in, u_out, flux,
                                      flux_off, sweep_order: int, gamma: float,
                                      p_floor: float = 0.0, flags: int = TVD_KERNEL_AUTO,
                                      smax=None, sums=None, stream=None, check: bool = True,
                                      flux_weight: float = 1.0, accumulate: int = 0):
        st = self.lib.tvd_patch_advance_flux_gather(
            self.h, batch.ref, _ptr(nbr), n_sources, _ptr(u_in), _ptr(u_out), _ptr(flux),
            _ptr(flux_off), flux_weight, accumulate, sweep_order, gamma, p_floor, flags,
            _ptr(smax), _ptr(sums), _stream(stream))
        return self._check(st) if check else st

    def tvd_patch_advance_stream_flux(self, batch: Batch, nbr, n_sources: int, chains: "Chains",
                                      u_in, u_out, flux, flux_off, sweep_order: int,
                                      gamma: float, p_floor: float = 0.0,
                                      flux_weight: float = 1.0, accumulate: int = 0,
                                      stream=None, check: bool = True):
        st = self.lib.tvd_patch_advance_stream_flux(
            self.h, batch.ref, _ptr(nbr), n_sources, chains.ref, _ptr(u_in), _ptr(u_out),
            _ptr(flux), _ptr(flux_off), flux_weight, accumulate, sweep_order, gamma, p_floor,
            _stream(stream))
        return self._check(st) if check else st

    def tvd_fill_coarse_fine(self, fine: Batch, nbr, n_sources: int, fine_interior, coarse: Batch,
                             coarse_old, coarse_new, w: float, cnbr, corigin, stream=None,
                             check: bool = True):
        st = self.lib.tvd_fill_coarse_fine(self.h, fine.ref, _ptr(nbr), n_sources,
                                           _ptr(fine_interior), coarse.ref, _ptr(coarse_old),
                                           _ptr(coarse_new), w, _ptr(cnbr), _ptr(corigin),
                                           _stream(stream))
        return self._check(st) if check else st

    def tvd_lerp(self, dtype: int, n: int, a, b, out, w: float, stream=None, check: bool = True):
        st = self.lib.tvd_lerp(self.h, dtype, n, _ptr(a), _ptr(b), _ptr(out), w, _stream(stream))
        return self._check(st) if check else st

    def tvd_restrict(self, coarse: Batch, u_coarse, fine: Batch, u_fine, rows, stream=None,
                     check: bool = True):
        n = 0 if rows is None else int(rows.shape[0])
        st = self.lib.tvd_restrict(self.h, coarse.ref, _ptr(u_coarse), fine.ref, _ptr(u_fine),
                                   _ptr(rows), n, _stream(stream))
        return self._check(st) if check else st

    def tvd_flux_correct(self, coarse: Batch, u_coarse, coarse_flux, coarse_flux_off, fine: Batch,
                         fine_flux, fine_flux_off, rows, pass_count, stream=None,
                         check: bool = True):
        pc = (ctypes.c_int32 * 6)(*[int(v) for v in pass_count])
        st = self.lib.tvd_flux_correct(self.h, coarse.ref, _ptr(u_coarse), _ptr(coarse_flux),
                                       _ptr(coarse_flux_off), fine.ref, _ptr(fine_flux),
                                       _ptr(fine_flux_off), _ptr(rows), pc, _stream(stream))
        return self._check(st) if check else st

    def tvd_close_level(self, coarse: Batch, u_coarse, coarse_flux, coarse_flux_off, fine: Batch,
                        u_fine, fine_flux, fine_flux_off, restrict_rows, face_rows, face_start,
                        stream=None, check: bool = True):
        nr = 0 if restrict_rows is None else int(restrict_rows.shape[0])
        nf = 0 if face_rows is None else int(face_rows.shape[0])
        ng = 0 if face_start is None else int(face_start.shape[0]) - 1
        st = self.lib.tvd_close_level(self.h, coarse.ref, _ptr(u_coarse), _ptr(coarse_flux),
                                      _ptr(coarse_flux_off), fine.ref, _ptr(u_fine),
                                      _ptr(fine_flux), _ptr(fine_flux_off), _ptr(restrict_rows),
                                      nr, _ptr(face_rows), nf, _ptr(face_start), ng,
                                      _stream(stream))
        return self._check(st) if check else st

    def tvd_poisson_sor(self, dtype: int, n_groups: int, phi_in, rho, phi_out, G: float,
                        dh: float = 1.0, d_dh=None, omega: float = 0.0, min_iter: int = 0,
                        max_iter: int = 1000, tol: float = 0.0, iters=None, resid=None,
                        stream=None, check: bool = True):
        st = self.lib.tvd_poisson_sor(self.h, dtype, n_groups, _ptr(phi_in), _ptr(rho),
                                      _ptr(phi_out), G, dh, _ptr(d_dh), omega, min_iter, max_iter,
                                      tol, _ptr(iters), _ptr(resid), _stream(stream))
        return self._check(st) if check else st

    def tvd_gravity(self, batch: Batch, u, phi, stream=None, check: bool = True):
        st = self.lib.tvd_gravity(self.h, batch.ref, _ptr(u), _ptr(phi), _stream(stream))
        return self._check(st) if check else st

    def tvd_max_signal_speed(self, batch: Batch, u, layout: int, gamma: float, smax,
                             p_floor: float = 0.0, stream=None):
        return self._check(self.lib.tvd_max_signal_speed(
            self.h, batch.ref, _ptr(u), layout, gamma, p_floor, _ptr(smax), _stream(stream)))

    def tvd_dt_from_speed(self, batch: Batch, smax, cfl: float, dt_out, stream=None):
        return self._check(self.lib.tvd_dt_from_speed(
            self.h, batch.ref, _ptr(smax), cfl, _ptr(dt_out), _stream(stream)))

    def tvd_conservation_sums(self, batch: Batch, u, layout: int, sums, stream=None):
        return self._check(self.lib.tvd_conservation_sums(
            self.h, batch.ref, _ptr(u), layout, _ptr(sums), _stream(stream)))

    def tvd_set_variant(self, dtype: int, edge: int, index: int):
        return self._check(self.lib.tvd_set_variant(self.h, dtype, edge, index))

    def tvd_autotune(self, batch: Batch, nbr, u_in, u_out, gamma: float, p_floor: float = 0.0,
                     reps: int = 3):
        """Returns (chosen variant index, ms per xyz+zyx pair)."""
        idx = ctypes.c_int32(-1)
        ms = ctypes.c_float(0.0)
        self._check(self.lib.tvd_autotune(self.h, batch.ref, _ptr(nbr), _ptr(u_in), _ptr(u_out),
                                          gamma, p_floor, reps, ctypes.byref(idx),
                                          ctypes.byref(ms)))
        return idx.value, ms.value

    def tvd_graph_begin(self, stream):
        return self._check(self.lib.tvd_graph_begin(self.h, _stream(stream)))

    def tvd_graph_end(self, stream):
        g = ctypes.c_void_p()
        self._check(self.lib.tvd_graph_end(self.h, _stream(stream), ctypes.byref(g)))
        return Graph(self.lib, g)

    def tvd_read_flags(self, stream=None):
        a = ctypes.c_int64(0)
        b = ctypes.c_int64(0)
        st = self.lib.tvd_read_flags(self.h, ctypes.byref(a), ctypes.byref(b), _stream(stream))
        if st < 0 and st != TVD_ERR_NONPHYSICAL:
            self._check(st)
        return st, a.value, b.value

    def tvd_fill_ghosts(self, batch: Batch, nbr, interior, ghosted, stream=None):
        return self._check(self.lib.tvd_fill_ghosts(
            self.h, batch.ref, _ptr(nbr), _ptr(interior), _ptr(ghosted), _stream(stream)))

    def tvd_fill_ghosts_amr(self, fine: Batch, nbr, fine_interior, fine_ghosted, coarse: Batch,
                            coarse_interior, cnbr, corigin, stream=None):
        return self._check(self.lib.tvd_fill_ghosts_amr(
            self.h, fine.ref, _ptr(nbr), _ptr(fine_interior), _ptr(fine_ghosted), coarse.ref,
            _ptr(coarse_interior), _ptr(cnbr), _ptr(corigin), _stream(stream)))


class Graph:
    """A recorded step sequence (tvd_graph); replay() launches it."""

    def __init__(self, lib, handle):
        self.lib = lib
        self.h = handle

    def tvd_graph_launch(self, stream=None):
        st = self.lib.tvd_graph_launch(self.h, _stream(stream))
        if st == TVD_ERR_STATE:
            raise TvdError(st, "graph retired: the workspace was replaced by tvd_reserve or "
                               "the context destroyed after the capture")
        if st != TVD_OK:
            raise TvdError(st, "tvd_graph_launch failed")

    replay = tvd_graph_launch

    def close(self):
        if self.h:
            self.lib.tvd_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def variants():
    """[(index, edge, threads, lds_pad, split)] of the compiled batched-kernel variants."""
    lib = load()
    out = []
    for i in range(lib.tvd_variant_count()):
        v = [ctypes.c_int32() for _ in range(4)]
        lib.tvd_variant_info(i, *[ctypes.byref(x) for x in v])
        out.append((i,) + tuple(x.value for x in v))
    return out


def exported_symbols(path: str = LIB_PATH):
    """Names from EXPORTS that the built library exports (no device needed)."""
    lib = ctypes.CDLL(path)
    return [n for n in EXPORTS if hasattr(lib, n)]


def dtype_code(torch_dtype) -> int:
    import torch
    if torch_dtype == torch.float32:
        return TVD_F32
    if torch_dtype == torch.float64:
        return TVD_F64
    raise ValueError("state tensors must be float32 or float64")


def as_numpy(t) -> np.ndarray:
    return t.detach().cpu().numpy()
