"""ctypes binding of the C ABI in ``include/sps.h`` (argument marshalling only).

Every function has the name of the C entry point it wraps and forwards its
arguments: torch tensors become device pointers, pitches and the current HIP
stream; host arrays become pointers.  All arithmetic runs in the HIP library
``_lib/libsps.so``; if that library is missing this module raises instead of
falling back to anything else.

torch is imported first on purpose: the library then binds to the HIP
runtime torch already loaded, so device pointers and streams are shared.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Sequence

import numpy as np
import torch

from .build import LIB_PATH

SPS_ZERO_PAD = 1

_STATUS = {0: "SPS_OK", 1: "SPS_ERR_INVALID_ARG", 2: "SPS_ERR_RANGE", 3: "SPS_ERR_NOMEM",
           4: "SPS_ERR_DEVICE", 5: "SPS_ERR_OVERFLOW", 6: "SPS_ERR_TRUNCATED"}


class SpsError(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        self.status = status
        self.name = _STATUS.get(status, str(status))
        super().__init__(f"{func}: {self.name}: {msg}")


class sps_obs_desc(ctypes.Structure):
    _fields_ = [("nchan", ctypes.c_int32), ("freq_mhz", ctypes.POINTER(ctypes.c_double)),
                ("fref_mhz", ctypes.c_double), ("tsamp_s", ctypes.c_double),
                ("ndm", ctypes.c_int32), ("dm", ctypes.POINTER(ctypes.c_double))]


class sps_candidate(ctypes.Structure):
    _fields_ = [("dm_idx", ctypes.c_int32), ("width", ctypes.c_int32), ("t_idx", ctypes.c_int64),
                ("snr", ctypes.c_float), ("reserved", ctypes.c_float), ("dm", ctypes.c_double),
                ("toa_s", ctypes.c_double)]


class sps_subband_desc(ctypes.Structure):
    _fields_ = [("nchan", ctypes.c_int32), ("freq_mhz", ctypes.POINTER(ctypes.c_double)),
                ("fref_mhz", ctypes.c_double), ("tsamp_s", ctypes.c_double),
                ("ndm", ctypes.c_int32), ("dm_lo", ctypes.c_double), ("dm_step", ctypes.c_double),
                ("n0", ctypes.c_int32), ("nsub", ctypes.c_int32)]


class sps_beam(ctypes.Structure):
    _fields_ = [("X", ctypes.c_void_p), ("pitch", ctypes.c_int64), ("nsamp_in", ctypes.c_int64),
                ("Y", ctypes.c_void_p), ("nout", ctypes.c_int64), ("snr", ctypes.c_void_p),
                ("best_w", ctypes.c_void_p), ("stats", ctypes.c_void_p)]


class sps_detect_params(ctypes.Structure):
    _fields_ = [("threshold", ctypes.c_float), ("tile_dm", ctypes.c_int32),
                ("tile_t", ctypes.c_int64), ("nms_dm", ctypes.c_int32), ("nms_t", ctypes.c_int64)]


class sps_feed(ctypes.Structure):
    _fields_ = [("host", ctypes.c_void_p), ("src_pitch", ctypes.c_int64), ("nsrc", ctypes.c_int32),
                ("first", ctypes.c_int32)]


class sps_chunk_record(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_int32), ("worker", ctypes.c_int32), ("index", ctypes.c_int64),
                ("arrival_s", ctypes.c_double), ("start_s", ctypes.c_double),
                ("upload_s", ctypes.c_double), ("compute_s", ctypes.c_double),
                ("end_s", ctypes.c_double), ("n_cand", ctypes.c_int32), ("status", ctypes.c_int32),
                ("n_cnn", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class sps_cnn_candidate(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("cell_dm", ctypes.c_int32), ("cell_t", ctypes.c_int32),
                ("prob", ctypes.c_float), ("row", ctypes.c_float), ("col", ctypes.c_float)]


_lib = None


def library() -> ctypes.CDLL:
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        P, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
        lib.sps_plan_create.argtypes = [ctypes.POINTER(sps_obs_desc), ctypes.POINTER(P)]
        lib.sps_plan_destroy.argtypes = [P]
        lib.sps_plan_delays.argtypes = [P, P, ctypes.POINTER(i32)]
        lib.sps_dedisperse.argtypes = [P, P, i64, i64, P, i64, u32, P]
        lib.sps_boxcar_snr.argtypes = [P, P, i64, P, i32, P, P, P, P]
        lib.sps_detect.argtypes = [P, P, P, i64, P, i32, ctypes.POINTER(sps_detect_params),
                                   ctypes.POINTER(sps_candidate), i32, ctypes.POINTER(i32), P]
        lib.sps_boxcar_pool.argtypes = [P, P, i64, P, i32, P, ctypes.c_float, P,
                                        ctypes.POINTER(i64), P]
        lib.sps_batch_set_tiles.argtypes = [P, P, ctypes.c_float, ctypes.POINTER(i64)]
        lib.sps_search.argtypes = [P, P, i64, P, i32, P, P, P, ctypes.POINTER(sps_detect_params),
                                   ctypes.POINTER(sps_candidate), i32, ctypes.POINTER(i32), P]
        lib.sps_detect_noalloc.argtypes = [P, P, P, i64, P, i32,
                                           ctypes.POINTER(sps_detect_params),
                                           ctypes.POINTER(sps_candidate), i32,
                                           ctypes.POINTER(i32), P]
        lib.sps_plan_set_tiling.argtypes = [P, i32, i32, i32, i32, i32]
        lib.sps_plan_get_tiling.argtypes = [P] + [ctypes.POINTER(i32)] * 6
        lib.sps_subband_plan_create.argtypes = [ctypes.POINTER(sps_subband_desc), ctypes.POINTER(P)]
        lib.sps_subband_tables.argtypes = [P, P, P, P, ctypes.POINTER(i32)]
        lib.sps_dedisperse_subband.argtypes = [P, P, i64, i64, P, i64, u32, P]
        lib.sps_zero_dm.argtypes = [P, i64, i64, i32, P, i64, P]
        lib.sps_downsample_sqrt.argtypes = [P, i64, i64, i32, i32, P, i64, P]
        lib.sps_batch_create.argtypes = [P, i32, ctypes.POINTER(sps_beam), P, i32,
                                         ctypes.POINTER(sps_detect_params), u32, ctypes.POINTER(P)]
        lib.sps_batch_destroy.argtypes = [P]
        lib.sps_batch_enqueue.argtypes = [P, P]
        lib.sps_batch_launch_graph.argtypes = [P, P]
        lib.sps_batch_candidates.argtypes = [P, i32, ctypes.POINTER(sps_candidate), i32,
                                             ctypes.POINTER(i32), P]
        lib.sps_batch_candidates_all.argtypes = [P, ctypes.POINTER(sps_candidate), i32,
                                                 ctypes.POINTER(i32), P]
        lib.sps_plan_autotune.argtypes = [P, i64, i32, P, P, ctypes.POINTER(i32)]
        lib.sps_batch_autotune.argtypes = [P, i32, P, P, ctypes.POINTER(i32)]
        lib.sps_tiling_count.argtypes = []
        lib.sps_tiling_count.restype = i32
        lib.sps_tiling_describe.argtypes = [i32] + [ctypes.POINTER(i32)] * 5
        lib.sps_probe_peaks.argtypes = [i32, ctypes.POINTER(ctypes.c_double), i32]
        lib.sps_server_create.argtypes = [i64, i32, ctypes.POINTER(P)]
        lib.sps_server_destroy.argtypes = [P]
        lib.sps_server_add_stream.argtypes = [P, ctypes.POINTER(sps_obs_desc), P, i32,
                                              ctypes.POINTER(sps_detect_params), i64,
                                              ctypes.POINTER(i32)]
        lib.sps_server_memory.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64)]
        lib.sps_server_stream_info.argtypes = [P, i32, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                               ctypes.POINTER(ctypes.c_double)]
        lib.sps_server_push.argtypes = [P, i32, P, i64, P, ctypes.POINTER(sps_candidate), i32,
                                        ctypes.POINTER(i32), ctypes.POINTER(i32)]
        lib.sps_server_set_detector.argtypes = [P, P, ctypes.c_float, ctypes.c_float]
        lib.sps_server_run.argtypes = [P, ctypes.POINTER(sps_feed), ctypes.c_double,
                                       ctypes.c_double, ctypes.POINTER(sps_chunk_record), i32,
                                       ctypes.POINTER(i32)]
        lib.sps_cnn_param_count.argtypes = []
        lib.sps_cnn_param_count.restype = i64
        lib.sps_cnn_create.argtypes = [i32, ctypes.POINTER(P)]
        lib.sps_cnn_destroy.argtypes = [P]
        for f in ("sps_cnn_set_params", "sps_cnn_get_params", "sps_cnn_set_grads",
                  "sps_cnn_get_grads"):
            getattr(lib, f).argtypes = [P, P]
        lib.sps_cnn_activations.argtypes = [P, i32, i32, P]
        lib.sps_cnn_set_loss_weights.argtypes = [P, ctypes.c_float, ctypes.c_float]
        lib.sps_cnn_signals.argtypes = [P, i32, i32, P]
        lib.sps_cnn_pool_tiles.argtypes = [P, i64, i32, i64, ctypes.c_float, P, P]
        lib.sps_cnn_pool_tile_grid.argtypes = [P, i64, i32, i64, ctypes.c_float, P,
                                               ctypes.POINTER(i64), P]
        lib.sps_cnn_max_batch.argtypes = [P]
        lib.sps_cnn_max_batch.restype = i32
        lib.sps_cnn_forward.argtypes = [P, P, i32, P, P]
        lib.sps_cnn_infer.argtypes = [P, P, i32, P, P]
        lib.sps_cnn_loss_grad.argtypes = [P, P, P, i32, P, P]
        lib.sps_cnn_adam.argtypes = [P, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                     ctypes.c_float, P]
        lib.sps_cnn_train_step.argtypes = [P, P, P, i32, ctypes.c_float, P, P]
        lib.sps_cnn_detect.argtypes = [P, P, i32, ctypes.c_float,
                                       ctypes.POINTER(sps_cnn_candidate), i32,
                                       ctypes.POINTER(i32), P]
        for f in ("sps_cnn_create", "sps_cnn_destroy", "sps_cnn_set_params", "sps_cnn_get_params",
                  "sps_cnn_set_grads", "sps_cnn_get_grads", "sps_cnn_activations", "sps_cnn_signals",
                  "sps_cnn_set_loss_weights",
                  "sps_cnn_pool_tiles", "sps_cnn_pool_tile_grid", "sps_cnn_forward", "sps_cnn_infer", "sps_cnn_loss_grad", "sps_cnn_adam",
                  "sps_cnn_train_step", "sps_cnn_detect"):
            getattr(lib, f).restype = ctypes.c_int
        for f in ("sps_server_create", "sps_server_destroy", "sps_server_add_stream",
                  "sps_server_memory", "sps_server_stream_info", "sps_server_push",
                  "sps_server_run", "sps_server_set_detector"):
            getattr(lib, f).restype = ctypes.c_int
        for f in ("sps_plan_create", "sps_plan_destroy", "sps_plan_delays", "sps_dedisperse",
                  "sps_boxcar_snr", "sps_search", "sps_boxcar_pool", "sps_batch_set_tiles",
                  "sps_detect", "sps_detect_noalloc",
                  "sps_plan_set_tiling",
                  "sps_plan_get_tiling",
                  "sps_subband_plan_create", "sps_subband_tables", "sps_dedisperse_subband",
                  "sps_zero_dm", "sps_downsample_sqrt", "sps_batch_create", "sps_batch_destroy",
                  "sps_batch_enqueue", "sps_batch_launch_graph", "sps_batch_candidates",
                  "sps_batch_candidates_all", "sps_plan_autotune", "sps_batch_autotune", "sps_tiling_describe",
                  "sps_probe_peaks"):
            getattr(lib, f).restype = ctypes.c_int
        lib.sps_last_error.argtypes = []
        lib.sps_last_error.restype = ctypes.c_char_p
        _lib = lib
    return _lib


def header_functions() -> list:
    """Names of the functions include/sps.h declares."""
    hdr = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "include", "sps.h")
    text = open(hdr).read()
    return sorted(set(re.findall(r"^\s*(?:sps_status|const char \*|int32_t|int64_t)\s*(sps_\w+)\s*\(",
                                 text, re.M)))


def sps_last_error() -> str:
    return library().sps_last_error().decode()


def _check(rc: int, func: str) -> None:
    if rc != 0:
        raise SpsError(rc, func, sps_last_error())


def _stream(stream) -> Optional[int]:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _dev(t: torch.Tensor, dtype, name: str) -> int:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != dtype:
        raise TypeError(f"{name} must be a {dtype} tensor on a GPU")
    return t.data_ptr()


def _dev_or_none(t: Optional[torch.Tensor], dtype, name: str) -> Optional[int]:
    return None if t is None else _dev(t, dtype, name)


class Plan:
    """Owns an sps_plan handle; closed explicitly or when garbage collected."""

    def __init__(self, handle: int, nchan: int, ndm: int):
        self.handle = handle
        self.nchan = nchan
        self.ndm = ndm

    def close(self) -> None:
        if self.handle:
            sps_plan_destroy(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def sps_plan_create(freq_mhz: Sequence[float], fref_mhz: float, tsamp_s: float,
                    dm: Sequence[float]) -> Plan:
    f = np.ascontiguousarray(freq_mhz, dtype=np.float64)
    m = np.ascontiguousarray(dm, dtype=np.float64)
    desc = sps_obs_desc(f.size, f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(fref_mhz),
                        float(tsamp_s), m.size, m.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    h = ctypes.c_void_p()
    _check(library().sps_plan_create(ctypes.byref(desc), ctypes.byref(h)), "sps_plan_create")
    return Plan(h.value, f.size, m.size)


def sps_plan_destroy(plan: Plan) -> None:
    h, plan.handle = plan.handle, None
    if h:
        _check(library().sps_plan_destroy(h), "sps_plan_destroy")


def sps_plan_delays(plan: Plan):
    """(delay table int32 [ndm][nchan], max delay)."""
    D = np.empty((plan.ndm, plan.nchan), dtype=np.int32)
    mx = ctypes.c_int32()
    _check(library().sps_plan_delays(plan.handle, D.ctypes.data, ctypes.byref(mx)),
           "sps_plan_delays")
    return D, int(mx.value)


def sps_plan_set_tiling(plan: Plan, m: int, dpw: int, nw: int, cs: int,
                        waves_per_eu: int = 0) -> None:
    _check(library().sps_plan_set_tiling(plan.handle, m, dpw, nw, cs, waves_per_eu),
           "sps_plan_set_tiling")


def sps_plan_get_tiling(plan: Plan) -> dict:
    v = [ctypes.c_int32() for _ in range(6)]
    _check(library().sps_plan_get_tiling(plan.handle, *[ctypes.byref(x) for x in v]),
           "sps_plan_get_tiling")
    return dict(zip(("m", "dpw", "nw", "cs", "waves_per_eu", "lds_bytes"), (x.value for x in v)))


def sps_dedisperse(plan: Plan, X: torch.Tensor, nsamp_in: int, Y: torch.Tensor, nout: int,
                   flags: int = 0, stream=None) -> None:
    if X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be [nchan][pitch] with unit sample stride")
    if Y.dim() != 2 or not Y.is_contiguous():
        raise ValueError("Y must be a contiguous [ndm][nout] tensor")
    xp = _dev(X, torch.uint8, "X")
    yp = _dev(Y, torch.int32, "Y") if Y.dtype == torch.int32 else _dev(Y, torch.uint32, "Y")
    _check(library().sps_dedisperse(plan.handle, xp, X.stride(0), int(nsamp_in), yp, int(nout),
                                    int(flags), _stream(stream)), "sps_dedisperse")


def sps_boxcar_snr(plan: Plan, Y: torch.Tensor, nout: int, widths: Sequence[int],
                   snr: torch.Tensor, best_w: torch.Tensor, stats: Optional[torch.Tensor] = None,
                   stream=None) -> None:
    w = np.ascontiguousarray(widths, dtype=np.int32)
    yp = _dev(Y, torch.int32, "Y") if Y.dtype == torch.int32 else _dev(Y, torch.uint32, "Y")
    sp = _dev(stats, torch.int32, "stats") if stats is not None else None
    _check(library().sps_boxcar_snr(plan.handle, yp, int(nout), w.ctypes.data, w.size,
                                    _dev(snr, torch.float32, "snr"),
                                    _dev(best_w, torch.uint8, "best_w"), sp, _stream(stream)),
           "sps_boxcar_snr")


def sps_search(plan: Plan, Y: torch.Tensor, nout: int, widths: Sequence[int],
               snr: Optional[torch.Tensor], best_w: Optional[torch.Tensor],
               stats: Optional[torch.Tensor], threshold: float,
               tile_dm: int, tile_t: int, nms_dm: int, nms_t: int, cap: int = 4096,
               stream=None, allow_truncated: bool = False):
    """Statistics, boxcar S/N and detection in one call; returns (candidates, number found).
    snr and best_w None together: no planes are written."""
    w = np.ascontiguousarray(widths, dtype=np.int32)
    yp = _dev(Y, torch.int32, "Y") if Y.dtype == torch.int32 else _dev(Y, torch.uint32, "Y")
    sp = _dev(stats, torch.int32, "stats") if stats is not None else None
    prm = sps_detect_params(float(threshold), int(tile_dm), int(tile_t), int(nms_dm), int(nms_t))
    out = (sps_candidate * max(cap, 1))()
    n = ctypes.c_int32()
    rc = library().sps_search(plan.handle, yp, int(nout), w.ctypes.data, w.size,
                              _dev_or_none(snr, torch.float32, "snr"),
                              _dev_or_none(best_w, torch.uint8, "best_w"),
                              sp, ctypes.byref(prm), out, int(cap), ctypes.byref(n),
                              _stream(stream))
    if not (rc == 6 and allow_truncated):
        _check(rc, "sps_search")
    k = min(int(n.value), cap)
    arr = np.frombuffer(out, dtype=CANDIDATE_DTYPE)[:k].copy()
    return arr, int(n.value)


def sps_boxcar_pool(plan: Plan, Y: torch.Tensor, nout: int, widths: Sequence[int],
                    stats: Optional[torch.Tensor], scale: float, tiles: torch.Tensor,
                    stream=None) -> int:
    """Statistics and boxcar straight into bf16 detector tiles; returns the tile count."""
    w = np.ascontiguousarray(widths, dtype=np.int32)
    yp = _dev(Y, torch.int32, "Y") if Y.dtype == torch.int32 else _dev(Y, torch.uint32, "Y")
    sp = _dev(stats, torch.int32, "stats") if stats is not None else None
    n = ctypes.c_int64()
    _check(library().sps_boxcar_pool(plan.handle, yp, int(nout), w.ctypes.data, w.size, sp,
                                     float(scale), _tiles_ptr(tiles), ctypes.byref(n),
                                     _stream(stream)), "sps_boxcar_pool")
    return int(n.value)


CANDIDATE_DTYPE = np.dtype([("dm_idx", np.int32), ("width", np.int32), ("t_idx", np.int64),
                            ("snr", np.float32), ("reserved", np.float32), ("dm", np.float64),
                            ("toa_s", np.float64)])


def sps_detect(plan: Plan, snr: torch.Tensor, best_w: torch.Tensor, nout: int,
               widths: Sequence[int], threshold: float, tile_dm: int, tile_t: int, nms_dm: int,
               nms_t: int, cap: int = 4096, stream=None, allow_truncated: bool = False):
    """Returns (structured array of candidates, number found)."""
    return _detect("sps_detect", plan, snr, best_w, nout, widths, threshold, tile_dm, tile_t,
                   nms_dm, nms_t, cap, stream, allow_truncated)


def sps_detect_noalloc(plan: Plan, snr: torch.Tensor, best_w: torch.Tensor, nout: int,
                       widths: Sequence[int], threshold: float, tile_dm: int, tile_t: int,
                       nms_dm: int, nms_t: int, cap: int = 4096, stream=None,
                       allow_truncated: bool = False):
    """sps_detect on the library's fixed device scratch (no device allocation)."""
    return _detect("sps_detect_noalloc", plan, snr, best_w, nout, widths, threshold, tile_dm,
                   tile_t, nms_dm, nms_t, cap, stream, allow_truncated)


def _detect(name, plan, snr, best_w, nout, widths, threshold, tile_dm, tile_t, nms_dm, nms_t,
            cap, stream, allow_truncated):
    w = np.ascontiguousarray(widths, dtype=np.int32)
    prm = sps_detect_params(float(threshold), int(tile_dm), int(tile_t), int(nms_dm), int(nms_t))
    out = (sps_candidate * max(cap, 1))()
    n = ctypes.c_int32()
    rc = getattr(library(), name)(plan.handle, _dev(snr, torch.float32, "snr"),
                              _dev(best_w, torch.uint8, "best_w"), int(nout), w.ctypes.data,
                              w.size, ctypes.byref(prm), out, int(cap), ctypes.byref(n),
                              _stream(stream))
    if not (rc == 6 and allow_truncated):
        _check(rc, name)
    k = min(int(n.value), cap)
    arr = np.frombuffer(out, dtype=CANDIDATE_DTYPE)[:k].copy()
    return arr, int(n.value)


def sps_subband_plan_create(freq_mhz: Sequence[float], fref_mhz: float, tsamp_s: float, ndm: int,
                            dm_lo: float, dm_step: float, n0: int, nsub: int) -> Plan:
    f = np.ascontiguousarray(freq_mhz, dtype=np.float64)
    desc = sps_subband_desc(f.size, f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                            float(fref_mhz), float(tsamp_s), int(ndm), float(dm_lo),
                            float(dm_step), int(n0), int(nsub))
    h = ctypes.c_void_p()
    _check(library().sps_subband_plan_create(ctypes.byref(desc), ctypes.byref(h)),
           "sps_subband_plan_create")
    plan = Plan(h.value, f.size, int(ndm))
    plan.n0, plan.nsub = int(n0), int(nsub)
    return plan


def sps_subband_tables(plan: Plan):
    """(coarse delays [ceil(ndm/n0)][nchan], residuals [ndm][nsub], F_s [nsub], max delay)."""
    nc = (plan.ndm + plan.n0 - 1) // plan.n0
    Dc = np.empty((nc, plan.nchan), dtype=np.int32)
    R = np.empty((plan.ndm, plan.nsub), dtype=np.int32)
    F = np.empty(plan.nsub, dtype=np.float64)
    mx = ctypes.c_int32()
    _check(library().sps_subband_tables(plan.handle, Dc.ctypes.data, R.ctypes.data,
                                        F.ctypes.data, ctypes.byref(mx)), "sps_subband_tables")
    return Dc, R, F, int(mx.value)


def sps_dedisperse_subband(plan: Plan, X: torch.Tensor, nsamp_in: int, Y: torch.Tensor, nout: int,
                           flags: int = 0, stream=None) -> None:
    if X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be [nchan][pitch] with unit sample stride")
    if Y.dim() != 2 or not Y.is_contiguous():
        raise ValueError("Y must be a contiguous [ndm][nout] tensor")
    xp = _dev(X, torch.uint8, "X")
    yp = _dev(Y, torch.int32, "Y") if Y.dtype == torch.int32 else _dev(Y, torch.uint32, "Y")
    _check(library().sps_dedisperse_subband(plan.handle, xp, X.stride(0), int(nsamp_in), yp,
                                            int(nout), int(flags), _stream(stream)),
           "sps_dedisperse_subband")


def sps_zero_dm(X: torch.Tensor, nsamp: int, Xo: torch.Tensor, stream=None) -> None:
    if X.stride(1) != 1 or Xo.stride(1) != 1 or X.shape[0] != Xo.shape[0]:
        raise ValueError("X and Xo must be [nchan][pitch] with unit sample stride")
    _check(library().sps_zero_dm(_dev(X, torch.uint8, "X"), X.stride(0), int(nsamp), X.shape[0],
                                 _dev(Xo, torch.uint8, "Xo"), Xo.stride(0), _stream(stream)),
           "sps_zero_dm")


def sps_downsample_sqrt(X: torch.Tensor, nsamp: int, factor: int, Xo: torch.Tensor,
                        stream=None) -> None:
    if X.stride(1) != 1 or Xo.stride(1) != 1 or X.shape[0] != Xo.shape[0]:
        raise ValueError("X and Xo must be [nchan][pitch] with unit sample stride")
    _check(library().sps_downsample_sqrt(_dev(X, torch.uint8, "X"), X.stride(0), int(nsamp),
                                         X.shape[0], int(factor), _dev(Xo, torch.uint8, "Xo"),
                                         Xo.stride(0), _stream(stream)), "sps_downsample_sqrt")


class Batch:
    """Owns an sps_batch handle and keeps its plan and tensors alive."""

    def __init__(self, handle, plan, keep, widths):
        self.handle, self.plan, self._keep, self.widths = handle, plan, keep, widths
        self.nbeams = len(keep)
        self._all_out = None  # sps_batch_candidates_all's record array, reused per cap

    def close(self) -> None:
        if self.handle:
            sps_batch_destroy(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def sps_batch_create(plan: Plan, beams: Sequence[dict], widths: Sequence[int], threshold: float,
                     tile_dm: int, tile_t: int, nms_dm: int, nms_t: int, flags: int = 0) -> Batch:
    """beams: dicts with tensors X, Y, snr, best_w, stats and ints nsamp_in, nout; snr and
    best_w may be None (in every beam): no planes are written."""
    arr = (sps_beam * len(beams))()
    keep = []
    for i, b in enumerate(beams):
        X, Y = b["X"], b["Y"]
        if X.dim() != 2 or X.stride(1) != 1:
            raise ValueError("X must be [nchan][pitch] with unit sample stride")
        yp = _dev(Y, torch.int32, "Y") if Y.dtype == torch.int32 else _dev(Y, torch.uint32, "Y")
        arr[i] = sps_beam(_dev(X, torch.uint8, "X"), X.stride(0), int(b["nsamp_in"]), yp,
                          int(b["nout"]), _dev_or_none(b.get("snr"), torch.float32, "snr"),
                          _dev_or_none(b.get("best_w"), torch.uint8, "best_w"),
                          _dev(b["stats"], torch.int32, "stats"))
        keep.append(b)
    w = np.ascontiguousarray(widths, dtype=np.int32)
    prm = sps_detect_params(float(threshold), int(tile_dm), int(tile_t), int(nms_dm), int(nms_t))
    h = ctypes.c_void_p()
    _check(library().sps_batch_create(plan.handle, len(beams), arr, w.ctypes.data, w.size,
                                      ctypes.byref(prm), int(flags), ctypes.byref(h)),
           "sps_batch_create")
    return Batch(h.value, plan, keep, [int(x) for x in w])


def sps_batch_destroy(batch: Batch) -> None:
    h, batch.handle = batch.handle, None
    if h:
        _check(library().sps_batch_destroy(h), "sps_batch_destroy")


def sps_batch_enqueue(batch: Batch, stream=None) -> None:
    _check(library().sps_batch_enqueue(batch.handle, _stream(stream)), "sps_batch_enqueue")


def sps_batch_launch_graph(batch: Batch, stream) -> None:
    _check(library().sps_batch_launch_graph(batch.handle, _stream(stream)), "sps_batch_launch_graph")


def sps_batch_set_tiles(batch: Batch, tiles: Optional[torch.Tensor], scale: float = 0.0) -> int:
    """Tile mode (tiles a [n][256][512] 16-bit tensor) or search mode (None);
    returns the batch's tile count."""
    n = ctypes.c_int64()
    tp = _tiles_ptr(tiles) if tiles is not None else None
    _check(library().sps_batch_set_tiles(batch.handle, tp, float(scale), ctypes.byref(n)),
           "sps_batch_set_tiles")
    batch._tiles = tiles  # kept alive while the batch writes into it
    return int(n.value)


def sps_batch_candidates(batch: Batch, beam: int, cap: int = 4096, stream=None,
                         allow_truncated: bool = False):
    out = (sps_candidate * max(cap, 1))()
    n = ctypes.c_int32()
    rc = library().sps_batch_candidates(batch.handle, int(beam), out, int(cap), ctypes.byref(n),
                                        _stream(stream))
    if not (rc == 6 and allow_truncated):
        _check(rc, "sps_batch_candidates")
    k = min(int(n.value), cap)
    arr = np.frombuffer(out, dtype=CANDIDATE_DTYPE)[:k].copy()
    return arr, int(n.value)


def sps_batch_candidates_all(batch: Batch, cap: int = 4096, stream=None,
                             allow_truncated: bool = False):
    """Every beam's candidates in one call: a list of (candidates, number found) per beam."""
    nb = batch.nbeams
    if batch._all_out is None or len(batch._all_out) != max(nb * cap, 1):
        batch._all_out = (sps_candidate * max(nb * cap, 1))()
    out = batch._all_out  # every record returned is copied out below
    n = (ctypes.c_int32 * nb)()
    rc = library().sps_batch_candidates_all(batch.handle, out, int(cap), n, _stream(stream))
    if not (rc == 6 and allow_truncated):
        _check(rc, "sps_batch_candidates_all")
    view = np.frombuffer(out, dtype=CANDIDATE_DTYPE)  # no copy of the whole array
    return [(view[b * cap:b * cap + min(int(n[b]), cap)].copy(), int(n[b])) for b in range(nb)]


def sps_tiling_count() -> int:
    return int(library().sps_tiling_count())


def sps_tiling_describe(index: int) -> dict:
    v = [ctypes.c_int32() for _ in range(5)]
    _check(library().sps_tiling_describe(int(index), *[ctypes.byref(x) for x in v]),
           "sps_tiling_describe")
    return dict(zip(("m", "dpw", "nw", "cs", "waves_per_eu"), (x.value for x in v)))


def sps_probe_peaks(device: int = 0) -> dict:
    """Sustained lane-ops/s of v_add_u32, v_add3_u32, v_perm_b32 and LDS read
    bytes/s (16-byte and 4-byte reads) of the device."""
    rates = (ctypes.c_double * 5)()
    _check(library().sps_probe_peaks(int(device), rates, 5), "sps_probe_peaks")
    return {"valu_add_ops_per_s": rates[0], "valu_add3_ops_per_s": rates[1],
            "valu_perm_ops_per_s": rates[2], "lds_read_bytes_per_s": rates[3],
            "lds_read32_bytes_per_s": rates[4]}


def sps_batch_autotune(batch: Batch, iters: int = 3, stream=None) -> list:
    """Mean ms of the batch's dedispersion launch per compiled tiling (-1 where
    it does not fit); the batch keeps the fastest."""
    n = sps_tiling_count()
    ms = np.full(n, -1.0, dtype=np.float32)
    tried = ctypes.c_int32()
    _check(library().sps_batch_autotune(batch.handle, int(iters), _stream(stream),
                                        ms.ctypes.data, ctypes.byref(tried)), "sps_batch_autotune")
    return [float(x) for x in ms]


def sps_plan_autotune(plan: Plan, nout_probe: int, iters: int = 3, stream=None) -> list:
    """Mean ms per compiled tiling (-1 where it does not fit); keeps the fastest."""
    n = sps_tiling_count()
    ms = np.full(n, -1.0, dtype=np.float32)
    tried = ctypes.c_int32()
    _check(library().sps_plan_autotune(plan.handle, int(nout_probe), int(iters), _stream(stream),
                                       ms.ctypes.data, ctypes.byref(tried)), "sps_plan_autotune")
    return [float(x) for x in ms]


class Server:
    """Owns an sps_server handle and keeps the feeds of a run alive."""

    def __init__(self, handle):
        self.handle = handle
        self.widths = {}
        self.detector = None

    def close(self) -> None:
        if self.handle:
            sps_server_destroy(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


RECORD_DTYPE = np.dtype([("stream", np.int32), ("worker", np.int32), ("index", np.int64),
                         ("arrival_s", np.float64), ("start_s", np.float64),
                         ("upload_s", np.float64), ("compute_s", np.float64),
                         ("end_s", np.float64), ("n_cand", np.int32), ("status", np.int32),
                         ("n_cnn", np.int32), ("reserved", np.int32)])


def sps_server_create(hbm_budget: int, nworkers: int) -> Server:
    h = ctypes.c_void_p()
    _check(library().sps_server_create(int(hbm_budget), int(nworkers), ctypes.byref(h)),
           "sps_server_create")
    return Server(h.value)


def sps_server_destroy(server: Server) -> None:
    h, server.handle = server.handle, None
    if h:
        _check(library().sps_server_destroy(h), "sps_server_destroy")


def sps_server_add_stream(server: Server, freq_mhz: Sequence[float], fref_mhz: float,
                          tsamp_s: float, dm: Sequence[float], widths: Sequence[int],
                          threshold: float, tile_dm: int, tile_t: int, nms_dm: int, nms_t: int,
                          chunk_len: int) -> int:
    f = np.ascontiguousarray(freq_mhz, dtype=np.float64)
    m = np.ascontiguousarray(dm, dtype=np.float64)
    desc = sps_obs_desc(f.size, f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(fref_mhz),
                        float(tsamp_s), m.size, m.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    w = np.ascontiguousarray(widths, dtype=np.int32)
    prm = sps_detect_params(float(threshold), int(tile_dm), int(tile_t), int(nms_dm), int(nms_t))
    sid = ctypes.c_int32()
    _check(library().sps_server_add_stream(server.handle, ctypes.byref(desc), w.ctypes.data, w.size,
                                           ctypes.byref(prm), int(chunk_len), ctypes.byref(sid)),
           "sps_server_add_stream")
    server.widths[int(sid.value)] = [int(x) for x in w]
    return int(sid.value)


def sps_server_memory(server: Server) -> dict:
    u, b = ctypes.c_int64(), ctypes.c_int64()
    _check(library().sps_server_memory(server.handle, ctypes.byref(u), ctypes.byref(b)),
           "sps_server_memory")
    return {"used": int(u.value), "budget": int(b.value)}


def sps_server_stream_info(server: Server, stream_id: int) -> dict:
    c, o, d = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
    _check(library().sps_server_stream_info(server.handle, int(stream_id), ctypes.byref(c),
                                            ctypes.byref(o), ctypes.byref(d)),
           "sps_server_stream_info")
    return {"chunk_len": int(c.value), "overlap": int(o.value), "duration_s": float(d.value)}


def _host_ptr(a, name: str):
    if isinstance(a, torch.Tensor):
        if a.device.type != "cpu" or a.dtype != torch.uint8 or a.dim() != 2 or a.stride(1) != 1:
            raise TypeError(f"{name} must be a uint8 [nchan][pitch] host tensor")
        return a.data_ptr(), a.stride(0)
    a = np.asarray(a)
    if a.dtype != np.uint8 or a.ndim != 2 or a.strides[1] != 1:
        raise TypeError(f"{name} must be a uint8 [nchan][pitch] host array")
    return a.ctypes.data, a.strides[0]


def sps_server_push(server: Server, stream_id: int, chunk, Y_copy: Optional[torch.Tensor] = None,
                    cap: int = 4096, allow_truncated: bool = False, with_cnn: bool = False):
    """Searches the stream's next chunk (host uint8 [nchan][>= chunk_len]); returns
    (candidates, number found), plus the attached detector's count if with_cnn."""
    hp, pitch = _host_ptr(chunk, "chunk")
    yp = None
    if Y_copy is not None:
        yp = (_dev(Y_copy, torch.int32, "Y_copy") if Y_copy.dtype == torch.int32
              else _dev(Y_copy, torch.uint32, "Y_copy"))
    out = (sps_candidate * max(cap, 1))()
    n, ncnn = ctypes.c_int32(), ctypes.c_int32()
    rc = library().sps_server_push(server.handle, int(stream_id), hp, int(pitch), yp, out,
                                   int(cap), ctypes.byref(n), ctypes.byref(ncnn))
    if not (rc == 6 and allow_truncated):
        _check(rc, "sps_server_push")
    k = min(int(n.value), cap)
    arr = np.frombuffer(out, dtype=CANDIDATE_DTYPE)[:k].copy()
    if with_cnn:
        return arr, int(n.value), int(ncnn.value)
    return arr, int(n.value)


def sps_server_set_detector(server: Server, net, threshold: float = 0.9,
                            scale: float = 0.125) -> None:
    """Attaches net (a Cnn, or None to detach) to every chunk the server searches."""
    _check(library().sps_server_set_detector(server.handle, net.handle if net else None,
                                             float(threshold), float(scale)),
           "sps_server_set_detector")
    server.detector = net  # keeps the network alive while attached


def sps_server_run(server: Server, feeds: Sequence[dict], run_s: float, compression: float,
                   cap: int = 1 << 16) -> np.ndarray:
    """feeds[i]: dict(host=uint8 tensor/array [nsrc * nchan][src_pitch], nsrc, first).
    Returns the chunk records (structured array, arrival order)."""
    arr = (sps_feed * len(feeds))()
    keep = []
    for i, f in enumerate(feeds):
        hp, pitch = _host_ptr(f["host"], "feed")
        arr[i] = sps_feed(hp, int(pitch), int(f.get("nsrc", 1)), int(f.get("first", 0)))
        keep.append(f["host"])
    recs = (sps_chunk_record * max(cap, 1))()
    n = ctypes.c_int32()
    _check(library().sps_server_run(server.handle, arr, float(run_s), float(compression), recs,
                                    int(cap), ctypes.byref(n)), "sps_server_run")
    k = min(int(n.value), cap)
    return np.frombuffer(bytes(recs)[:k * ctypes.sizeof(sps_chunk_record)],
                         dtype=RECORD_DTYPE).copy()


class Cnn:
    """Owns an sps_cnn handle."""

    def __init__(self, handle, max_batch):
        self.handle, self.max_batch = handle, max_batch

    def close(self) -> None:
        if self.handle:
            sps_cnn_destroy(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


CNN_CANDIDATE_DTYPE = np.dtype([("tile", np.int32), ("cell_dm", np.int32), ("cell_t", np.int32),
                                ("prob", np.float32), ("row", np.float32), ("col", np.float32)])
CNN_LAYERS = ((1, 16, 2), (16, 32, 2), (32, 64, 2), (64, 128, 2), (128, 128, 2), (128, 128, 1))
CNN_TILE = (256, 512)
CNN_GRID = (8, 16)


def sps_cnn_param_count() -> int:
    return int(library().sps_cnn_param_count())


def sps_cnn_create(max_batch: int) -> Cnn:
    h = ctypes.c_void_p()
    _check(library().sps_cnn_create(int(max_batch), ctypes.byref(h)), "sps_cnn_create")
    return Cnn(h.value, int(max_batch))


def sps_cnn_destroy(net: Cnn) -> None:
    h, net.handle = net.handle, None
    if h:
        _check(library().sps_cnn_destroy(h), "sps_cnn_destroy")


def _params_vec(a) -> np.ndarray:
    v = np.ascontiguousarray(a, dtype=np.float32).ravel()
    if v.size != sps_cnn_param_count():
        raise ValueError(f"expected {sps_cnn_param_count()} parameters, got {v.size}")
    return v


def sps_cnn_set_params(net: Cnn, params) -> None:
    v = _params_vec(params)
    _check(library().sps_cnn_set_params(net.handle, v.ctypes.data), "sps_cnn_set_params")


def sps_cnn_set_loss_weights(net: Cnn, pos_weight: float = 32.0, lambda_box: float = 1.0) -> None:
    _check(library().sps_cnn_set_loss_weights(net.handle, float(pos_weight), float(lambda_box)),
           "sps_cnn_set_loss_weights")


def sps_cnn_get_params(net: Cnn) -> np.ndarray:
    v = np.empty(sps_cnn_param_count(), np.float32)
    _check(library().sps_cnn_get_params(net.handle, v.ctypes.data), "sps_cnn_get_params")
    return v


def sps_cnn_set_grads(net: Cnn, grads) -> None:
    v = _params_vec(grads)
    _check(library().sps_cnn_set_grads(net.handle, v.ctypes.data), "sps_cnn_set_grads")


def sps_cnn_get_grads(net: Cnn) -> np.ndarray:
    v = np.empty(sps_cnn_param_count(), np.float32)
    _check(library().sps_cnn_get_grads(net.handle, v.ctypes.data), "sps_cnn_get_grads")
    return v


def sps_cnn_activations(net: Cnn, layer: int, n: int) -> np.ndarray:
    """bf16 bit patterns NHWC [n][h][w][cout] of 3x3 layer `layer`."""
    size = 256 // 2 ** min(layer + 1, 5), 512 // 2 ** min(layer + 1, 5)
    out = np.empty((n, size[0], size[1], CNN_LAYERS[layer][1]), np.uint16)
    _check(library().sps_cnn_activations(net.handle, int(layer), int(n), out.ctypes.data),
           "sps_cnn_activations")
    return out


def sps_cnn_signals(net: Cnn, layer: int, n: int) -> np.ndarray:
    """bf16 bit patterns NHWC [n][h][w][cout] of the signal at 3x3 layer `layer`."""
    size = 256 // 2 ** min(layer + 1, 5), 512 // 2 ** min(layer + 1, 5)
    out = np.empty((n, size[0], size[1], CNN_LAYERS[layer][1]), np.uint16)
    _check(library().sps_cnn_signals(net.handle, int(layer), int(n), out.ctypes.data),
           "sps_cnn_signals")
    return out


def _tiles_ptr(tiles: torch.Tensor) -> int:
    if (not isinstance(tiles, torch.Tensor) or tiles.device.type != "cuda"
            or tiles.dtype not in (torch.uint16, torch.int16, torch.bfloat16)
            or not tiles.is_contiguous() or tuple(tiles.shape[-2:]) != CNN_TILE):
        raise TypeError("tiles must be a contiguous 16-bit [n][256][512] tensor on a GPU")
    return tiles.data_ptr()


def sps_cnn_pool_tiles(snr: torch.Tensor, nout: int, scale: float, tiles: torch.Tensor,
                       stream=None) -> None:
    if snr.dim() != 2 or snr.stride(1) != 1:
        raise ValueError("snr must be [ndm][pitch] with unit stride")
    if tiles.dtype not in (torch.uint16, torch.int16, torch.bfloat16) or not tiles.is_contiguous():
        raise TypeError("tiles must be a contiguous 16-bit tensor")
    _check(library().sps_cnn_pool_tiles(_dev(snr, torch.float32, "snr"), snr.stride(0),
                                        snr.shape[0], int(nout), float(scale), tiles.data_ptr(),
                                        _stream(stream)), "sps_cnn_pool_tiles")


def sps_cnn_pool_tile_grid(snr: torch.Tensor, nout: int, scale: float,
                           tiles: Optional[torch.Tensor], stream=None) -> int:
    """Cuts the plane into whole 512-trial x 4096-sample tiles, pooled; returns
    their number."""
    if snr.dim() != 2 or snr.stride(1) != 1:
        raise ValueError("snr must be [ndm][pitch] with unit stride")
    need = (snr.shape[0] // 512) * (int(nout) // 4096)
    tp = None
    if tiles is not None:
        if (tiles.dtype not in (torch.uint16, torch.int16, torch.bfloat16)
                or not tiles.is_contiguous() or tiles.numel() < need * 256 * 512):
            raise TypeError("tiles must be a contiguous 16-bit tensor of >= n x 256 x 512")
        tp = tiles.data_ptr()
    elif need:
        raise TypeError("tiles needed for a plane of whole tiles")
    nt = ctypes.c_int64()
    _check(library().sps_cnn_pool_tile_grid(_dev(snr, torch.float32, "snr"), snr.stride(0),
                                            snr.shape[0], int(nout), float(scale), tp,
                                            ctypes.byref(nt), _stream(stream)),
           "sps_cnn_pool_tile_grid")
    return int(nt.value)


def sps_cnn_max_batch(net: Cnn) -> int:
    return int(library().sps_cnn_max_batch(net.handle))


def sps_cnn_forward(net: Cnn, tiles: torch.Tensor, n: int, head: Optional[torch.Tensor] = None,
                    stream=None) -> None:
    hp = _dev(head, torch.float32, "head") if head is not None else None
    _check(library().sps_cnn_forward(net.handle, _tiles_ptr(tiles), int(n), hp, _stream(stream)),
           "sps_cnn_forward")


def sps_cnn_infer(net: Cnn, tiles: torch.Tensor, n: int, head: Optional[torch.Tensor] = None,
                  stream=None) -> None:
    hp = _dev(head, torch.float32, "head") if head is not None else None
    _check(library().sps_cnn_infer(net.handle, _tiles_ptr(tiles), int(n), hp, _stream(stream)),
           "sps_cnn_infer")


def sps_cnn_loss_grad(net: Cnn, tiles: torch.Tensor, labels: torch.Tensor, n: int,
                      loss: Optional[torch.Tensor] = None, stream=None) -> None:
    lp = _dev(loss, torch.float32, "loss") if loss is not None else None
    _check(library().sps_cnn_loss_grad(net.handle, _tiles_ptr(tiles),
                                       _dev(labels, torch.float32, "labels"), int(n), lp,
                                       _stream(stream)), "sps_cnn_loss_grad")


def sps_cnn_adam(net: Cnn, lr: float, beta1: float = 0.9, beta2: float = 0.999,
                 eps: float = 1e-8, stream=None) -> None:
    _check(library().sps_cnn_adam(net.handle, float(lr), float(beta1), float(beta2), float(eps),
                                  _stream(stream)), "sps_cnn_adam")


def sps_cnn_train_step(net: Cnn, tiles: torch.Tensor, labels: torch.Tensor, n: int, lr: float,
                       loss: Optional[torch.Tensor] = None, stream=None) -> None:
    lp = _dev(loss, torch.float32, "loss") if loss is not None else None
    _check(library().sps_cnn_train_step(net.handle, _tiles_ptr(tiles),
                                        _dev(labels, torch.float32, "labels"), int(n), float(lr),
                                        lp, _stream(stream)), "sps_cnn_train_step")


def sps_cnn_detect(net: Cnn, tiles: torch.Tensor, n: int, threshold: float, cap: int = 65536,
                   stream=None, allow_truncated: bool = False):
    out = (sps_cnn_candidate * max(cap, 1))()
    k = ctypes.c_int32()
    rc = library().sps_cnn_detect(net.handle, _tiles_ptr(tiles), int(n), float(threshold), out,
                                  int(cap), ctypes.byref(k), _stream(stream))
    if not (rc == 6 and allow_truncated):
        _check(rc, "sps_cnn_detect")
    m = min(int(k.value), cap)
    arr = np.frombuffer(bytes(out)[:m * ctypes.sizeof(sps_cnn_candidate)],
                        dtype=CNN_CANDIDATE_DTYPE).copy()
    return arr, int(k.value)


def plan_for(wl) -> Plan:
    """Plan for a workload description (see ``workloads``)."""
    return sps_plan_create(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, wl.dms())
