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


class sps_detect_params(ctypes.Structure):
    _fields_ = [("threshold", ctypes.c_float), ("tile_dm", ctypes.c_int32),
                ("tile_t", ctypes.c_int64), ("nms_dm", ctypes.c_int32), ("nms_t", ctypes.c_int64)]


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
        lib.sps_plan_set_tiling.argtypes = [P, i32, i32, i32, i32, i32]
        lib.sps_plan_get_tiling.argtypes = [P] + [ctypes.POINTER(i32)] * 6
        for f in ("sps_plan_create", "sps_plan_destroy", "sps_plan_delays", "sps_dedisperse",
                  "sps_boxcar_snr", "sps_detect", "sps_plan_set_tiling", "sps_plan_get_tiling"):
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
    return sorted(set(re.findall(r"^\s*(?:sps_status|const char \*)\s*(sps_\w+)\s*\(", text, re.M)))


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


CANDIDATE_DTYPE = np.dtype([("dm_idx", np.int32), ("width", np.int32), ("t_idx", np.int64),
                            ("snr", np.float32), ("reserved", np.float32), ("dm", np.float64),
                            ("toa_s", np.float64)])


def sps_detect(plan: Plan, snr: torch.Tensor, best_w: torch.Tensor, nout: int,
               widths: Sequence[int], threshold: float, tile_dm: int, tile_t: int, nms_dm: int,
               nms_t: int, cap: int = 4096, stream=None, allow_truncated: bool = False):
    """Returns (structured array of candidates, number found)."""
    w = np.ascontiguousarray(widths, dtype=np.int32)
    prm = sps_detect_params(float(threshold), int(tile_dm), int(tile_t), int(nms_dm), int(nms_t))
    out = (sps_candidate * max(cap, 1))()
    n = ctypes.c_int32()
    rc = library().sps_detect(plan.handle, _dev(snr, torch.float32, "snr"),
                              _dev(best_w, torch.uint8, "best_w"), int(nout), w.ctypes.data,
                              w.size, ctypes.byref(prm), out, int(cap), ctypes.byref(n),
                              _stream(stream))
    if not (rc == 6 and allow_truncated):
        _check(rc, "sps_detect")
    k = min(int(n.value), cap)
    arr = np.frombuffer(bytes(out)[:k * ctypes.sizeof(sps_candidate)], dtype=CANDIDATE_DTYPE).copy()
    return arr, int(n.value)


def plan_for(wl) -> Plan:
    """Plan for a workload description (see ``workloads``)."""
    return sps_plan_create(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, wl.dms())
