"""Plain CPU oracle for the single-pulse search hot path.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the tests, the smoke check and
the CPU-baseline leg of the benchmark may import this package.  It shares no
code with the GPU library (``paper_2511_02328_amd``) and never imports it.

The arithmetic lives in ``sps_oracle.c`` (plain C, double precision, built by
``oracle.build``); this module only marshals numpy arrays.  Each function
names the passage of the paper it follows:

* :func:`delays`      -- Sec. 2.3, Eq. (KDM) and Eq. (coarse_delay).
* :func:`dedisperse`  -- Sec. 2.3, brute-force dedispersion; zero outside
  bounds as in Eq. (stage1).
* :func:`stats`       -- per-row lower median / MAD (reading of the S/N
  normalisation, which the paper does not define).
* :func:`boxcar`      -- Sec. 1, step (iii): boxcar matched filter bank.
* :func:`detect`      -- tile maxima, threshold, greedy suppression; record
  fields from Sec. 2 (DM, TOA referenced to the top of the band, S/N, width).
* :func:`row_checksums` -- per-row sums of the dedispersed plane from
  per-channel prefix sums (a property that holds at any size).
* :func:`subband_residuals`, :func:`subband_dedisperse` -- the paper's
  two-stage subband method, Sec. 2.3, Eq. (coarse_delay), Eq. (stage1),
  Eq. (residual), Eq. (stage2).
* :func:`zero_dm` -- the zero-DM filter cited in Sec. 2.1 (formula read as
  channel-mean subtraction, stated in the C source).
* :func:`downsample_sqrt` -- square-law downsampling, Sec. 2.2.

Every function here is pinned by tests against values the paper and the
mathematics fix (closed forms, exact rational arithmetic, brute force on tiny
inputs, library special cases); none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB_PATH, build

_lib = None

_ERRORS = {-1: "invalid argument", -2: "out of memory", -3: "overflow"}


def _load():
    global _lib
    if _lib is None:
        path = os.environ.get("SPS_ORACLE_LIB", LIB_PATH)
        if path == LIB_PATH and not os.path.exists(LIB_PATH):
            build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i32, i64, f32, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double
        lib.sps_oracle_delays.argtypes = [i32, P, f64, f64, i32, P, P]
        lib.sps_oracle_dedisperse.argtypes = [i32, P, i64, i64, i32, P, i64, P]
        lib.sps_oracle_stats.argtypes = [i32, i64, P, P]
        lib.sps_oracle_boxcar.argtypes = [i32, i64, P, P, i32, P, P, P, P]
        lib.sps_oracle_detect.argtypes = [i32, i64, P, P, f32, i32, i64, i32, i64,
                                          i32, P, P, P, P, P]
        lib.sps_oracle_row_checksums.argtypes = [i32, P, i64, i64, i32, P, i64, P]
        lib.sps_oracle_threads.argtypes = []
        lib.sps_oracle_subband_residuals.argtypes = [i32, P, f64, f64, i32, P, i32, f64, f64,
                                                     i32, P, P, P]
        lib.sps_oracle_subband_dedisperse.argtypes = [i32, P, i64, i64, i32, P, i32, P, i32, i32,
                                                      P, i64, P]
        lib.sps_oracle_zero_dm.argtypes = [i32, P, i64, i64, P, i64]
        lib.sps_oracle_downsample_sqrt.argtypes = [i32, P, i64, i64, i32, P, i64]
        for name in ("delays", "dedisperse", "stats", "boxcar", "detect",
                     "row_checksums", "threads", "subband_residuals", "subband_dedisperse",
                     "zero_dm", "downsample_sqrt"):
            getattr(lib, "sps_oracle_" + name).restype = ctypes.c_int
        _lib = lib
    return _lib


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise ValueError(f"oracle {what}: {_ERRORS.get(rc, rc)}")


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def threads() -> int:
    """Threads the oracle's parallel loops use."""
    return int(_load().sps_oracle_threads())


def delays(freq_mhz, fref_mhz: float, tsamp_s: float, dm) -> np.ndarray:
    """Integer delay table D[d][c] (int32, [ndm][nchan]); Eq. (coarse_delay)."""
    f = np.ascontiguousarray(freq_mhz, dtype=np.float64)
    m = np.ascontiguousarray(dm, dtype=np.float64)
    D = np.empty((m.size, f.size), dtype=np.int32)
    _check(_load().sps_oracle_delays(f.size, _ptr(f), float(fref_mhz), float(tsamp_s),
                                     m.size, _ptr(m), _ptr(D)), "delays")
    return D


def _x_layout(X: np.ndarray, nsamp_in):
    X = np.asarray(X)
    if X.dtype != np.uint8 or X.ndim != 2:
        raise ValueError("X must be a 2-D uint8 array [nchan][pitch]")
    if X.strides[1] != 1 or X.strides[0] < X.shape[1]:
        X = np.ascontiguousarray(X)
    pitch = X.strides[0]
    n = X.shape[1] if nsamp_in is None else int(nsamp_in)
    if n > X.shape[1]:
        raise ValueError("nsamp_in exceeds the row length of X")
    return X, pitch, n


def dedisperse(X: np.ndarray, D: np.ndarray, nout: int, nsamp_in=None) -> np.ndarray:
    """Brute-force dedispersion Y[d][t] = sum_c X[c][t + D[d][c]] (uint32)."""
    X, pitch, n = _x_layout(X, nsamp_in)
    D = np.ascontiguousarray(D, dtype=np.int32)
    if D.shape[1] != X.shape[0]:
        raise ValueError("delay table and X disagree on the channel count")
    Y = np.empty((D.shape[0], int(nout)), dtype=np.uint32)
    _check(_load().sps_oracle_dedisperse(X.shape[0], _ptr(X), pitch, n, D.shape[0],
                                         _ptr(D), int(nout), _ptr(Y)), "dedisperse")
    return Y


def stats(Y: np.ndarray) -> np.ndarray:
    """Per-row (lower median, MAD) as int64 [ndm][2]."""
    Y = np.ascontiguousarray(Y, dtype=np.uint32)
    S = np.empty((Y.shape[0], 2), dtype=np.int64)
    _check(_load().sps_oracle_stats(Y.shape[0], Y.shape[1], _ptr(Y), _ptr(S)), "stats")
    return S


def boxcar(Y: np.ndarray, st: np.ndarray, widths, want_f64: bool = False):
    """Boxcar S/N: returns (snr f32 [ndm][nout], best width index u8[, snr f64])."""
    Y = np.ascontiguousarray(Y, dtype=np.uint32)
    st = np.ascontiguousarray(st, dtype=np.int64)
    w = np.ascontiguousarray(widths, dtype=np.int32)
    snr = np.empty(Y.shape, dtype=np.float32)
    best = np.empty(Y.shape, dtype=np.uint8)
    s64 = np.empty(Y.shape, dtype=np.float64) if want_f64 else None
    _check(_load().sps_oracle_boxcar(Y.shape[0], Y.shape[1], _ptr(Y), _ptr(st), w.size,
                                     _ptr(w), _ptr(snr), _ptr(best),
                                     _ptr(s64) if want_f64 else None), "boxcar")
    return (snr, best, s64) if want_f64 else (snr, best)


def detect(snr: np.ndarray, best: np.ndarray, threshold: float, tile_dm: int, tile_t: int,
           nms_dm: int, nms_t: int, cap: int = 1 << 16):
    """Candidates as a dict of arrays (d, t, w index, snr) plus the true count."""
    snr = np.ascontiguousarray(snr, dtype=np.float32)
    best = np.ascontiguousarray(best, dtype=np.uint8)
    if snr.shape != best.shape:
        raise ValueError("snr and best differ in shape")
    od = np.empty(cap, np.int32)
    ot = np.empty(cap, np.int64)
    ow = np.empty(cap, np.int32)
    os_ = np.empty(cap, np.float32)
    nf = np.zeros(1, np.int64)
    _check(_load().sps_oracle_detect(snr.shape[0], snr.shape[1], _ptr(snr), _ptr(best),
                                     float(threshold), int(tile_dm), int(tile_t), int(nms_dm),
                                     int(nms_t), int(cap), _ptr(od), _ptr(ot), _ptr(ow),
                                     _ptr(os_), _ptr(nf)), "detect")
    n = int(nf[0])
    k = min(n, cap)
    return {"d": od[:k].copy(), "t": ot[:k].copy(), "w": ow[:k].copy(),
            "snr": os_[:k].copy(), "n_found": n}


def row_checksums(X: np.ndarray, D: np.ndarray, nout: int, nsamp_in=None) -> np.ndarray:
    """sum_t Y[d][t] for every row, without forming Y (uint64 [ndm])."""
    X, pitch, n = _x_layout(X, nsamp_in)
    D = np.ascontiguousarray(D, dtype=np.int32)
    out = np.empty(D.shape[0], dtype=np.uint64)
    _check(_load().sps_oracle_row_checksums(X.shape[0], _ptr(X), pitch, n, D.shape[0],
                                            _ptr(D), int(nout), _ptr(out)), "row_checksums")
    return out


def pipeline(X: np.ndarray, D: np.ndarray, nout: int, widths, nsamp_in=None):
    """dedisperse -> stats -> boxcar on the CPU; returns (Y, stats, snr, best)."""
    Y = dedisperse(X, D, nout, nsamp_in)
    st = stats(Y)
    snr, best = boxcar(Y, st, widths)
    return Y, st, snr, best


def equal_subbands(nchan: int, nsub: int) -> np.ndarray:
    """Subband boundaries [nsub + 1]: contiguous, sizes differing by at most one."""
    return np.array([(s * nchan) // nsub for s in range(nsub + 1)], dtype=np.int32)


def subband_residuals(freq_mhz, fref_mhz: float, tsamp_s: float, sub, ndm: int, dm_lo: float,
                      ddm: float, n0: int):
    """(R int32 [ndm][nsub], F_s [nsub], coarse DMs [ceil(ndm/n0)]); Eq. (residual)."""
    f = np.ascontiguousarray(freq_mhz, dtype=np.float64)
    sb = np.ascontiguousarray(sub, dtype=np.int32)
    nsub = sb.size - 1
    R = np.empty((ndm, nsub), dtype=np.int32)
    F = np.empty(nsub, dtype=np.float64)
    dmc = np.empty((ndm + n0 - 1) // n0, dtype=np.float64)
    _check(_load().sps_oracle_subband_residuals(f.size, _ptr(f), float(fref_mhz), float(tsamp_s),
                                                nsub, _ptr(sb), int(ndm), float(dm_lo), float(ddm),
                                                int(n0), _ptr(R), _ptr(F), _ptr(dmc)),
           "subband_residuals")
    return R, F, dmc


def subband_dedisperse(X: np.ndarray, Dc: np.ndarray, sub, R: np.ndarray, n0: int, nout: int,
                       nsamp_in=None) -> np.ndarray:
    """Two-stage subband dedispersion, Eq. (stage1) + Eq. (stage2) (uint32 [ndm][nout])."""
    X, pitch, n = _x_layout(X, nsamp_in)
    Dc = np.ascontiguousarray(Dc, dtype=np.int32)
    sb = np.ascontiguousarray(sub, dtype=np.int32)
    R = np.ascontiguousarray(R, dtype=np.int32)
    Y = np.empty((R.shape[0], int(nout)), dtype=np.uint32)
    _check(_load().sps_oracle_subband_dedisperse(X.shape[0], _ptr(X), pitch, n, Dc.shape[0],
                                                 _ptr(Dc), sb.size - 1, _ptr(sb), R.shape[0],
                                                 int(n0), _ptr(R), int(nout), _ptr(Y)),
           "subband_dedisperse")
    return Y


def zero_dm(X: np.ndarray, nsamp=None) -> np.ndarray:
    """Zero-DM filtered copy of X[:, :nsamp] (uint8)."""
    X, pitch, n = _x_layout(X, nsamp)
    out = np.zeros((X.shape[0], n), dtype=np.uint8)
    _check(_load().sps_oracle_zero_dm(X.shape[0], _ptr(X), pitch, n, _ptr(out), max(n, 1) if n else 0),
           "zero_dm")
    return out


def downsample_sqrt(X: np.ndarray, factor: int, nsamp=None) -> np.ndarray:
    """Square-law downsampled copy (uint8 [nchan][nsamp // factor])."""
    X, pitch, n = _x_layout(X, nsamp)
    nout = n // int(factor)
    out = np.zeros((X.shape[0], max(nout, 1)), dtype=np.uint8)
    _check(_load().sps_oracle_downsample_sqrt(X.shape[0], _ptr(X), pitch, n, int(factor),
                                              _ptr(out), max(nout, 1)), "downsample_sqrt")
    return out[:, :nout]


_cnn_mod = None


def cnn():
    """The detector oracle module (``oracle/detector.py``), or the copy named by the
    environment variable SPS_CNN_ORACLE_SRC (used to plant mistakes in tests)."""
    global _cnn_mod
    if _cnn_mod is None:
        src = os.environ.get("SPS_CNN_ORACLE_SRC")
        if src:
            import importlib.util
            spec = importlib.util.spec_from_file_location("oracle_cnn_copy", src)
            mod = importlib.util.module_from_spec(spec)
            spec.loader.exec_module(mod)
            _cnn_mod = mod
        else:
            from . import detector as mod
            _cnn_mod = mod
    return _cnn_mod
