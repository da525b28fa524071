"""Comparison rules shared by the GPU parity tests (no GPU code here).

S/N: |g - o| <= 1e-5 max(1, |o|).  Best-width index: identical wherever the
oracle's best width wins by more than that tolerance; at near-ties the
GPU's width must itself reach the oracle's maximum within the tolerance,
its S/N taken from the boxcar formula on the oracle's plane."""
import numpy as np

import oracle

SNR_RTOL = 1e-5


def check_snr(Yo, sto, widths, snr_g, best_g, label=""):
    """GPU S/N and widths of rows Yo (oracle plane, stats sto) against the oracle."""
    snro, besto, s64 = oracle.boxcar(Yo, sto, widths, want_f64=True)
    tol = SNR_RTOL * np.maximum(1.0, np.abs(snro.astype(np.float64)))
    err = np.abs(snr_g.astype(np.float64) - snro.astype(np.float64))
    assert np.all(err <= tol), f"{label}: max S/N error {err.max()}"
    mism = np.nonzero(best_g != besto)
    if mism[0].size == 0:
        return snro, besto
    r, t = mism
    bg = best_g[r, t].astype(np.int64)
    assert np.all(bg < len(widths)) and np.all(besto[r, t] < len(widths)), \
        f"{label}: width index 0xFF differs"
    w = np.asarray(widths, np.int64)[bg]
    P = np.zeros((Yo.shape[0], Yo.shape[1] + 1), np.int64)
    np.cumsum(Yo.astype(np.int64), axis=1, out=P[:, 1:])
    med = sto[r, 0].astype(np.float64)
    mad = sto[r, 1].astype(np.float64)
    s_w = ((P[r, t + w] - P[r, t]).astype(np.float64) - w * med) / (1.4826 * mad * np.sqrt(w))
    assert np.all(np.abs(s_w - s64[r, t]) <= 2 * tol[r, t]), f"{label}: width mismatch off a near-tie"
    return snro, besto


def check_candidates_exact(cands, n, co, widths, label=""):
    """GPU candidates against oracle.detect on the same plane: identical, in order."""
    assert n == co["n_found"], f"{label}: {n} candidates, oracle {co['n_found']}"
    k = min(n, len(cands))
    assert list(cands["dm_idx"][:k]) == list(co["d"][:k]), label
    assert list(cands["t_idx"][:k]) == list(co["t"][:k]), label
    assert list(cands["width"][:k]) == [widths[i] for i in co["w"][:k]], label
    assert np.array_equal(cands["snr"][:k], co["snr"][:k]), label


def check_candidates_close(cands, n, co, widths, label=""):
    """GPU candidates against oracle.detect on the oracle's own plane: the
    same (d, t, w) set, S/N within the tolerance."""
    assert n == co["n_found"], f"{label}: {n} candidates, oracle {co['n_found']}"
    got = sorted(zip(cands["dm_idx"], cands["t_idx"], cands["width"]))
    want = sorted(zip(co["d"], co["t"], [widths[i] for i in co["w"]]))
    assert got == want, label
    assert np.allclose(np.sort(cands["snr"]), np.sort(co["snr"]), rtol=SNR_RTOL, atol=0), label
