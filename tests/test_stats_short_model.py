"""CPU model of the short-row statistics form (rows of at most 4096 values).

The GPU form centres a window of 4096 unit bins on the row mean, takes the
median from the window's inclusive prefix P, and finds the MAD, the least m
with P[med + m] - P[med - m - 1] > k, in two ballot steps over one wave
(m = 33 l + 32 for lanes l < 64, then 33 consecutive values).  Rows the
window cannot hold go to an exact radix selection.  This model takes the same
decisions in the same order; wherever it keeps a row it must agree with the
exact order statistics, and it must hand over the rows whose median or MAD
lies outside the window."""
import numpy as np
import pytest

W = 4096


def window_model(v):
    """(median, MAD) from the window, or None where the GPU form falls back."""
    n = v.size
    k = (n - 1) // 2
    centre = ((int(np.sum(v >> 8)) << 8) // n) + 128
    lo = centre - W // 2 if centre > W // 2 else 0
    x = v.astype(np.int64) - lo
    inw = (x >= 0) & (x < W)
    below, inside = int(np.sum(v < lo)), int(inw.sum())
    if not (k >= below and k - below < inside):
        return None
    P = np.cumsum(np.bincount(x[inw], minlength=W))
    mloc = int(np.count_nonzero(P <= k - below))  # first bin whose prefix exceeds the rank
    mspan = min(mloc + 1, W - mloc)

    def reaches(m):
        m = min(m, mspan - 1)
        return P[mloc + m] - (P[mloc - m - 1] if m < mloc else 0) >= k + 1

    first = [reaches(33 * lane + 32) for lane in range(64)]
    if not any(first):
        return None
    f = first.index(True)
    second = [lane < 33 and reaches(33 * f + lane) for lane in range(64)]
    return lo + mloc, 33 * f + second.index(True)


def exact(v):
    s = np.sort(v.astype(np.int64))
    k = (v.size - 1) // 2
    med = int(s[k])
    return med, int(np.sort(np.abs(v.astype(np.int64) - med))[k])


def _row(kind, n, rng):
    if kind == "noise":
        v = rng.normal(32768, 256, n)
    elif kind == "wide":
        v = rng.normal(500000, rng.uniform(1, 4000), n)
    elif kind == "near_zero":
        v = np.abs(rng.normal(0, 700, n))
    elif kind == "constant":
        v = np.full(n, 1234.0)
    elif kind == "bimodal":
        v = rng.choice([100000, 900000], n) + rng.integers(-5, 6, n)
    else:  # spikes that drag the mean
        v = rng.normal(400000, 300, n)
        v[::97] += 600000
    return np.clip(np.rint(v), 0, 255 * 4096).astype(np.int64)


@pytest.mark.parametrize("kind", ["noise", "wide", "near_zero", "constant", "bimodal", "spikes"])
def test_window_model_matches_order_statistics(kind):
    rng = np.random.default_rng(len(kind))
    kept = 0
    for n in (1, 2, 3, 5, 64, 1023, 3001, 4095, 4096):
        for _ in range(12):
            v = _row(kind, n, rng)
            r = window_model(v)
            if r is not None:
                kept += 1
                assert r == exact(v), (kind, n)
    if kind in ("noise", "near_zero", "constant"):
        assert kept == 9 * 12   # the window holds every such row
    if kind == "bimodal":
        assert kept <= 2 * 12   # only rows of one or two values can be held


def test_window_model_hands_over_a_mad_past_the_window():
    # a median inside the window but a MAD wider than its half: the first
    # ballot finds no lane and the row goes to the radix selection
    v = np.concatenate([np.full(1000, 500000), np.full(1500, 497000), np.full(1500, 503000)])
    assert window_model(v) is None
    assert exact(v) == (500000, 3000)
