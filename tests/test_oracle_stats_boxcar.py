"""Pins for the oracle's row statistics and boxcar S/N.

Statistics: hand-worked rows, numpy's own selection routine (np.partition)
and a constant row.  Boxcar: the w = 1 closed form, prefix-sum differences
from np.cumsum, a noiseless top-hat with a constructed sigma, exact ties,
edge windows and the degenerate MAD = 0 row.
"""
import numpy as np
import pytest

import oracle


def test_hand_worked_stats():
    Y = np.array([[1, 2, 3, 4, 100], [1, 2, 3, 4, 0], [5, 5, 5, 5, 5]], np.uint32)
    st = oracle.stats(Y)
    # row 0: sorted 1 2 3 4 100 -> rank 2 -> 3; |dev| 2 1 0 1 97 -> 0 1 1 2 97 -> 1
    # row 1: sorted 0 1 2 3 4 -> 2; |dev| 1 0 1 2 2 -> 0 1 1 2 2 -> 1
    assert st.tolist() == [[3, 1], [2, 1], [5, 0]]
    # even length: lower median (rank (n-1)//2)
    st = oracle.stats(np.array([[4, 1, 3, 2]], np.uint32))
    # sorted 1 2 3 4 -> rank 1 -> 2; |dev| 2 1 1 0 -> 0 1 1 2 -> 1
    assert st.tolist() == [[2, 1]]


@pytest.mark.parametrize("n", [1, 2, 3, 10, 1001, 4096])
def test_stats_against_numpy_partition(n):
    rng = np.random.Generator(np.random.PCG64(n))
    Y = rng.integers(0, 2 ** 20, size=(4, n)).astype(np.uint32)
    Y[1] = rng.integers(1000, 1010, size=n)  # many ties
    st = oracle.stats(Y)
    k = (n - 1) // 2
    for d in range(Y.shape[0]):
        med = np.partition(Y[d].astype(np.int64), k)[k]
        mad = np.partition(np.abs(Y[d].astype(np.int64) - med), k)[k]
        assert st[d].tolist() == [med, mad]


def _row_with_sigma(n, med, s):
    # alternating med - s, med + s, ... plus one med: median = med, MAD = s
    r = np.empty(n, np.int64)
    r[0::2] = med - s
    r[1::2] = med + s
    r[n // 2] = med
    return r


def test_w1_is_normalised_row():
    rng = np.random.Generator(np.random.PCG64(2))
    Y = rng.integers(100000, 101000, size=(3, 257)).astype(np.uint32)
    st = oracle.stats(Y)
    snr, best, s64 = oracle.boxcar(Y, st, [1], want_f64=True)
    for d in range(3):
        med, mad = st[d]
        want = (Y[d].astype(np.float64) - med) / (1.4826 * mad)
        assert np.allclose(s64[d], want, rtol=1e-15, atol=0)
        assert np.array_equal(snr[d], want.astype(np.float32))
    assert np.all(best == 0)


def test_against_cumsum_differences():
    rng = np.random.Generator(np.random.PCG64(3))
    widths = [1, 2, 3, 5, 8, 13]
    Y = rng.integers(0, 5000, size=(4, 300)).astype(np.uint32)
    st = oracle.stats(Y)
    snr, best, s64 = oracle.boxcar(Y, st, widths, want_f64=True)
    for d in range(4):
        P = np.concatenate([[0], np.cumsum(Y[d].astype(np.int64))])
        med, mad = st[d]
        n = Y.shape[1]
        allw = np.full((len(widths), n), -np.inf)
        allf = np.full((len(widths), n), -np.inf, np.float32)
        for i, w in enumerate(widths):
            B = P[w:] - P[:-w]
            s = (B - w * med) / (1.4826 * mad * np.sqrt(w))
            allw[i, :n - w + 1] = s
            allf[i, :n - w + 1] = s.astype(np.float32)
        bi = np.argmax(allf, axis=0)  # first maximum = smallest width
        assert np.array_equal(best[d], bi.astype(np.uint8))
        assert np.allclose(s64[d], allw[bi, np.arange(n)], rtol=1e-13)
        assert np.array_equal(snr[d], allf[bi, np.arange(n)])


def test_top_hat_closed_form():
    # baseline: 20% exactly med, 40% med - s, 40% med + s -> median med, MAD s;
    # a top-hat of height A over w0 samples of exact baseline med
    n, med, s = 1001, 50000, 40
    i = np.arange(n)
    row = np.full(n, med, np.int64)
    row[(i % 5 == 1) | (i % 5 == 2)] = med - s
    row[(i % 5 == 3) | (i % 5 == 4)] = med + s
    A, w0, t0 = 900, 16, 401
    row[t0:t0 + w0] = med + A
    Y = row[None, :].astype(np.uint32)
    st = oracle.stats(Y)
    assert st.tolist() == [[med, s]]
    snr, best, s64 = oracle.boxcar(Y, st, [1, 2, 4, 8, 16, 32], want_f64=True)
    want = A * w0 / (1.4826 * s * np.sqrt(w0))
    assert best[0, t0] == 4 and abs(s64[0, t0] - want) < 1e-9 * want
    assert np.argmax(snr[0]) == t0


def test_exact_tie_takes_smallest_width():
    # relative to the median the window reads (a, a, 0, 0): S/N_1 = a/sigma and
    # S/N_4 = 2a / (2 sigma), equal in exact and in binary arithmetic
    n, med, s, a = 401, 10000, 10, 300
    row = _row_with_sigma(n, med, s)
    t0 = 101
    row[t0 - 3:t0 + 8] = med
    row[t0] = med + a
    row[t0 + 1] = med + a
    Y = row[None, :].astype(np.uint32)
    st = oracle.stats(Y)
    assert st.tolist() == [[med, s]]
    snr, best = oracle.boxcar(Y, st, [1, 4])
    assert best[0, t0] == 0
    assert snr[0, t0] == np.float32(a / (1.4826 * s))


def test_edges_and_degenerate_rows():
    Y = np.array([[3, 9, 1, 4, 8, 2, 7], [6] * 7], np.uint32)
    st = oracle.stats(Y)
    snr, best = oracle.boxcar(Y, st, [2, 4])
    # only full windows: w = 4 up to t = 3, w = 2 up to t = 5, nothing at t = 6
    assert best[0, 6] == 0xFF and snr[0, 6] == 0
    assert best[0, 5] == 0
    # MAD = 0: S/N is 0 and the smallest width wins
    assert st[1, 1] == 0
    assert np.all(snr[1] == 0) and np.all(best[1, :6] == 0) and best[1, 6] == 0xFF


def test_rejects_bad_widths():
    Y = np.zeros((1, 8), np.uint32)
    st = oracle.stats(Y)
    for bad in ([2, 1], [0, 1], [1, 1]):
        with pytest.raises(ValueError):
            oracle.boxcar(Y, st, bad)
