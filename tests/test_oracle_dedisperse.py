"""Pins for the oracle's brute-force dedispersion (Sec. 2.3; Eq. stage1's
zero-outside-bounds convention) and its row-checksum property.

Checked against: per-(d, t) pure-Python brute force, an np.add.at
formulation, the plain channel sum at DM 0, impulse responses that recover
the delay table, constant and linear inputs, and a pulse laid exactly on a
trial's rounded delays.
"""
import numpy as np
import pytest

import oracle
from sps_inputs import synth
from sps_inputs.workloads import SINGLE_BEAM


def _brute_python(X, D, nout, nsamp_in):
    nchan = X.shape[0]
    Y = np.zeros((D.shape[0], nout), dtype=np.int64)
    for d in range(D.shape[0]):
        for t in range(nout):
            s = 0
            for c in range(nchan):
                i = t + int(D[d, c])
                if i < nsamp_in:
                    s += int(X[c, i])
            Y[d, t] = s
    return Y


def _brute_add_at(X, D, nout, nsamp_in):
    ndm, nchan = D.shape
    Y = np.zeros((ndm, nout), dtype=np.int64)
    t = np.arange(nout)
    for d in range(ndm):
        idx = t[None, :] + D[d][:, None]
        ok = idx < nsamp_in
        vals = np.where(ok, X[np.arange(nchan)[:, None], np.minimum(idx, nsamp_in - 1)], 0)
        np.add.at(Y[d], np.broadcast_to(t, idx.shape).ravel(), vals.ravel().astype(np.int64))
    return Y


@pytest.mark.parametrize("seed,nchan,ndm,nout,extra", [
    (1, 3, 4, 7, 5), (2, 5, 3, 11, 0), (3, 1, 1, 1, 0), (4, 7, 6, 13, -4), (5, 4, 2, 9, 40)])
def test_tiny_brute_force(seed, nchan, ndm, nout, extra):
    rng = np.random.Generator(np.random.PCG64(seed))
    D = np.sort(rng.integers(0, 9, size=(ndm, nchan)).astype(np.int32), axis=0)
    nsamp_in = max(1, nout + int(D.max()) + extra)
    X = rng.integers(0, 256, size=(nchan, nsamp_in + 3), dtype=np.uint8)
    got = oracle.dedisperse(X, D, nout, nsamp_in)
    assert np.array_equal(got, _brute_python(X, D, nout, nsamp_in))
    assert np.array_equal(got, _brute_add_at(X, D, nout, nsamp_in))


def test_pitch_padding_is_ignored():
    rng = np.random.Generator(np.random.PCG64(9))
    D = rng.integers(0, 20, size=(5, 6)).astype(np.int32)
    X = rng.integers(0, 256, size=(6, 64), dtype=np.uint8)
    a = oracle.dedisperse(X, D, 30, nsamp_in=40)
    X2 = X.copy()
    X2[:, 40:] = 255
    assert np.array_equal(a, oracle.dedisperse(X2, D, 30, nsamp_in=40))
    assert np.array_equal(a, _brute_python(X, D, 30, 40))


def test_dm0_is_channel_sum():
    wl = SINGLE_BEAM
    D = oracle.delays(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, wl.dms()[:3])
    X = synth.random_bytes(wl.nchan, 6000, seed=3)
    Y = oracle.dedisperse(X, D, 4096)
    assert np.array_equal(Y[0], X[:, :4096].astype(np.uint64).sum(axis=0))


def test_impulse_response_recovers_delays():
    wl = SINGLE_BEAM
    dms = wl.dms()[::37]
    D = oracle.delays(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, dms)
    nout = 64
    nsamp = nout + int(D.max()) + 1
    for c in (0, 77, 255):
        for tstar in (int(D[:, c].max()) + 5, int(D[:, c].max()) + 40):
            X = np.zeros((wl.nchan, nsamp), np.uint8)
            X[c, tstar] = 1
            Y = oracle.dedisperse(X, D, nout, nsamp)
            for d in range(len(dms)):
                nz = np.flatnonzero(Y[d])
                t = tstar - int(D[d, c])
                assert list(nz) == ([t] if 0 <= t < nout else [])


def test_constant_and_linearity():
    wl = SINGLE_BEAM
    D = oracle.delays(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, wl.dms()[::50])
    nsamp = 500 + int(D.max())
    X = np.full((wl.nchan, nsamp), 7, np.uint8)
    assert np.all(oracle.dedisperse(X, D, 500) == 7 * wl.nchan)
    A = synth.random_bytes(wl.nchan, nsamp, seed=5, hi=100)
    B = synth.random_bytes(wl.nchan, nsamp, seed=6, hi=100)
    ya = oracle.dedisperse(A, D, 500).astype(np.int64)
    yb = oracle.dedisperse(B, D, 500).astype(np.int64)
    yab = oracle.dedisperse(A + B, D, 500).astype(np.int64)
    assert np.array_equal(ya + yb, yab)


def test_zero_outside_bounds():
    rng = np.random.Generator(np.random.PCG64(11))
    D = np.array([[0, 3, 6]], np.int32)
    X = rng.integers(1, 256, size=(3, 10), dtype=np.uint8)
    Y = oracle.dedisperse(X, D, 10, nsamp_in=10)
    # sample t = 9: only channel 0 is inside (9 + 3 and 9 + 6 fall past the end)
    assert Y[0, 9] == X[0, 9]
    assert Y[0, 5] == int(X[0, 5]) + int(X[1, 8])


def test_pulse_on_rounded_delays_gives_exact_peak():
    # A top-hat of height A, w samples long, laid on trial d*'s rounded delays.
    wl = SINGLE_BEAM
    D = oracle.delays(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, wl.dms())
    dstar, t0, w, A = 300, 1000, 8, 40
    nsamp = wl.nout + int(D.max())
    X = np.zeros((wl.nchan, nsamp), np.uint8)
    for c in range(wl.nchan):
        X[c, t0 + D[dstar, c]: t0 + D[dstar, c] + w] = A
    Y = oracle.dedisperse(X, D[[dstar - 1, dstar, dstar + 1]], wl.nout)
    assert np.all(Y[1, t0:t0 + w] == A * wl.nchan)
    assert Y[1].max() == A * wl.nchan and Y[0].max() < A * wl.nchan and Y[2].max() < A * wl.nchan


def test_max_value_fits_u32():
    D = np.zeros((1, 300), np.int32)
    X = np.full((300, 4), 255, np.uint8)
    assert np.all(oracle.dedisperse(X, D, 4) == 255 * 300)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_row_checksums_match_brute_force(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    nchan, ndm, nout = 9, 7, 50
    D = np.sort(rng.integers(0, 30, size=(ndm, nchan)).astype(np.int32), axis=0)
    nsamp = nout + 20  # some rows run past the end: zero-padded
    X = rng.integers(0, 256, size=(nchan, nsamp), dtype=np.uint8)
    want = _brute_python(X, D, nout, nsamp).sum(axis=1)
    assert np.array_equal(oracle.row_checksums(X, D, nout).astype(np.int64), want)
