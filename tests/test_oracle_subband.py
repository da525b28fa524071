"""Pins for the oracle's version of the paper's own method (Sec. 2.3 subband
dedispersion) and of the pre-dedispersion steps (zero-DM filter, square-law
downsampling, Sec. 2.1-2.2).

Subband: with N0 = 1 the residuals vanish and the method must equal brute
force exactly (Eq. residual with dDM = 0); for any N0 it must equal brute
force run with the effective per-channel delay D_j(m),c + R_m,s (stage 1 and
stage 2 are a regrouping of one shift-and-sum); the residuals follow
Eq. (residual) exactly (rational arithmetic); and the effective delays stay
within the smearing estimate of Eq. (sb_smear) plus rounding.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from sps_inputs import synth
from sps_inputs.workloads import SINGLE_BEAM

K = 4148.808


def _setup(wl, nsub, n0, ndm=None):
    ndm = ndm or wl.ndm
    ddm = (wl.dm_hi - wl.dm_lo) / (wl.ndm - 1)
    sub = oracle.equal_subbands(wl.nchan, nsub)
    R, F, dmc = oracle.subband_residuals(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, sub, ndm,
                                         wl.dm_lo, ddm, n0)
    Dc = oracle.delays(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, dmc)
    return sub, R, F, dmc, Dc, ddm


def _effective(Dc, sub, R, n0):
    ndm, nsub = R.shape
    nchan = Dc.shape[1]
    s_of_c = np.repeat(np.arange(nsub), np.diff(sub))
    j = np.arange(ndm) // n0
    return (Dc[j] + R[:, s_of_c]).astype(np.int32)


@pytest.mark.parametrize("nsub", [1, 4, 16, 256])
def test_n0_one_is_brute_force(nsub):
    wl = SINGLE_BEAM
    sub, R, F, dmc, Dc, ddm = _setup(wl, nsub, 1, ndm=64)
    assert np.all(R == 0)
    D = oracle.delays(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, wl.dms()[:64])
    assert np.array_equal(Dc, D)
    nsamp = 600 + int(D.max())
    X = synth.random_bytes(wl.nchan, nsamp, seed=nsub)
    assert np.array_equal(oracle.subband_dedisperse(X, Dc, sub, R, 1, 600),
                          oracle.dedisperse(X, D, 600))


@pytest.mark.parametrize("nsub,n0", [(8, 4), (32, 8), (16, 3), (5, 16)])
def test_regrouping_identity(nsub, n0):
    # stage 1 + stage 2 == one shift-and-sum with the effective delays
    wl = SINGLE_BEAM
    sub, R, F, dmc, Dc, ddm = _setup(wl, nsub, n0, ndm=96)
    Deff = _effective(Dc, sub, R, n0)
    nsamp = 500 + int(Deff.max()) - 37  # some outputs run past the end
    X = synth.random_bytes(wl.nchan, nsamp, seed=n0)
    assert np.array_equal(oracle.subband_dedisperse(X, Dc, sub, R, n0, 500),
                          oracle.dedisperse(X, Deff, 500))


def test_residuals_exact_and_structure():
    wl = SINGLE_BEAM
    nsub, n0 = 16, 8
    sub, R, F, dmc, Dc, ddm = _setup(wl, nsub, n0)
    f = wl.freqs_mhz()
    m = np.arange(wl.ndm)
    assert np.all(R[m % n0 == 0] == 0)
    assert np.all(R >= 0)
    assert np.all(np.diff(R.reshape(-1, n0, nsub)[: wl.ndm // n0], axis=1) >= 0)
    # F_s: 1/F^2 is the mean of 1/f^2 over the subband
    for s in range(nsub):
        fc = f[sub[s]:sub[s + 1]]
        assert abs(1 / F[s] ** 2 - np.mean(1 / fc ** 2)) < 1e-18
        assert fc.min() <= F[s] <= fc.max()
    # Eq. (residual) in exact rational arithmetic from the double inputs, with
    # 1/F_s^2 the exact mean of 1/f_c^2
    rng = np.random.Generator(np.random.PCG64(3))
    fref2 = Fraction(wl.fref_mhz) ** 2
    inv = [sum(1 / Fraction(float(fc)) ** 2 for fc in f[sub[s]:sub[s + 1]]) / (sub[s + 1] - sub[s])
           for s in range(nsub)]
    for mm, s in zip(rng.integers(0, wl.ndm, 300), rng.integers(0, nsub, 300)):
        dm_m = Fraction(wl.dm_lo + float(mm) * ddm)
        dm_j = Fraction(wl.dm_lo + float((mm // n0) * n0) * ddm)
        x = Fraction(K) * (dm_m - dm_j) / Fraction(wl.tsamp_s) * (inv[s] - 1 / fref2)
        tie = abs(x - Fraction(2 * math.floor(x) + 1, 2))
        if tie > Fraction(1, 10 ** 9):
            assert int(R[mm, s]) == math.floor(x + Fraction(1, 2))


@pytest.mark.parametrize("nsub,n0", [(16, 4), (32, 8), (64, 16)])
def test_smearing_bound(nsub, n0):
    # |effective delay - brute-force delay| <= Eq. (sb_smear) / t_samp + rounding
    wl = SINGLE_BEAM
    sub, R, F, dmc, Dc, ddm = _setup(wl, nsub, n0)
    D = oracle.delays(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, wl.dms())
    Deff = _effective(Dc, sub, R, n0)
    f = wl.freqs_mhz()
    bw = (wl.f_hi_mhz - wl.f_lo_mhz) / wl.nchan
    dDM = (np.arange(wl.ndm) % n0) * ddm
    worst = 0.0
    for s in range(nsub):
        cs = slice(sub[s], sub[s + 1])
        width = (sub[s + 1] - sub[s]) * bw            # the subband width Delta f_s
        smear = 2 * K * dDM * width / F[s] ** 3 / wl.tsamp_s
        err = np.abs(Deff[:, cs].astype(np.int64) - D[:, cs]).max(axis=1)
        assert np.all(err <= 1.05 * smear + 1.5)
        worst = max(worst, float(err.max()))
    assert worst >= 1  # the approximation is not exact for N0 > 1


def test_subband_finds_the_pulse():
    wl = SINGLE_BEAM
    sub, R, F, dmc, Dc, ddm = _setup(wl, 32, 4)
    Deff = _effective(Dc, sub, R, 4)
    nsamp = wl.nout + int(Deff.max())
    X, truth = synth.make_filterbank(wl, nsamp)
    Y = oracle.subband_dedisperse(X, Dc, sub, R, 4, wl.nout)
    st = oracle.stats(Y)
    snr, best = oracle.boxcar(Y, st, wl.widths)
    d, t = np.unravel_index(np.argmax(snr), snr.shape)
    assert abs(wl.dms()[d] - 300) < 20 and abs(t - 2000) < 40 and snr[d, t] > 150


def test_zero_dm_removes_broadband_series():
    rng = np.random.Generator(np.random.PCG64(5))
    nchan, n = 37, 300
    a = rng.integers(60, 120, nchan)
    b = rng.integers(0, 100, n)
    X = (a[:, None] + b[None, :]).astype(np.uint8)
    Z = oracle.zero_dm(X)
    # m(t) = b_t + round-half-up(mean a): every column becomes a - round(mean a) + 128
    ma = (int(a.sum()) + nchan // 2) // nchan
    assert np.all(Z == (a - ma + 128)[:, None])
    # one channel: everything becomes the mid-level
    assert np.all(oracle.zero_dm(X[:1]) == 128)
    # clipping at both ends
    Y = np.zeros((2, 4), np.uint8)
    Y[0] = 255
    z = oracle.zero_dm(Y)
    assert np.all(z[0] == 255) and np.all(z[1] == 0)  # m = 128: 255-128+128, 0-128+128


def test_downsample_closed_forms():
    n = 64
    for v, want in ((0, 0), (255, 255), (128, 181), (1, 16), (64, 128)):
        X = np.full((2, n), v, np.uint8)
        for fct in (1, 2, 7, 64):
            out = oracle.downsample_sqrt(X, fct)
            assert out.shape == (2, n // fct)
            assert np.all(out == want), (v, fct)
    # exact tie: N = 4, S = 255 -> sqrt(255 * 255 / 4) = 127.5 -> rounds up to 128
    X = np.array([[64, 64, 64, 63]], np.uint8)
    assert oracle.downsample_sqrt(X, 4)[0, 0] == 128
    # V sqrt(S) / sqrt(N V) == sqrt(V S / N): against numpy on random bins
    rng = np.random.Generator(np.random.PCG64(9))
    X = rng.integers(0, 256, (5, 999), dtype=np.uint8)
    for fct in (1, 3, 8):
        nb = 999 // fct
        S = X[:, :nb * fct].reshape(5, nb, fct).astype(np.int64).sum(axis=2)
        ref = np.minimum(np.floor(255 * np.sqrt(S) / np.sqrt(fct * 255) + 0.5), 255)
        got = oracle.downsample_sqrt(X, fct).astype(np.int64)
        assert np.abs(got - ref).max() <= 1 and np.mean(got == ref) > 0.999
