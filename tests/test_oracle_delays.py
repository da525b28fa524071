"""Pins for the oracle's integer delay table (Sec. 2.3, Eq. KDM / coarse_delay).

The checks come from outside the oracle: the physical dispersion constant
from CODATA constants, the textbook 4.15 ms GHz^-2 rule, exact rational
arithmetic, hand-worked tiny cases and the monotonicity the law implies.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.constants as sc

import oracle
from sps_inputs.workloads import FULL_SCALE, SINGLE_BEAM

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def _table(wl):
    return oracle.delays(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, wl.dms())


def test_constant_matches_cold_plasma_physics():
    # e^2 / (8 pi^2 eps0 m_e c) in SI, converted to s MHz^2 per (pc cm^-3):
    # the physical law behind Eq. (phys_delay).  The printed K_DM (read in
    # seconds) must agree to 1e-4; a ms reading would be off by 1e3.
    k_si = sc.e ** 2 / (8 * math.pi ** 2 * sc.epsilon_0 * sc.m_e * sc.c)
    k_phys = k_si * (sc.parsec * 1e6) / 1e12
    paper = json.load(open(GOLDEN))["K_DM"]["value"]
    assert abs(paper - k_phys) / k_phys < 1e-4
    # And the oracle uses it in those units: one channel, DM 1, t_samp 1 us.
    f = np.array([1000.0])
    D = oracle.delays(f, 1500.0, 1e-6, np.array([1.0]))
    want = k_phys * (1 / 1000.0 ** 2 - 1 / 1500.0 ** 2) / 1e-6
    assert abs(int(D[0, 0]) - want) <= 0.5 + 1e-4 * want


def test_ghz_rule_of_thumb_full_band():
    # 4.148808 ms * DM * (f_GHz^-2 - f_ref,GHz^-2), the GHz form of Eq. (KDM).
    wl = SINGLE_BEAM
    D = _table(wl)
    f_ghz = wl.freqs_mhz() / 1e3
    for d in (1, 100, 511):
        dm = wl.dms()[d]
        want = 4.148808e-3 * dm * (1 / f_ghz ** 2 - 1 / 1.5 ** 2) / wl.tsamp_s
        assert np.all(np.abs(D[d] - want) <= 0.5 + 1e-9 * want)
    # DM 1000 across 1000-1500 MHz: 4.148808 ms * 1000 * (1 - 1/2.25) = 2.3049 s
    assert abs(D[511, -1] * wl.tsamp_s - 2.3049) < 0.01


def _exact_rounded(K, dm, tsamp, f, fref):
    x = K * Fraction(dm) / Fraction(tsamp) * (1 / Fraction(f) ** 2 - 1 / Fraction(fref) ** 2)
    r = math.floor(x + Fraction(1, 2))
    return r, abs(x - Fraction(2 * math.floor(x) + 1, 2))


@pytest.mark.parametrize("wl", [SINGLE_BEAM, FULL_SCALE], ids=["single_beam", "full_scale"])
def test_exact_rational_rounding_sampled(wl):
    # Rounding computed exactly from the double inputs (no floating point).
    D = _table(wl)
    K = Fraction(4148.808)
    rng = np.random.Generator(np.random.PCG64(7))
    ds = rng.integers(0, wl.ndm, 300)
    cs = rng.integers(0, wl.nchan, 300)
    f = wl.freqs_mhz()
    dms = wl.dms()
    for d, c in zip(ds, cs):
        r, tie_dist = _exact_rounded(K, dms[d], wl.tsamp_s, f[c], wl.fref_mhz)
        assert D[d, c] == r
        assert tie_dist > 1e-9  # fp64 evaluation is far from any tie


def test_exact_rational_rounding_full_single_beam_bottom_and_top():
    wl = SINGLE_BEAM
    D = _table(wl)
    K = Fraction(4148.808)
    f = wl.freqs_mhz()
    dms = wl.dms()
    for c in (0, 1, wl.nchan // 2, wl.nchan - 2, wl.nchan - 1):
        for d in range(wl.ndm):
            r, _ = _exact_rounded(K, dms[d], wl.tsamp_s, f[c], wl.fref_mhz)
            assert D[d, c] == r


def test_spot_values():
    # Largest delays and per-step increments of the two workloads.
    D1 = _table(SINGLE_BEAM)
    assert D1.max() == D1[-1, -1] == 23364
    assert D1[-1, 0] == 24                       # top channel at DM 1000
    assert np.diff(D1[:, -1]).max() == 46
    D2 = _table(FULL_SCALE)
    assert D2.max() == D2[-1, -1] == 95969
    assert np.diff(D2[:, -1]).max() == 47


def test_round_not_truncate_hand_worked():
    # f = 1 MHz, f_ref = 2 MHz: 1/f^2 - 1/f_ref^2 = 3/4 exactly.
    # t_samp = K/2, DM = 1: K DM / t_samp = 2 exactly, so x = 1.5 -> 2.
    K = 4148.808
    D = oracle.delays(np.array([1.0]), 2.0, K / 2, np.array([1.0]))
    assert D[0, 0] == 2
    # t_samp = K: x = 0.75 -> 1 (truncation would give 0).
    D = oracle.delays(np.array([1.0]), 2.0, K, np.array([1.0]))
    assert D[0, 0] == 1
    # t_samp = 4K: x = 0.1875 -> 0.
    D = oracle.delays(np.array([1.0]), 2.0, 4 * K, np.array([1.0]))
    assert D[0, 0] == 0


def test_structure_of_the_law():
    D = _table(SINGLE_BEAM)
    assert np.all(D[0] == 0)                     # DM = 0
    assert np.all(np.diff(D, axis=0) >= 0)       # non-decreasing in DM
    assert np.all(np.diff(D, axis=1) >= 0)       # channel 0 at the top: non-decreasing with c
    # a channel exactly at f_ref has zero delay at every DM
    Dz = oracle.delays(np.array([1500.0, 1200.0]), 1500.0, 1e-4, np.array([0.0, 500.0, 3000.0]))
    assert np.all(Dz[:, 0] == 0)
    # linear in DM before rounding: D(2 DM) within 1 of 2 D(DM)
    Dh = oracle.delays(SINGLE_BEAM.freqs_mhz(), 1500.0, 1e-4, np.array([250.0, 500.0]))
    assert np.all(np.abs(Dh[1] - 2 * Dh[0]) <= 1)


def test_rejects_channels_above_reference():
    with pytest.raises(ValueError):
        oracle.delays(np.array([1600.0]), 1500.0, 1e-4, np.array([1.0]))
    with pytest.raises(ValueError):
        oracle.delays(np.array([1400.0]), 1500.0, 0.0, np.array([1.0]))
    with pytest.raises(ValueError):
        oracle.delays(np.array([1400.0]), 1500.0, 1e-4, np.array([-1.0]))
