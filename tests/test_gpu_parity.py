"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bars: dedispersion and statistics bit-exact; S/N within
|g - o| <= 1e-5 max(1, |o|); the best-width index identical wherever the
oracle's two best widths differ by more than that tolerance, otherwise the
GPU's choice must itself reach the oracle's maximum within tolerance;
detection identical on identical planes.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from sps_inputs import synth  # noqa: E402
from sps_inputs.workloads import SINGLE_BEAM, Workload  # noqa: E402

pytestmark = pytest.mark.gpu

SNR_RTOL = 1e-5


@pytest.fixture(scope="module")
def sps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_02328_amd import sps as mod
    mod.library()
    return mod


def to_device_pitched(X: np.ndarray, nsamp_in: int, pad: int = 0) -> torch.Tensor:
    pitch = ((nsamp_in + 15) // 16) * 16 + 16 * pad
    t = torch.zeros((X.shape[0], max(pitch, 16)), dtype=torch.uint8, device="cuda")
    t[:, :nsamp_in] = torch.from_numpy(np.ascontiguousarray(X[:, :nsamp_in])).cuda()
    # garbage in the padding must not be read
    if t.shape[1] > nsamp_in:
        t[:, nsamp_in:] = 0xA5
    return t


def gpu_dedisperse(sps, plan, Xd, nsamp_in, nout, flags=0):
    Y = torch.empty((plan.ndm, nout), dtype=torch.int32, device="cuda")
    sps.sps_dedisperse(plan, Xd, nsamp_in, Y, nout, flags)
    torch.cuda.synchronize()
    return Y.cpu().numpy().view(np.uint32)


def check_snr(snr_g, best_g, snr_o, best_o, s64_all_o=None):
    tol = SNR_RTOL * np.maximum(1.0, np.abs(snr_o.astype(np.float64)))
    err = np.abs(snr_g.astype(np.float64) - snr_o.astype(np.float64))
    assert np.all(err <= tol), f"max S/N error {err.max()}"
    mism = best_g != best_o
    if mism.any():
        # only near-ties may differ: the GPU's width must reach the max within tolerance
        assert s64_all_o is not None, f"{mism.sum()} best-width mismatches"
        idx = np.nonzero(mism)
        alt = s64_all_o[best_g[idx].astype(np.int64), idx[0], idx[1]]
        assert np.all(np.abs(alt - snr_o[idx]) <= 2 * tol[idx])


def all_width_snr(Y, st, widths):
    """S/N of every width (oracle formula per width, for near-tie checks)."""
    out = np.full((len(widths),) + Y.shape, -np.inf)
    for i, w in enumerate(widths):
        snr_i, best_i, s64 = oracle.boxcar(Y, st, [w], want_f64=True)
        ok = best_i == 0
        out[i][ok] = s64[ok]
    return out


def test_plan_delays_match_oracle(sps):
    wl = SINGLE_BEAM
    with sps.plan_for(wl) as plan:
        D, mx = sps.sps_plan_delays(plan)
    Do = oracle.delays(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, wl.dms())
    assert np.array_equal(D, Do) and mx == Do.max() == 23364


def test_single_beam_end_to_end(sps):
    wl = SINGLE_BEAM
    Do = oracle.delays(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, wl.dms())
    nsamp = wl.nout + int(Do.max())
    X, truth = synth.make_filterbank(wl, nsamp)
    Yo, sto, snro, besto = oracle.pipeline(X, Do, wl.nout, wl.widths)
    with sps.plan_for(wl) as plan:
        Xd = to_device_pitched(X, nsamp, pad=3)
        Yd = torch.empty((wl.ndm, wl.nout), dtype=torch.int32, device="cuda")
        sps.sps_dedisperse(plan, Xd, nsamp, Yd, wl.nout)
        snr = torch.empty((wl.ndm, wl.nout), dtype=torch.float32, device="cuda")
        best = torch.empty((wl.ndm, wl.nout), dtype=torch.uint8, device="cuda")
        st = torch.empty((wl.ndm, 2), dtype=torch.int32, device="cuda")
        sps.sps_boxcar_snr(plan, Yd, wl.nout, wl.widths, snr, best, st)
        cands, n = sps.sps_detect(plan, snr, best, wl.nout, wl.widths, 8.0, 64, 4096, 16, 128)
        torch.cuda.synchronize()
        Yg = Yd.cpu().numpy().view(np.uint32)
        assert np.array_equal(Yg, Yo), "dedispersion differs"
        assert np.array_equal(st.cpu().numpy().astype(np.int64), sto), "row stats differ"
        check_snr(snr.cpu().numpy(), best.cpu().numpy(), snro, besto,
                  all_width_snr(Yo, sto, wl.widths))
    co = oracle.detect(snro, besto, 8.0, 64, 4096, 16, 128)
    assert n == co["n_found"]
    assert list(cands["dm_idx"]) == list(co["d"]) and list(cands["t_idx"]) == list(co["t"])
    assert list(cands["width"]) == [wl.widths[i] for i in co["w"]]
    assert np.allclose(cands["snr"], co["snr"], rtol=SNR_RTOL)
    top = cands[0]
    assert top["dm_idx"] in (153, 154) and abs(top["toa_s"] - truth.pulses[0].toa_s) < 0.2


def _random_case(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    nchan = int(rng.choice([1, 2, 3, 15, 16, 17, 31, 255, 256, 257, 300, 513]))
    ndm = int(rng.choice([1, 2, 5, 15, 16, 17, 33, 40]))
    nout = int(rng.choice([1, 3, 7, 64, 255, 1279, 1280, 1281, 2560, 3001, 5000]))
    f_hi = float(rng.uniform(400, 2000))
    f_lo = f_hi * float(rng.uniform(0.5, 0.95))
    tsamp = float(rng.choice([64e-6, 98.304e-6, 2.56e-4, 1e-3]))
    dm_hi = float(rng.uniform(0, 300))
    wl = Workload("rand", nchan, f_lo, f_hi, tsamp, nout, ndm, 0.0, dm_hi, (1,))
    return rng, wl


@pytest.mark.parametrize("seed", range(24))
def test_dedisperse_random_shapes_bitexact(sps, seed):
    rng, wl = _random_case(seed)
    Do = oracle.delays(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, wl.dms())
    full = wl.nout + int(Do.max())
    zero_pad = seed % 3 == 0
    nsamp = max(1, full - int(rng.integers(0, full))) if zero_pad else full + int(rng.integers(0, 5))
    X = synth.random_bytes(wl.nchan, nsamp, seed=seed + 100)
    if seed % 4 == 1:
        X[:, :] = 255  # largest sums
    Yo = oracle.dedisperse(X, Do, wl.nout, nsamp)
    try:
        plan = sps.plan_for(wl)
    except sps.SpsError as e:
        pytest.skip(f"plan refused: {e}")
    with plan:
        Yg = gpu_dedisperse(sps, plan, to_device_pitched(X, nsamp, pad=seed % 2), nsamp, wl.nout,
                            sps.SPS_ZERO_PAD if zero_pad else 0)
    assert np.array_equal(Yg, Yo)


@pytest.mark.parametrize("seed", range(6))
def test_dedisperse_every_tiling_bitexact(sps, seed):
    # every compiled tiling on shapes with partial slabs (channel counts off
    # the 8- and 16-channel slabs), partial DM blocks and ragged time tiles;
    # the staged delay table is rebuilt for each tiling
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    nchan = int([7, 17, 40, 129, 263, 9][seed])
    ndm = int(rng.choice([3, 9, 17, 23]))
    nout = int(rng.choice([700, 1281, 3001, 4099]))
    # small delay spreads fit the short staged rows; larger ones need the
    # tilings with longer rows (4, 5 and 8 KB)
    dm_hi = [12.0, 150.0, 10.0, 250.0, 7.0, 420.0][seed]
    wl = Workload("tiles", nchan, 1100.0, 1500.0, 98.304e-6, nout, ndm, 0.0, dm_hi, (1,))
    Do = oracle.delays(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, wl.dms())
    nsamp = nout + int(Do.max()) - (int(rng.integers(0, 50)) if seed % 2 else 0)
    X = synth.random_bytes(nchan, nsamp, seed=seed + 500)
    Yo = oracle.dedisperse(X, Do, nout, nsamp)
    Xd = to_device_pitched(X, nsamp, pad=1)
    tried = set()
    with sps.plan_for(wl) as plan:
        for i in range(sps.sps_tiling_count()):
            t = sps.sps_tiling_describe(i)
            try:
                sps.sps_plan_set_tiling(plan, t["m"], t["dpw"], t["nw"], t["cs"],
                                        t["waves_per_eu"])
            except sps.SpsError as e:
                assert e.name == "SPS_ERR_RANGE"  # rows too long for this tiling
                continue
            got = sps.sps_plan_get_tiling(plan)
            assert (got["m"], got["cs"], got["waves_per_eu"]) == (t["m"], t["cs"], t["waves_per_eu"])
            Yg = gpu_dedisperse(sps, plan, Xd, nsamp, nout, sps.SPS_ZERO_PAD)
            assert np.array_equal(Yg, Yo), got
            tried.add(tuple(sorted(got.items())))
        sps.sps_plan_set_tiling(plan, 0, 0, 0, 0, 0)  # the plain kernel
        assert np.array_equal(gpu_dedisperse(sps, plan, Xd, nsamp, nout, sps.SPS_ZERO_PAD), Yo)
    assert tried


def test_dedisperse_strict_mode_rejects_short_input(sps):
    wl = SINGLE_BEAM
    with sps.plan_for(wl) as plan:
        _, mx = sps.sps_plan_delays(plan)
        Xd = torch.zeros((wl.nchan, 16 * ((wl.nout + mx + 15) // 16)), dtype=torch.uint8,
                         device="cuda")
        Y = torch.empty((wl.ndm, wl.nout), dtype=torch.int32, device="cuda")
        with pytest.raises(sps.SpsError) as ei:
            sps.sps_dedisperse(plan, Xd, wl.nout + mx - 1, Y, wl.nout)
        assert ei.value.name == "SPS_ERR_RANGE"
        sps.sps_dedisperse(plan, Xd, wl.nout + mx, Y, wl.nout)  # exactly enough
        torch.cuda.synchronize()


@pytest.mark.parametrize("seed", range(8))
def test_stats_and_boxcar_random(sps, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    nchan = int(rng.choice([4, 64, 256, 4096]))
    ndm = int(rng.choice([1, 3, 8]))
    nout = int(rng.choice([1, 2, 5, 100, 4095, 4096, 4097, 10000]))
    wmax_pow = int(rng.integers(0, 9))
    widths = [2 ** i for i in range(wmax_pow + 1) if 2 ** i <= nout]
    if seed % 2:
        widths = sorted(set([1, 3, 5, 7, 12, 100]) & set(range(1, nout + 1))) or [1]
    Y = rng.integers(0, 255 * nchan + 1, size=(ndm, nout)).astype(np.uint32)
    if seed % 3 == 0:
        Y[0] = rng.integers(1000, 1003, size=nout)  # heavy ties
    if seed == 4:
        Y[-1] = 77  # MAD = 0
    sto = oracle.stats(Y)
    snro, besto = oracle.boxcar(Y, sto, widths)
    wl = Workload("s", nchan, 1000.0, 1500.0, 1e-4, nout, ndm, 0.0, 1.0, tuple(widths))
    with sps.plan_for(wl) as plan:
        Yd = torch.from_numpy(Y.view(np.int32)).cuda()
        snr = torch.empty((ndm, nout), dtype=torch.float32, device="cuda")
        best = torch.empty((ndm, nout), dtype=torch.uint8, device="cuda")
        st = torch.empty((ndm, 2), dtype=torch.int32, device="cuda")
        sps.sps_boxcar_snr(plan, Yd, nout, widths, snr, best, st)
        torch.cuda.synchronize()
        assert np.array_equal(st.cpu().numpy().astype(np.int64), sto)
        check_snr(snr.cpu().numpy(), best.cpu().numpy(), snro, besto, all_width_snr(Y, sto, widths))


@pytest.mark.parametrize("npow,nout", [(1, 4096), (1, 4100), (3, 4), (3, 7), (7, 4096),
                                       (7, 4096 + 62), (7, 4096 + 63), (9, 4096 + 256),
                                       (9, 3 * 4096 - 1), (13, 4097), (13, 2 * 4096 + 4095),
                                       (13, 3 * 4096)])
def test_boxcar_pow2_segment_tails(sps, npow, nout):
    """Power-of-two width lists 1 .. 2^(npow-1) on rows whose last segment
    ends inside, at, or just past the widest window; with a row of ties and
    a row of MAD 0."""
    rng = np.random.Generator(np.random.PCG64(100 * npow + nout % 97))
    ndm, nchan = 4, 256
    widths = [2 ** i for i in range(npow)]
    Y = rng.integers(0, 255 * nchan + 1, size=(ndm, nout)).astype(np.uint32)
    Y[1] = rng.integers(1000, 1003, size=nout)
    Y[2] = 77
    sto = oracle.stats(Y)
    snro, besto = oracle.boxcar(Y, sto, widths)
    wl = Workload("s", nchan, 1000.0, 1500.0, 1e-4, nout, ndm, 0.0, 1.0, tuple(widths))
    with sps.plan_for(wl) as plan:
        Yd = torch.from_numpy(Y.view(np.int32)).cuda()
        snr = torch.empty((ndm, nout), dtype=torch.float32, device="cuda")
        best = torch.empty((ndm, nout), dtype=torch.uint8, device="cuda")
        st = torch.empty((ndm, 2), dtype=torch.int32, device="cuda")
        sps.sps_boxcar_snr(plan, Yd, nout, widths, snr, best, st)
        torch.cuda.synchronize()
        assert np.array_equal(st.cpu().numpy().astype(np.int64), sto)
        check_snr(snr.cpu().numpy(), best.cpu().numpy(), snro, besto, all_width_snr(Y, sto, widths))


def test_boxcar_prefix_near_float_limit(sps):
    """Segments whose window prefix of Y - med peaks just below, at and just
    above +-2^24, where the kernel switches between a float and an integer
    prefix (both exact).  Each row holds med + (+1, -1, 0) repeated (median
    500000, MAD 1, so an S/N computed from a numerator off by one misses the
    bound by far) and, inside its second segment, a plateau that lifts the
    window's prefix to T; outputs after the plateau read prefix values T - 1
    and T, whose odd members a float could not hold past 2^24."""
    nchan, nout, med = 4096, 3 * 4096 + 100, 500000
    widths = [2 ** i for i in range(9)]
    targets = [2 ** 24 - 2, 2 ** 24 - 1, 2 ** 24, 2 ** 24 + 1, 2 ** 24 + 2001, -(2 ** 24 - 2),
               -(2 ** 24 + 1), 2 ** 28]
    Y = np.empty((len(targets), nout), dtype=np.int64)
    base = med + np.tile(np.array([1, -1, 0]), nout // 3 + 1)[:nout]
    t0 = 4096 + 999  # prefix 0 there (a multiple of 3 past the segment start)
    for r, T in enumerate(targets):
        Y[r] = base
        D = 400000 if T > 0 else -400000
        L, R = divmod(abs(T), 400000)
        Y[r, t0:t0 + L] = med + D
        Y[r, t0 + L] = med + (R if T > 0 else -R)
        Y[r, t0 + L + 1:t0 + L + 4] = med  # then the pattern again, prefix T - 1 or T
    assert Y.min() >= 0 and Y.max() <= 255 * nchan
    Y = Y.astype(np.uint32)
    sto = oracle.stats(Y)
    assert np.all(sto[:, 0] == med) and np.all(sto[:, 1] == 1)
    snro, besto = oracle.boxcar(Y, sto, widths)
    wl = Workload("s", nchan, 1000.0, 1500.0, 1e-4, nout, len(targets), 0.0, 1.0, tuple(widths))
    with sps.plan_for(wl) as plan:
        Yd = torch.from_numpy(Y.view(np.int32)).cuda()
        snr = torch.empty(Y.shape, dtype=torch.float32, device="cuda")
        best = torch.empty(Y.shape, dtype=torch.uint8, device="cuda")
        st = torch.empty((len(targets), 2), dtype=torch.int32, device="cuda")
        sps.sps_boxcar_snr(plan, Yd, nout, widths, snr, best, st)
        torch.cuda.synchronize()
        assert np.array_equal(st.cpu().numpy().astype(np.int64), sto)
        check_snr(snr.cpu().numpy(), best.cpu().numpy(), snro, besto, all_width_snr(Y, sto, widths))


@pytest.mark.parametrize("seed", range(6))
def test_detect_same_plane(sps, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    ndm, nout = int(rng.integers(1, 100)), int(rng.integers(1, 20000))
    snr = (rng.standard_normal((ndm, nout)) * 1.5).astype(np.float32)
    snr[rng.integers(0, ndm, 20), rng.integers(0, nout, 20)] = 9.5  # exact ties
    best = rng.integers(0, 3, (ndm, nout)).astype(np.uint8)
    widths = [1, 2, 4]
    td, tt = int(rng.integers(1, 70)), int(rng.integers(1, 5000))
    rd, rt = int(rng.integers(0, 20)), int(rng.integers(0, 300))
    co = oracle.detect(snr, best, 6.0, td, tt, rd, rt, cap=100000)
    wl = Workload("d", 8, 1000.0, 1500.0, 1e-4, nout, ndm, 0.0, 10.0, (1,))
    with sps.plan_for(wl) as plan:
        cands, n = sps.sps_detect(plan, torch.from_numpy(snr).cuda(), torch.from_numpy(best).cuda(),
                                  nout, widths, 6.0, td, tt, rd, rt, cap=8192)
    assert n == co["n_found"]
    assert np.array_equal(cands["dm_idx"], co["d"]) and np.array_equal(cands["t_idx"], co["t"])
    assert np.array_equal(cands["snr"], co["snr"])
    assert list(cands["width"]) == [widths[i] for i in co["w"]]
    dms = wl.dms()
    assert np.array_equal(cands["dm"], dms[co["d"]])
    assert np.allclose(cands["toa_s"], (co["t"] + 0.5 * cands["width"]) * wl.tsamp_s, rtol=0, atol=1e-12)


def test_detect_truncation_and_errors(sps):
    ndm, nout = 8, 100
    snr = np.zeros((ndm, nout), np.float32)
    snr[0, 5] = snr[4, 50] = snr[7, 99] = 20.0
    best = np.zeros((ndm, nout), np.uint8)
    wl = Workload("d", 8, 1000.0, 1500.0, 1e-4, nout, ndm, 0.0, 10.0, (1,))
    with sps.plan_for(wl) as plan:
        s, b = torch.from_numpy(snr).cuda(), torch.from_numpy(best).cuda()
        cands, n = sps.sps_detect(plan, s, b, nout, [1], 10.0, 4, 10, 0, 0, cap=2,
                                  allow_truncated=True)
        assert n == 3 and len(cands) == 2
        with pytest.raises(sps.SpsError) as ei:
            sps.sps_detect(plan, s, b, nout, [1], 10.0, 4, 10, 0, 0, cap=2)
        assert ei.value.name == "SPS_ERR_TRUNCATED"
        with pytest.raises(sps.SpsError) as ei:
            sps.sps_detect(plan, s, b, nout, [1], 0.0, 4, 10, 0, 0)
        assert ei.value.name == "SPS_ERR_INVALID_ARG"


def test_argument_errors(sps):
    wl = SINGLE_BEAM
    with pytest.raises(sps.SpsError) as ei:
        sps.sps_plan_create([1600.0], 1500.0, 1e-4, [1.0])
    assert ei.value.name == "SPS_ERR_INVALID_ARG"
    with pytest.raises(sps.SpsError):
        sps.sps_plan_create([1400.0], 1500.0, 1e-4, [2.0, 1.0])  # descending DMs
    with sps.plan_for(wl) as plan:
        Y = torch.empty((wl.ndm, 64), dtype=torch.int32, device="cuda")
        snr = torch.empty((wl.ndm, 64), dtype=torch.float32, device="cuda")
        best = torch.empty((wl.ndm, 64), dtype=torch.uint8, device="cuda")
        for widths, name in (([2, 1], "SPS_ERR_INVALID_ARG"), ([0], "SPS_ERR_INVALID_ARG"),
                             ([1, 128], "SPS_ERR_RANGE")):
            with pytest.raises(sps.SpsError) as ei:
                sps.sps_boxcar_snr(plan, Y, 64, widths, snr, best)
            assert ei.value.name == name
        X = torch.zeros((wl.nchan, 40000), dtype=torch.uint8, device="cuda")
        X2 = torch.zeros((wl.nchan, 40001), dtype=torch.uint8, device="cuda")
        with pytest.raises(sps.SpsError) as ei:  # pitch not a multiple of 16
            sps.sps_dedisperse(plan, X2, 40000, Y, 64)
        assert ei.value.name == "SPS_ERR_INVALID_ARG"
        with pytest.raises(sps.SpsError) as ei:
            sps.sps_dedisperse(plan, X, 40000, Y, 64, flags=2)
        assert ei.value.name == "SPS_ERR_INVALID_ARG"


@pytest.mark.parametrize("radius", [(1, 1), (2, 3), (10, 10)])
def test_detect_dense_chains(sps, radius):
    # one offer per element: long suppression chains; (10, 10) forces the
    # one-by-one scan, the others the parallel rounds
    rng = np.random.Generator(np.random.PCG64(sum(radius)))
    ndm, nout = 40, 200
    snr = (10 + rng.standard_normal((ndm, nout))).astype(np.float32)
    snr[5, 5:60] = 20.0 - np.arange(55, dtype=np.float32) * 0.1  # a ridge of decreasing peaks
    best = np.zeros((ndm, nout), np.uint8)
    rd, rt = radius
    co = oracle.detect(snr, best, 8.0, 1, 1, rd, rt, cap=100000)
    wl = Workload("d", 8, 1000.0, 1500.0, 1e-4, nout, ndm, 0.0, 10.0, (1,))
    with sps.plan_for(wl) as plan:
        cands, n = sps.sps_detect(plan, torch.from_numpy(snr).cuda(), torch.from_numpy(best).cuda(),
                                  nout, [1], 8.0, 1, 1, rd, rt, cap=8192)
    assert n == co["n_found"]
    assert np.array_equal(cands["dm_idx"], co["d"]) and np.array_equal(cands["t_idx"], co["t"])


@pytest.mark.parametrize("case", ["noise", "narrow", "near_zero", "near_top", "constant",
                                  "wide_mad", "spread", "bimodal", "spikes"])
@pytest.mark.parametrize("nout", [1, 2, 3, 5, 64, 1023, 3001, 4095, 4096, 4097])
def test_stats_short_rows(sps, case, nout):
    """Rows of at most 4096 values take the short-row form: a window of
    unit bins around the row mean, with the exact radix fallback for rows it
    cannot hold (a spread far wider than the window, two clusters far from
    their mean, a MAD wider than the window's half).  Odd lengths leave every
    row after the first unaligned; 4097 takes the long-row form on the same
    shapes."""
    rng = np.random.Generator(np.random.PCG64(1000 * nout + len(case)))
    nchan, ndm = 4096, 5
    vmax = 255 * nchan
    if case == "noise":
        Y = rng.normal(32768, 256, (ndm, nout))
    elif case == "narrow":
        Y = rng.normal(300000, 3, (ndm, nout))
    elif case == "near_zero":
        Y = np.abs(rng.normal(0, 700, (ndm, nout)))
    elif case == "near_top":
        Y = vmax - np.abs(rng.normal(0, 900, (ndm, nout)))
    elif case == "constant":
        Y = np.full((ndm, nout), 123457.0)
    elif case == "wide_mad":   # MAD near or past the window's half-width
        Y = rng.normal(500000, 3100, (ndm, nout))
    elif case == "spread":
        Y = rng.uniform(0, vmax, (ndm, nout))
    elif case == "bimodal":
        centre = rng.choice([100000, 900000], size=(ndm, nout))
        Y = centre + rng.integers(-5, 6, size=(ndm, nout))
    else:                      # noise with a few huge samples pulling the mean
        Y = rng.normal(400000, 300, (ndm, nout))
        Y[:, ::97] += 600000
    Y = np.clip(np.rint(Y), 0, vmax).astype(np.uint32)
    sto = oracle.stats(Y)
    wl = Workload("s", nchan, 1000.0, 1500.0, 1e-4, nout, ndm, 0.0, 1.0, (1,))
    with sps.plan_for(wl) as plan:
        snr = torch.empty((ndm, nout), dtype=torch.float32, device="cuda")
        best = torch.empty((ndm, nout), dtype=torch.uint8, device="cuda")
        st = torch.empty((ndm, 2), dtype=torch.int32, device="cuda")
        sps.sps_boxcar_snr(plan, torch.from_numpy(Y.view(np.int32)).cuda(), nout, [1], snr,
                           best, st)
        torch.cuda.synchronize()
        assert np.array_equal(st.cpu().numpy().astype(np.int64), sto)


@pytest.mark.parametrize("case", ["noise", "narrow", "near_zero", "near_top", "spiky", "step",
                                  "trimodal", "short"])
def test_stats_windowed_rows(sps, case):
    """Rows whose sampled window holds the median and the MAD (noise, narrow,
    windows clipped at 0 and past the top), a row whose sample misleads (a
    step whose lower 45 % hold half the sampled runs) and one whose MAD lies
    far outside the window (three narrow clusters): the last two are decided
    by the exact fallback reads."""
    rng = np.random.Generator(np.random.PCG64(len(case)))
    nchan, ndm, nout = 4096, 6, 50000
    vmax = 255 * nchan
    if case == "noise":
        Y = rng.normal(524288, 1024, (ndm, nout))
    elif case == "narrow":
        Y = rng.normal(300000, 3, (ndm, nout))
    elif case == "near_zero":
        Y = np.abs(rng.normal(0, 700, (ndm, nout)))
    elif case == "near_top":
        Y = vmax - np.abs(rng.normal(0, 900, (ndm, nout)))
    elif case == "spiky":
        Y = rng.normal(500000, 800, (ndm, nout))
        Y[:, ::7] += rng.uniform(0, 200000, Y[:, ::7].shape)
    elif case == "step":
        Y = rng.normal(500000, 50, (ndm, nout))
        Y[:, :nout * 45 // 100] = rng.normal(100000, 50, (ndm, nout * 45 // 100))
    elif case == "trimodal":
        centre = rng.choice([100000, 500000, 900000], p=[0.35, 0.3, 0.35], size=(ndm, nout))
        Y = centre + rng.integers(-5, 6, size=(ndm, nout))
    else:  # shorter than the sample: the whole row is the sample
        nout = 3001
        Y = rng.normal(400000, 2000, (ndm, nout))
    Y = np.clip(np.rint(Y), 0, vmax).astype(np.uint32)
    sto = oracle.stats(Y)
    wl = Workload("s", nchan, 1000.0, 1500.0, 1e-4, nout, ndm, 0.0, 1.0, (1, 2, 4))
    with sps.plan_for(wl) as plan:
        snr = torch.empty((ndm, nout), dtype=torch.float32, device="cuda")
        best = torch.empty((ndm, nout), dtype=torch.uint8, device="cuda")
        st = torch.empty((ndm, 2), dtype=torch.int32, device="cuda")
        sps.sps_boxcar_snr(plan, torch.from_numpy(Y.view(np.int32)).cuda(), nout, [1, 2, 4], snr,
                           best, st)
        torch.cuda.synchronize()
        assert np.array_equal(st.cpu().numpy().astype(np.int64), sto)
