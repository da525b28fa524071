"""GPU parity of sps_search, the one-call search whose boxcar pass also
gathers the tile maxima (Sec. 1 step iii; Sec. 2, candidate record):
statistics identical to the oracle, S/N within 1e-5 relative (near-tie
width rule), and candidates identical to the oracle's tile / threshold /
greedy-suppression rule on the S/N plane the call wrote.  Tilings cover a
tile length that is a multiple of the boxcar segment (one reduction per
segment), tile lengths that cut segments (per-thread merges), one-sample
tiles, tile lengths of whole waves (one merge per wave and column), ragged
rows and rows of MAD 0.  The search without planes (each tile key carries
its peak's width) must give the same statistics and the same candidates on
every tiling, and on tiles that use every bit of the key's position field."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from _checks import check_candidates_exact, check_snr  # noqa: E402
from sps_inputs import synth  # noqa: E402
from sps_inputs.workloads import SINGLE_BEAM, Workload  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_02328_amd import sps as mod
    mod.library()
    return mod


def _run(sps, plan, Yd, nout, widths, ndm, args, cap=1 << 20):
    snr = torch.empty((ndm, nout), dtype=torch.float32, device="cuda")
    best = torch.empty((ndm, nout), dtype=torch.uint8, device="cuda")
    st = torch.empty((ndm, 2), dtype=torch.int32, device="cuda")
    cands, n = sps.sps_search(plan, Yd, nout, widths, snr, best, st, *args, cap=cap)
    torch.cuda.synchronize()
    return cands, n, snr, best, st


def test_single_beam_search(sps):
    wl = SINGLE_BEAM
    args = (8.0, 64, 4096, 16, 128)
    with sps.plan_for(wl) as plan:
        D, dmax = sps.sps_plan_delays(plan)
        nsamp = wl.nout + dmax
        X, _ = synth.make_filterbank(wl, nsamp)
        pitch = (nsamp + 15) // 16 * 16
        Xd = torch.zeros((wl.nchan, pitch), dtype=torch.uint8, device="cuda")
        Xd[:, :nsamp] = torch.from_numpy(X).cuda()
        Y = torch.empty((wl.ndm, wl.nout), dtype=torch.int32, device="cuda")
        sps.sps_dedisperse(plan, Xd, nsamp, Y, wl.nout)
        print("case sps_search single beam", flush=True)
        cands, n, snr, best, st = _run(sps, plan, Y, wl.nout, wl.widths, wl.ndm, args)
        # the separate calls on the same plan give the same candidates
        snr2 = torch.empty_like(snr)
        best2 = torch.empty_like(best)
        sps.sps_boxcar_snr(plan, Y, wl.nout, wl.widths, snr2, best2)
        c2, n2 = sps.sps_detect(plan, snr2, best2, wl.nout, wl.widths, *args, cap=1 << 20)
        torch.cuda.synchronize()
    Yo, sto, _, _ = oracle.pipeline(X, D, wl.nout, wl.widths)
    assert np.array_equal(Y.cpu().numpy().view(np.uint32), Yo)
    assert np.array_equal(st.cpu().numpy().astype(np.int64), sto)
    snr_g, best_g = snr.cpu().numpy(), best.cpu().numpy()
    check_snr(Yo, sto, wl.widths, snr_g, best_g, "single beam")
    co = oracle.detect(snr_g, best_g, *args, cap=1 << 20)
    check_candidates_exact(cands, n, co, wl.widths, "single beam")
    assert n >= 1 and cands["dm_idx"][0] in (153, 154)
    assert n2 == n and np.array_equal(c2, cands)


# (ndm, nout, widths, tile_dm, tile_t, nms_dm, nms_t, threshold)
CASES = [
    (64, 3 * 4096 + 777, (1, 2, 4, 8, 16, 32, 64), 16, 4096, 4, 200, 3.0),     # one reduction per segment
    (40, 2 * 8192 + 5, (1, 2, 4, 8), 7, 8192, 2, 100, 2.5),                     # long tiles, ragged
    (33, 10000, (1, 2, 4, 8, 16), 5, 1000, 3, 50, 2.0),                         # tiles cut segments
    (17, 9000, (1, 3, 5, 7, 12, 100), 4, 256, 1, 20, 2.0),                      # generic widths
    (9, 600, (1, 2, 4), 1, 1, 0, 0, 3.0),                                       # one-sample tiles
    (70, 4096, (1, 2, 4, 8, 16, 32, 64, 128, 256), 64, 4096, 16, 512, 1.5),     # full tiles, many offers
    (5, 1, (1,), 3, 7, 1, 1, 0.5),                                              # one output per row
    (21, 4736, (1, 2, 4, 8, 16, 32, 64), 3, 512, 2, 100, 2.0),                  # tiles of 64-multiples,
    (12, 8192, (1, 3, 5, 7, 12, 100), 4, 192, 1, 30, 2.0),                      # wave-level merges
    (20, 3 * 4096 + 100, (1, 3, 5, 7, 12, 100), 5, 4096, 2, 100, 2.0),         # generic widths,
    (8, 4096 + 2, (3, 5, 7), 3, 4096, 1, 10, 1.0),                              # whole segments; the
]                                                                               # last outputs fit no width


def _case_input(case):
    ndm, nout, widths, td, tt, rd, rt, thr = case
    widths = tuple(w for w in widths if w <= nout)
    rng = np.random.Generator(np.random.PCG64(ndm * 1000 + nout % 997))
    nchan = 256
    Y = rng.integers(0, 255 * nchan + 1, size=(ndm, nout)).astype(np.uint32)
    if ndm > 2:
        Y[1] = rng.integers(1000, 1003, size=nout)  # heavy ties
        Y[2] = 77  # MAD = 0: S/N 0 everywhere
    # a few bright windows so that some tiles clearly lead
    for _ in range(6):
        d, t = int(rng.integers(0, ndm)), int(rng.integers(0, nout))
        Y[d, t:t + 8] = 255 * nchan
    wl = Workload("search", nchan, 1000.0, 1500.0, 1e-4, nout, ndm, 0.0, 1.0, widths)
    return Y, widths, wl, (thr, td, tt, rd, rt)


def _run_no_planes(sps, plan, Yd, nout, widths, ndm, args, cap=1 << 20):
    st = torch.empty((ndm, 2), dtype=torch.int32, device="cuda")
    cands, n = sps.sps_search(plan, Yd, nout, widths, None, None, st, *args, cap=cap)
    torch.cuda.synchronize()
    return cands, n, st


@pytest.mark.parametrize("case", CASES)
def test_search_tilings_match_oracle(sps, case):
    ndm, nout = case[0], case[1]
    Y, widths, wl, args = _case_input(case)
    sto = oracle.stats(Y)
    print(f"case sps_search {case}", flush=True)
    with sps.plan_for(wl) as plan:
        Yd = torch.from_numpy(Y.view(np.int32)).cuda()
        cands, n, snr, best, st = _run(sps, plan, Yd, nout, widths, ndm, args)
        # a second call on the same plan (keys cleared again) gives the same
        c2, n2, _, _, _ = _run(sps, plan, Yd, nout, widths, ndm, args)
    assert np.array_equal(st.cpu().numpy().astype(np.int64), sto)
    snr_g, best_g = snr.cpu().numpy(), best.cpu().numpy()
    check_snr(Y, sto, widths, snr_g, best_g, str(case))
    co = oracle.detect(snr_g, best_g, *args, cap=1 << 20)
    check_candidates_exact(cands, n, co, widths, str(case))
    assert n2 == n and np.array_equal(c2, cands)


@pytest.mark.parametrize("case", CASES)
def test_search_without_planes(sps, case):
    """No S/N or width plane written: the statistics and the candidates
    (positions, widths, S/N, order) equal those of the search with planes,
    whose plane and candidates are held to the oracle here as well."""
    ndm, nout = case[0], case[1]
    Y, widths, wl, args = _case_input(case)
    print(f"case sps_search without planes {case}", flush=True)
    with sps.plan_for(wl) as plan:
        Yd = torch.from_numpy(Y.view(np.int32)).cuda()
        c0, n0, st0 = _run_no_planes(sps, plan, Yd, nout, widths, ndm, args)
        cands, n, snr, best, st = _run(sps, plan, Yd, nout, widths, ndm, args)
        c1, n1, _ = _run_no_planes(sps, plan, Yd, nout, widths, ndm, args)
    sto = oracle.stats(Y)
    assert np.array_equal(st0.cpu().numpy().astype(np.int64), sto)
    snr_g, best_g = snr.cpu().numpy(), best.cpu().numpy()
    check_snr(Y, sto, widths, snr_g, best_g, str(case))
    check_candidates_exact(cands, n, oracle.detect(snr_g, best_g, *args, cap=1 << 20), widths,
                           str(case))
    assert n0 == n and np.array_equal(c0, cands), f"{case}: without planes"
    assert n1 == n and np.array_equal(c1, cands), f"{case}: without planes, second call"


def test_search_without_planes_full_key(sps):
    """Tiles of 16 trials x 2^22 samples (and a ragged second column of 64):
    in-tile positions reach 2^26 - 1, the largest the key's position field
    holds.  The first tile's peak is one bright sample at its last position
    (t = 2^22 - 1, last trial; width 1), above a weaker one near its start;
    the candidates equal those of the search with planes, themselves equal
    to the oracle's rule on that plane."""
    ndm, tt = 16, 1 << 22
    nout = tt + 64
    rng = np.random.Generator(np.random.PCG64(2026))
    Y = rng.integers(0, 1000, size=(ndm, nout)).astype(np.uint32)
    Y[ndm - 1, tt - 1] = 255 * 64     # S/N about 43 at width 1
    Y[3, 100] = 8000                  # about 20
    widths = (1, 2, 4, 8, 16, 32)
    wl = Workload("search", 64, 1000.0, 1500.0, 1e-4, nout, ndm, 0.0, 1.0, widths)
    args = (6.0, ndm, tt, 2, 50)
    print("case sps_search without planes, full key", flush=True)
    with sps.plan_for(wl) as plan:
        Yd = torch.from_numpy(Y.view(np.int32)).cuda()
        del Y
        c0, n0, st0 = _run_no_planes(sps, plan, Yd, nout, widths, ndm, args)
        cands, n, snr, best, st = _run(sps, plan, Yd, nout, widths, ndm, args)
        assert torch.equal(st0, st)
        snr_g, best_g = snr.cpu().numpy(), best.cpu().numpy()
        del snr, best
        co = oracle.detect(snr_g, best_g, *args, cap=1 << 20)
        check_candidates_exact(cands, n, co, widths, "full key")
        assert n == 1 and cands["t_idx"][0] == tt - 1 and cands["dm_idx"][0] == ndm - 1
        assert cands["width"][0] == 1
        assert n0 == n and np.array_equal(c0, cands)
        # one output more per tile does not fit the key: RANGE, nothing run
        with pytest.raises(sps.SpsError, match="RANGE"):
            sps.sps_search(plan, Yd, nout, widths, None, None, st0, 6.0, ndm, tt + 1, 2, 50)


def test_search_planes_together(sps):
    """snr and best_w are NULL together or not at all."""
    Y, widths, wl, args = _case_input(CASES[4])
    with sps.plan_for(wl) as plan:
        Yd = torch.from_numpy(Y.view(np.int32)).cuda()
        snr = torch.empty(Y.shape, dtype=torch.float32, device="cuda")
        with pytest.raises(sps.SpsError, match="INVALID_ARG"):
            sps.sps_search(plan, Yd, Y.shape[1], widths, snr, None, None, *args)
