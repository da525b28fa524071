"""GPU parity of the batched path (many beams of one plan in batched
launches, optionally replayed from a HIP graph) against the oracle on every
beam (planes and statistics bit-exact, S/N within 1e-5 with the near-tie
width rule, candidates identical), with the single-beam calls as an extra
check, and of the autotuner's choice."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from _checks import check_candidates_close, check_candidates_exact, check_snr  # noqa: E402
from sps_inputs import synth  # noqa: E402
from sps_inputs.workloads import SINGLE_BEAM, Workload, PulseModel  # noqa: E402

pytestmark = pytest.mark.gpu

DET = dict(threshold=7.0, tile_dm=16, tile_t=1024, nms_dm=8, nms_t=64)


@pytest.fixture(scope="module")
def sps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_02328_amd import sps as mod
    mod.library()
    return mod


def _wl(nout, seed):
    return Workload("b", 256, 1000.0, 1500.0, 98.304e-6, nout, 64, 0.0, 300.0, (1, 2, 4, 8, 16),
                    pulses=PulseModel(count=2, dm_range=(30.0, 280.0)), seed=seed)


def _beams(sps, plan, nouts, dmax, pad):
    beams = []
    for i, nout in enumerate(nouts):
        wl = _wl(nout, 100 + i)
        nsamp = nout + dmax
        X, _ = synth.make_filterbank(wl, nsamp)
        p = ((nsamp + 15) // 16) * 16 + 16 * pad
        Xd = torch.zeros((wl.nchan, p), dtype=torch.uint8, device="cuda")
        Xd[:, :nsamp] = torch.from_numpy(X).cuda()
        beams.append(dict(X=Xd, Xh=X, nsamp_in=nsamp, nout=nout,
                          Y=torch.zeros((64, nout), dtype=torch.int32, device="cuda"),
                          snr=torch.zeros((64, nout), dtype=torch.float32, device="cuda"),
                          best_w=torch.zeros((64, nout), dtype=torch.uint8, device="cuda"),
                          stats=torch.zeros((64, 2), dtype=torch.int32, device="cuda")))
    return beams


def _single(sps, plan, b, widths):
    Y = torch.empty_like(b["Y"])
    snr = torch.empty_like(b["snr"])
    best = torch.empty_like(b["best_w"])
    st = torch.empty_like(b["stats"])
    sps.sps_dedisperse(plan, b["X"], b["nsamp_in"], Y, b["nout"])
    sps.sps_boxcar_snr(plan, Y, b["nout"], widths, snr, best, st)
    c, n = sps.sps_detect(plan, snr, best, b["nout"], widths, cap=1 << 16, **DET)
    return Y, st, snr, best, c, n


def _oracle_beam(b, D, widths, label):
    """Every output of one batched beam against the oracle run on its input
    (read back from the device, so eager edits between replays count)."""
    Xh = b["X"][:, :b["nsamp_in"]].cpu().numpy()
    Yo, sto, _, _ = oracle.pipeline(Xh, D, b["nout"], widths, b["nsamp_in"])
    Yg = b["Y"].cpu().numpy().view(np.uint32)
    assert np.array_equal(Yg, Yo), f"{label} dedispersion"
    assert np.array_equal(b["stats"].cpu().numpy().astype(np.int64), sto), f"{label} stats"
    snr_g, best_g = b["snr"].cpu().numpy(), b["best_w"].cpu().numpy()
    snro, besto = check_snr(Yo, sto, widths, snr_g, best_g, label)
    return snr_g, best_g, snro, besto


def _check_beams(sps, plan, batch, beams, widths):
    D = oracle.delays(*_receiver(plan))
    for i, b in enumerate(beams):
        snr_g, best_g, snro, besto = _oracle_beam(b, D, widths, f"beam {i}")
        cb, nb = sps.sps_batch_candidates(batch, i, cap=1 << 16)
        det = (DET["threshold"], DET["tile_dm"], DET["tile_t"], DET["nms_dm"], DET["nms_t"])
        check_candidates_exact(cb, nb, oracle.detect(snr_g, best_g, *det), widths, f"beam {i}")
        check_candidates_close(cb, nb, oracle.detect(snro, besto, *det), widths, f"beam {i}")
        # and the single-filterbank calls agree with the batch
        Y, st, snr, best, c, n = _single(sps, plan, b, widths)
        assert torch.equal(b["Y"], Y), f"beam {i} dedispersion"
        assert torch.equal(b["stats"], st), f"beam {i} stats"
        assert torch.equal(b["snr"], snr) and torch.equal(b["best_w"], best), f"beam {i} S/N"
        assert nb == n and np.array_equal(cb, c), f"beam {i} candidates"


def _receiver(plan):
    wl = _wl(16, 0)
    assert plan.ndm == wl.ndm and plan.nchan == wl.nchan
    return wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, wl.dms()


# the last case: 40 beams, so the kernels' beam lookup (a binary search over
# the beams' first work items) takes several levels, with tiny, ragged and
# segment-edge lengths side by side
@pytest.mark.parametrize("nouts", [[3000, 5000, 1281, 7777, 4096], [16], [20000] * 3,
                                   [16, 17, 1000, 4095, 4096, 4097, 333, 8191] * 5,
                                   [4096, 3001, 17, 1000, 4095, 333]])
def test_batch_matches_oracle(sps, nouts):
    wl = _wl(nouts[0], 0)
    widths = list(wl.widths)
    with sps.plan_for(wl) as plan:
        _, dmax = sps.sps_plan_delays(plan)
        beams = _beams(sps, plan, nouts, dmax, pad=1)
        with sps.sps_batch_create(plan, beams, widths, **DET) as batch:
            sps.sps_batch_enqueue(batch)
            torch.cuda.synchronize()
            _check_beams(sps, plan, batch, beams, widths)


def test_graph_replays_match_eager(sps):
    nouts = [4000, 2500, 9000, 1300]
    wl = _wl(nouts[0], 0)
    widths = list(wl.widths)
    stream = torch.cuda.Stream()
    with sps.plan_for(wl) as plan:
        _, dmax = sps.sps_plan_delays(plan)
        beams = _beams(sps, plan, nouts, dmax, pad=0)
        with sps.sps_batch_create(plan, beams, widths, **DET) as batch:
            for rep in range(3):
                with torch.cuda.stream(stream):
                    # eager work between replays: new data in one beam
                    beams[rep % len(beams)]["X"][:, :64].random_(0, 256)
                    for b in beams:
                        b["Y"].zero_()
                        b["snr"].zero_()
                    sps.sps_batch_launch_graph(batch, stream)
                stream.synchronize()
                _check_beams(sps, plan, batch, beams, widths)


def test_autotune_keeps_results(sps):
    wl = SINGLE_BEAM
    with sps.plan_for(wl) as plan:
        _, dmax = sps.sps_plan_delays(plan)
        X = synth.random_bytes(wl.nchan, wl.nout + dmax, seed=5)
        Xd = torch.zeros((wl.nchan, ((wl.nout + dmax + 15) // 16) * 16), dtype=torch.uint8,
                         device="cuda")
        Xd[:, :wl.nout + dmax] = torch.from_numpy(X).cuda()
        Y0 = torch.empty((wl.ndm, wl.nout), dtype=torch.int32, device="cuda")
        sps.sps_dedisperse(plan, Xd, wl.nout + dmax, Y0, wl.nout)
        ms = sps.sps_plan_autotune(plan, 8192, 2)
        assert sum(m > 0 for m in ms) >= 2
        chosen = sps.sps_plan_get_tiling(plan)
        fastest = min((m, i) for i, m in enumerate(ms) if m > 0)[1]
        d = sps.sps_tiling_describe(fastest)
        assert all(chosen[k] == d[k] for k in ("m", "dpw", "nw", "cs", "waves_per_eu"))
        Y1 = torch.empty_like(Y0)
        sps.sps_dedisperse(plan, Xd, wl.nout + dmax, Y1, wl.nout)
        torch.cuda.synchronize()
        assert torch.equal(Y0, Y1)


def test_batch_autotune_keeps_results(sps):
    # the batch times its own batched launch per tiling, keeps the
    # fastest, and a graph captured before the autotuning is replaced
    nouts = [3000, 9000, 1281, 5000]
    wl = _wl(nouts[0], 0)
    widths = list(wl.widths)
    stream = torch.cuda.Stream()
    with sps.plan_for(wl) as plan:
        _, dmax = sps.sps_plan_delays(plan)
        plan_tiling = sps.sps_plan_get_tiling(plan)
        beams = _beams(sps, plan, nouts, dmax, pad=1)
        with sps.sps_batch_create(plan, beams, widths, **DET) as batch:
            sps.sps_batch_launch_graph(batch, stream)
            stream.synchronize()
            ms = sps.sps_batch_autotune(batch, 2, stream)
            assert sum(m > 0 for m in ms) >= 2
            assert sps.sps_plan_get_tiling(plan) == plan_tiling  # the plan is untouched
            for b in beams:
                b["Y"].zero_()
            sps.sps_batch_launch_graph(batch, stream)
            stream.synchronize()
            _check_beams(sps, plan, batch, beams, widths)


# tile lengths for each way the boxcar pass gathers tile maxima: a multiple
# of the boxcar segment (one reduction per segment), multiples of 64 on rows
# of 64-multiples (wave merges), and any other (per-thread merges)
@pytest.mark.parametrize("nouts,tile_t", [([3000, 5000, 1281, 7777, 4096], 1024),
                                          ([4096, 8192, 640, 12288], 1024),
                                          ([9000, 4096, 300, 16384], 4096),
                                          ([20000, 333, 6000], 777)])
def test_batch_without_planes(sps, nouts, tile_t):
    """A batch whose beams have no S/N or width planes (each tile key carries
    its peak's width) writes the same dedispersed planes and statistics and
    finds the same candidates as the batch with planes (held to the oracle
    per beam), on an eager run and on graph replays with eager edits in
    between."""
    wl = _wl(nouts[0], 0)
    widths = list(wl.widths)
    det = dict(DET, tile_t=tile_t)
    stream = torch.cuda.Stream()
    print(f"case batch without planes {nouts} tile_t {tile_t}", flush=True)
    with sps.plan_for(wl) as plan:
        _, dmax = sps.sps_plan_delays(plan)
        beams = _beams(sps, plan, nouts, dmax, pad=1)
        bare = [dict(X=b["X"], nsamp_in=b["nsamp_in"], nout=b["nout"],
                     Y=torch.zeros_like(b["Y"]), stats=torch.zeros_like(b["stats"]),
                     snr=None, best_w=None) for b in beams]
        D = oracle.delays(*_receiver(plan))
        dargs = (det["threshold"], det["tile_dm"], det["tile_t"], det["nms_dm"], det["nms_t"])
        with sps.sps_batch_create(plan, beams, widths, **det) as full, \
                sps.sps_batch_create(plan, bare, widths, **det) as batch:
            for rep in range(3):
                with torch.cuda.stream(stream):
                    if rep:
                        beams[rep % len(beams)]["X"][:, :64].random_(0, 256)
                        for b in bare:
                            b["Y"].zero_()
                    sps.sps_batch_enqueue(full, stream)
                    if rep == 0:
                        sps.sps_batch_enqueue(batch, stream)
                    else:
                        sps.sps_batch_launch_graph(batch, stream)
                stream.synchronize()
                for i, (b, q) in enumerate(zip(beams, bare)):
                    label = f"beam {i} rep {rep}"
                    assert torch.equal(q["Y"], b["Y"]), label
                    assert torch.equal(q["stats"], b["stats"]), label
                    cf, nf = sps.sps_batch_candidates(full, i, cap=1 << 16)
                    cb, nb = sps.sps_batch_candidates(batch, i, cap=1 << 16)
                    assert nb == nf and np.array_equal(cb, cf), label
                    if rep == 0 or i == rep % len(beams):
                        snr_g, best_g, _, _ = _oracle_beam(b, D, widths, label)
                        check_candidates_exact(cf, nf, oracle.detect(snr_g, best_g, *dargs),
                                               widths, label)


def test_batch_planes_all_or_none(sps):
    wl = _wl(3000, 0)
    with sps.plan_for(wl) as plan:
        _, dmax = sps.sps_plan_delays(plan)
        beams = _beams(sps, plan, [3000, 2000], dmax, pad=0)
        beams[1] = dict(beams[1], snr=None, best_w=None)
        with pytest.raises(sps.SpsError, match="INVALID_ARG"):
            sps.sps_batch_create(plan, beams, list(wl.widths), **DET)


def test_batch_candidates_all(sps):
    """Every beam's candidates in one call equal the per-beam calls: before
    the first run (none), with room for every record, with a cap that
    truncates, and with beams holding more records than one gathered slot
    (512), which take their own copies."""
    nouts = [20000, 3000, 8192, 16]
    wl = _wl(nouts[0], 0)
    widths = list(wl.widths)
    many = dict(threshold=1.0, tile_dm=4, tile_t=64, nms_dm=1, nms_t=4)
    with sps.plan_for(wl) as plan:
        _, dmax = sps.sps_plan_delays(plan)
        beams = _beams(sps, plan, nouts, dmax, pad=0)
        for det in (DET, many):
            print(f"case candidates_all {det}", flush=True)
            with sps.sps_batch_create(plan, beams, widths, **det) as batch:
                assert all(n == 0 for _, n in sps.sps_batch_candidates_all(batch, cap=16))
                sps.sps_batch_enqueue(batch)
                torch.cuda.synchronize()
                for cap in (1 << 16, 3):
                    got = sps.sps_batch_candidates_all(batch, cap=cap, allow_truncated=True)
                    for i in range(len(beams)):
                        c, n = sps.sps_batch_candidates(batch, i, cap=cap, allow_truncated=True)
                        assert got[i][1] == n and np.array_equal(got[i][0], c), (det, cap, i)
                if det is many:
                    counts = [n for _, n in sps.sps_batch_candidates_all(batch, cap=1 << 16)]
                    assert max(counts) > 512, counts
