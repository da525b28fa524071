"""GPU parity at the workloads' full sizes, in the launch configurations the
benchmark times: outputs the oracle can compute one by one are compared on
samples (whole DM rows, bit-exact), and every row is checked through a
property that holds at any size (its sum over time, from per-channel prefix
sums of the input).  Detection is compared on the GPU's own full S/N plane.

Covered: the full-scale chunk (4096 channels, 2048 DMs, 2^20 samples) on
brute force and on the subband method, the 19-beam batch (graph replay,
tiling from the batch autotuner; with and without S/N planes), a full-size
stream of the streaming server, and the ends of the paper's two
dedispersion timing sweeps."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from _checks import check_candidates_exact, check_snr  # noqa: E402
from sps_inputs import synth  # noqa: E402
from sps_inputs.workloads import BATCHED, FULL_SCALE, STREAMING  # noqa: E402

pytestmark = pytest.mark.gpu

SNR_RTOL = 1e-5
DET = dict(threshold=8.0, tile_dm=64, tile_t=4096, nms_dm=16, nms_t=512)


@pytest.fixture(scope="module")
def sps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_02328_amd import sps as mod
    mod.library()
    return mod


def _rows(ndm, k):
    return np.unique(np.linspace(0, ndm - 1, k).round().astype(np.int64))


@pytest.fixture(scope="module")
def full(sps):
    """The full-scale chunk through the default path, as the benchmark runs it."""
    wl = FULL_SCALE
    plan = sps.plan_for(wl)
    D, dmax = sps.sps_plan_delays(plan)
    nsamp = wl.nout + dmax
    pitch = (nsamp + 255) // 256 * 256
    X, _ = synth.make_filterbank(wl, nsamp, device="cuda", pitch=pitch)
    Y = torch.empty((wl.ndm, wl.nout), dtype=torch.int32, device="cuda")
    snr = torch.empty((wl.ndm, wl.nout), dtype=torch.float32, device="cuda")
    best = torch.empty((wl.ndm, wl.nout), dtype=torch.uint8, device="cuda")
    st = torch.empty((wl.ndm, 2), dtype=torch.int32, device="cuda")
    sps.sps_dedisperse(plan, X, nsamp, Y, wl.nout)
    sps.sps_boxcar_snr(plan, Y, wl.nout, wl.widths, snr, best, st)
    cands, n = sps.sps_detect(plan, snr, best, wl.nout, wl.widths, cap=4096,
                              allow_truncated=True, **DET)
    torch.cuda.synchronize()
    Xh = X.cpu().numpy()
    yield dict(wl=wl, plan=plan, D=D, nsamp=nsamp, X=X, Xh=Xh, Y=Y, snr=snr, best=best, st=st,
               cands=cands, n=n)
    plan.close()


def test_fullscale_rows_and_checksums(full):
    wl, D, Xh, nsamp = full["wl"], full["D"], full["Xh"], full["nsamp"]
    Do = oracle.delays(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, wl.dms())
    assert np.array_equal(D, Do)
    rows = _rows(wl.ndm, 6)
    Yo = oracle.dedisperse(Xh, Do[rows], wl.nout, nsamp)
    Yg = full["Y"][torch.from_numpy(rows).cuda()].cpu().numpy().view(np.uint32)
    assert np.array_equal(Yg, Yo), "sampled rows differ"
    sums_o = oracle.row_checksums(Xh, Do, wl.nout, nsamp)
    sums_g = full["Y"].sum(dim=1, dtype=torch.int64).cpu().numpy().astype(np.uint64)
    assert np.array_equal(sums_g, sums_o), f"{int((sums_g != sums_o).sum())} row sums differ"


def test_fullscale_stats_and_snr(full):
    wl = full["wl"]
    rows = _rows(wl.ndm, 3)
    idx = torch.from_numpy(rows).cuda()
    Yr = full["Y"][idx].cpu().numpy().view(np.uint32)
    sto = oracle.stats(Yr)
    assert np.array_equal(full["st"][idx].cpu().numpy().astype(np.int64), sto)
    snro, besto, s64 = oracle.boxcar(Yr, sto, wl.widths, want_f64=True)
    snrg = full["snr"][idx].cpu().numpy()
    bestg = full["best"][idx].cpu().numpy()
    tol = SNR_RTOL * np.maximum(1.0, np.abs(snro.astype(np.float64)))
    assert np.all(np.abs(snrg.astype(np.float64) - snro) <= tol)
    # widths may differ only at near-ties: the GPU's width must reach the
    # oracle's maximum within the tolerance (S/N of a width by its formula)
    mism = bestg != besto
    for r, t in zip(*np.nonzero(mism)):
        w = wl.widths[bestg[r, t]]
        med, mad = sto[r]
        s_w = (float(Yr[r, t:t + w].astype(np.float64).sum()) - w * med) / \
              (1.4826 * mad * np.sqrt(w))
        assert abs(s_w - s64[r, t]) <= 2 * tol[r, t], (r, t, w, s_w, s64[r, t])


def test_fullscale_detect_on_gpu_plane(full):
    wl = full["wl"]
    snr = full["snr"].cpu().numpy()
    best = full["best"].cpu().numpy()
    co = oracle.detect(snr, best, DET["threshold"], DET["tile_dm"], DET["tile_t"],
                       DET["nms_dm"], DET["nms_t"], cap=1 << 16)
    cg, n = full["cands"], full["n"]
    assert n == co["n_found"]
    k = min(n, len(cg))
    assert list(cg["dm_idx"][:k]) == list(co["d"][:k])
    assert list(cg["t_idx"][:k]) == list(co["t"][:k])
    assert list(cg["width"][:k]) == [wl.widths[i] for i in co["w"][:k]]
    assert np.array_equal(cg["snr"][:k], co["snr"][:k])


def test_fullscale_subband_rows(sps, full):
    # stage 1 + stage 2 is one shift-and-sum with the effective delays
    # D_eff[m][c] = Dc[j(m)][c] + R[m][s(c)], so sampled rows are brute force
    # over the effective table
    wl, Xh, X, nsamp = full["wl"], full["Xh"], full["X"], full["nsamp"]
    n0, nsub = 8, 32
    ddm = (wl.dm_hi - wl.dm_lo) / (wl.ndm - 1)
    with sps.sps_subband_plan_create(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, wl.ndm, wl.dm_lo,
                                     ddm, n0, nsub) as plan:
        Dc, R, F, mx = sps.sps_subband_tables(plan)
        sps.sps_plan_autotune(plan, 1 << 18, 2)  # picks the stage-1 form, as the benchmark does
        Y = torch.empty((wl.ndm, wl.nout), dtype=torch.int32, device="cuda")
        sps.sps_dedisperse_subband(plan, X, nsamp, Y, wl.nout)
        torch.cuda.synchronize()
        sub = oracle.equal_subbands(wl.nchan, nsub)
        Ro, Fo, dmc = oracle.subband_residuals(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, sub,
                                               wl.ndm, wl.dm_lo, ddm, n0)
        Dco = oracle.delays(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, dmc)
        assert np.array_equal(Dc, Dco) and np.array_equal(R, Ro)
        s_of_c = np.repeat(np.arange(nsub), np.diff(sub))
        rows = _rows(wl.ndm, 4)
        Deff = (Dco[rows // n0] + Ro[rows][:, s_of_c]).astype(np.int32)
        Yo = oracle.dedisperse(Xh, Deff, wl.nout, nsamp)
        Yg = Y[torch.from_numpy(rows).cuda()].cpu().numpy().view(np.uint32)
        assert np.array_equal(Yg, Yo)


def test_batched_19_beams_full_size(sps):
    bw = BATCHED
    wl0 = bw.base
    plan = sps.plan_for(wl0)
    _, dmax = sps.sps_plan_delays(plan)
    D = oracle.delays(wl0.freqs_mhz(), wl0.fref_mhz, wl0.tsamp_s, wl0.dms())
    lengths = bw.beam_lengths()
    beams = []
    for i, nout in enumerate(lengths):
        wl = bw.beam_workload(i, nout)
        nsamp = nout + dmax
        X, _ = synth.make_filterbank(wl, nsamp, device="cuda", pitch=(nsamp + 255) // 256 * 256)
        beams.append(dict(X=X, nsamp_in=nsamp, nout=nout,
                          Y=torch.empty((wl.ndm, nout), dtype=torch.int32, device="cuda"),
                          snr=torch.empty((wl.ndm, nout), dtype=torch.float32, device="cuda"),
                          best_w=torch.empty((wl.ndm, nout), dtype=torch.uint8, device="cuda"),
                          stats=torch.empty((wl.ndm, 2), dtype=torch.int32, device="cuda")))
    stream = torch.cuda.Stream()
    with sps.sps_batch_create(plan, beams, list(wl0.widths), **DET) as batch:
        sps.sps_batch_autotune(batch, 2, stream)  # as the benchmark does
        for _ in range(2):  # capture, then a replay
            sps.sps_batch_launch_graph(batch, stream)
        stream.synchronize()
        for i in (0, 1, len(beams) - 1):   # beams of different lengths
            b = beams[i]
            Xh = b["X"].cpu().numpy()
            rows = _rows(wl0.ndm, 3)
            Yo = oracle.dedisperse(Xh, D[rows], b["nout"], b["nsamp_in"])
            Yg = b["Y"][torch.from_numpy(rows).cuda()].cpu().numpy().view(np.uint32)
            assert np.array_equal(Yg, Yo), f"beam {i}"
            sums_o = oracle.row_checksums(Xh, D, b["nout"], b["nsamp_in"])
            sums_g = b["Y"].sum(dim=1, dtype=torch.int64).cpu().numpy().astype(np.uint64)
            assert np.array_equal(sums_g, sums_o), f"beam {i} row sums"
            idx = torch.from_numpy(rows).cuda()
            st = b["stats"][idx].cpu().numpy().astype(np.int64)
            sto = oracle.stats(Yo)
            assert np.array_equal(st, sto), f"beam {i} stats"
            check_snr(Yo, sto, wl0.widths, b["snr"][idx].cpu().numpy(),
                      b["best_w"][idx].cpu().numpy(), f"beam {i}")
            # candidates: the oracle's rule on the beam's whole GPU plane
            snr_full, best_full = b["snr"].cpu().numpy(), b["best_w"].cpu().numpy()
            co = oracle.detect(snr_full, best_full, DET["threshold"], DET["tile_dm"],
                               DET["tile_t"], DET["nms_dm"], DET["nms_t"], cap=1 << 16)
            del snr_full, best_full
            cb, nb = sps.sps_batch_candidates(batch, i, cap=1 << 16)
            check_candidates_exact(cb, nb, co, list(wl0.widths), f"beam {i}")
        # the same batch without planes (the search the benchmark also
        # times): the same statistics and, in every beam, the same candidates
        full = [sps.sps_batch_candidates(batch, i, cap=1 << 16) for i in range(len(beams))]
        stats = [b["stats"].clone() for b in beams]
        bare = [dict(b, snr=None, best_w=None) for b in beams]
        with sps.sps_batch_create(plan, bare, list(wl0.widths), **DET) as nb_batch:
            for b in beams:
                b["stats"].zero_()
            for _ in range(2):
                sps.sps_batch_launch_graph(nb_batch, stream)
            stream.synchronize()
            for i, b in enumerate(beams):
                assert torch.equal(b["stats"], stats[i]), f"beam {i} stats without planes"
                cb, nb = sps.sps_batch_candidates(nb_batch, i, cap=1 << 16)
                assert nb == full[i][1] and np.array_equal(cb, full[i][0]), \
                    f"beam {i} candidates without planes"
    plan.close()


def test_streaming_setup_a_full_size(sps):
    # one stream of the 1024-channel set-up, two consecutive 2^18-sample chunks
    wl = STREAMING.groups[0][1]
    L = wl.nout
    with sps.sps_server_create(64 << 30, 1) as server:
        sid = sps.sps_server_add_stream(server, wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s,
                                        wl.dms(), wl.widths, chunk_len=L, **DET)
        O = sps.sps_server_stream_info(server, sid)["overlap"]
        from dataclasses import replace
        Xs, _ = synth.make_filterbank(replace(wl, nout=2 * L), 2 * L, device="cuda")
        Xs = Xs.cpu().numpy()
        D = oracle.delays(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, wl.dms())
        rows = _rows(wl.ndm, 3)
        for k in range(2):
            Y = torch.zeros((wl.ndm, L), dtype=torch.int32, device="cuda")
            host = torch.from_numpy(np.ascontiguousarray(Xs[:, k * L:(k + 1) * L])).pin_memory()
            sps.sps_server_push(server, sid, host, Y_copy=Y, allow_truncated=True)
            torch.cuda.synchronize()
            win = np.zeros((wl.nchan, O + L), np.uint8)
            lo = k * L - O
            a = max(lo, 0)
            win[:, a - lo:] = Xs[:, a:(k + 1) * L]
            Yo = oracle.dedisperse(win, D[rows], L)
            Yg = Y[torch.from_numpy(rows).cuda()].cpu().numpy().view(np.uint32)
            assert np.array_equal(Yg, Yo), f"chunk {k}"
            sums_o = oracle.row_checksums(win, D, L)
            sums_g = Y.sum(dim=1, dtype=torch.int64).cpu().numpy().astype(np.uint64)
            assert np.array_equal(sums_g, sums_o), f"chunk {k} row sums"


@pytest.mark.parametrize("sweep,point", [("sweep_channels", 0), ("sweep_channels", -1),
                                         ("sweep_dms", -1)])
def test_sweep_ends_full_size(sps, sweep, point):
    """The ends of the paper's dedispersion timing sweeps (Sec. 3.1: 512 and
    8192 channels, 1500 DMs, 550,000 outputs; Sec. 3.2: 8192 DMs over 2048
    channels, 500,000 outputs) with the tiling the autotuner keeps, as the
    benchmark times them: sampled rows bit-exact, every row's sum exact.  At
    512 channels the subband method (32 subbands of 16 channels) too."""
    from sps_inputs.workloads import SWEEPS
    wl = SWEEPS[sweep][point]
    with sps.plan_for(wl) as plan:
        D, dmax = sps.sps_plan_delays(plan)
        nsamp = wl.nout + dmax
        sps.sps_plan_autotune(plan, 1 << 18, 2)
        X, _ = synth.make_filterbank(wl, nsamp, device="cuda", pitch=(nsamp + 255) // 256 * 256)
        Y = torch.empty((wl.ndm, wl.nout), dtype=torch.int32, device="cuda")
        sps.sps_dedisperse(plan, X, nsamp, Y, wl.nout)
        torch.cuda.synchronize()
        Xh = X.cpu().numpy()
        Do = oracle.delays(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, wl.dms())
        assert np.array_equal(D, Do)
        rows = _rows(wl.ndm, 2)
        Yo = oracle.dedisperse(Xh, Do[rows], wl.nout, nsamp)
        assert np.array_equal(Y[torch.from_numpy(rows).cuda()].cpu().numpy().view(np.uint32), Yo)
        sums_o = oracle.row_checksums(Xh, Do, wl.nout, nsamp)
        sums_g = Y.sum(dim=1, dtype=torch.int64).cpu().numpy().astype(np.uint64)
        assert np.array_equal(sums_g, sums_o)
    if wl.nchan == 512:
        n0, nsub = 8, 32
        ddm = (wl.dm_hi - wl.dm_lo) / (wl.ndm - 1)
        with sps.sps_subband_plan_create(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, wl.ndm,
                                         wl.dm_lo, ddm, n0, nsub) as plan:
            emax = sps.sps_subband_tables(plan)[3]
            sps.sps_plan_autotune(plan, 1 << 18, 2)
            # effective delays past the input read as zero, as in the oracle
            sps.sps_dedisperse_subband(plan, X, nsamp, Y, wl.nout,
                                       flags=sps.SPS_ZERO_PAD if emax > dmax else 0)
            torch.cuda.synchronize()
            sub = oracle.equal_subbands(wl.nchan, nsub)
            Ro, _, dmc = oracle.subband_residuals(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, sub,
                                                  wl.ndm, wl.dm_lo, ddm, n0)
            Dco = oracle.delays(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, dmc)
            s_of_c = np.repeat(np.arange(nsub), np.diff(sub))
            Deff = (Dco[rows // n0] + Ro[rows][:, s_of_c]).astype(np.int32)
            Yo = oracle.dedisperse(Xh, Deff, wl.nout, nsamp)
            assert np.array_equal(Y[torch.from_numpy(rows).cuda()].cpu().numpy().view(np.uint32),
                                  Yo)
