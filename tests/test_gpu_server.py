"""GPU tests of the streaming server: chunk-by-chunk search with the
dispersion overlap kept on the device must equal the oracle's search of the
whole concatenated series (bit-exact dedispersion, candidates as in the
single-call path), admission must respect the memory budget, and a timed run
must search every scheduled chunk in order.  With the learned detector
attached, each chunk's count of flagged cells must equal the network run
directly on the same S/N plane."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from sps_inputs import synth  # noqa: E402
from sps_inputs.workloads import PulseModel, Workload  # noqa: E402

pytestmark = pytest.mark.gpu

SNR_RTOL = 1e-5
DET = dict(threshold=7.0, tile_dm=16, tile_t=512, nms_dm=8, nms_t=64)


@pytest.fixture(scope="module")
def sps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_02328_amd import sps as mod
    mod.library()
    return mod


def _wl(nchan, ndm, dm_hi, tsamp, seed):
    return Workload("s", nchan, 1000.0, 1500.0, tsamp, 0, ndm, 0.0, dm_hi, (1, 2, 4, 8, 16, 32),
                    pulses=PulseModel(count=3, dm_range=(20.0, dm_hi * 0.9),
                                      fwhm_range_s=(0.5e-3, 3e-3), amp_range_sigma=(2.0, 4.0)),
                    seed=seed)


def _add(sps, server, wl, chunk):
    return sps.sps_server_add_stream(server, wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, wl.dms(),
                                     wl.widths, chunk_len=chunk, **DET)


def _series(wl, nchunks, chunk):
    """The stream's whole input: nchunks * chunk samples (pulses across chunk edges)."""
    from dataclasses import replace
    X, _ = synth.make_filterbank(replace(wl, nout=nchunks * chunk), nchunks * chunk)
    return X


def _oracle_chunk(wl, Xs, overlap, k, chunk):
    """Oracle search of chunk k: samples [k chunk - overlap, (k+1) chunk) of the
    series, zeros before its start; the overlap is D_max rounded up to 16."""
    D = oracle.delays(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, wl.dms())
    assert overlap == (int(D.max()) + 15) // 16 * 16
    lo = k * chunk - overlap
    win = np.zeros((wl.nchan, overlap + chunk), np.uint8)
    a = max(lo, 0)
    win[:, a - lo:] = Xs[:, a:(k + 1) * chunk]
    return oracle.pipeline(win, D, chunk, wl.widths)


def _check_chunk(Yg, cands, n, ref, widths):
    Yo, sto, snro, besto = ref
    assert np.array_equal(Yg, Yo), "dedispersion differs"
    co = oracle.detect(snro, besto, DET["threshold"], DET["tile_dm"], DET["tile_t"],
                       DET["nms_dm"], DET["nms_t"])
    assert n == co["n_found"]
    got = sorted(zip(cands["dm_idx"], cands["t_idx"], cands["width"]))
    want = sorted(zip(co["d"], co["t"], [widths[i] for i in co["w"]]))
    assert got == want
    s_g = np.sort(cands["snr"])
    s_o = np.sort(co["snr"])
    assert np.allclose(s_g, s_o, rtol=SNR_RTOL, atol=0)


@pytest.mark.parametrize("chunk", [1000, 4096, 7777])
def test_chunks_equal_whole_series(sps, chunk):
    # two set-ups, two streams of the first: rings are independent, plans shared
    wa = _wl(128, 96, 150.0, 98.304e-6, 21)
    wb = _wl(64, 40, 400.0, 196.608e-6, 22)
    nchunks = 4
    with sps.sps_server_create(8 << 30, 2) as server:
        ids = [_add(sps, server, wa, chunk), _add(sps, server, wb, chunk + 512),
               _add(sps, server, wa, chunk)]
        setups = [(wa, chunk, 21), (wb, chunk + 512, 22), (wa, chunk, 23)]
        series = []
        for (wl, L, seed) in setups:
            from dataclasses import replace
            series.append(_series(replace(wl, seed=seed), nchunks, L))
        for k in range(nchunks):
            for sid, (wl, L, _), Xs in zip(ids, setups, series):
                info = sps.sps_server_stream_info(server, sid)
                assert info["chunk_len"] == L
                Y = torch.zeros((wl.ndm, L), dtype=torch.int32, device="cuda")
                host = torch.from_numpy(np.ascontiguousarray(Xs[:, k * L:(k + 1) * L]))
                cands, n = sps.sps_server_push(server, sid, host, Y_copy=Y)
                torch.cuda.synchronize()
                ref = _oracle_chunk(wl, Xs, info["overlap"], k, L)
                _check_chunk(Y.cpu().numpy().view(np.uint32), cands, n, ref, wl.widths)


def test_admission_by_budget(sps):
    wa = _wl(128, 96, 150.0, 98.304e-6, 1)
    wb = _wl(64, 40, 400.0, 196.608e-6, 2)
    with sps.sps_server_create(1 << 40, 2) as probe:
        _add(sps, probe, wa, 4096)
        one = sps.sps_server_memory(probe)["used"]
        _add(sps, probe, wa, 4096)
        two = sps.sps_server_memory(probe)["used"]
    ring = two - one
    assert 0 < ring < one  # a second stream of a set-up costs its ring only
    with sps.sps_server_create(one + ring // 2, 2) as server:
        _add(sps, server, wa, 4096)
        assert sps.sps_server_memory(server)["used"] == one
        with pytest.raises(sps.SpsError) as e:
            _add(sps, server, wa, 4096)
        assert e.value.name == "SPS_ERR_NOMEM" and "refused" in str(e.value)
        assert sps.sps_server_memory(server)["used"] == one
        with pytest.raises(sps.SpsError):
            _add(sps, server, wb, 8192)  # new plans and planes do not fit either
        assert sps.sps_server_memory(server)["used"] == one
    with pytest.raises(sps.SpsError):
        sps.sps_server_create(0, 1)
    with pytest.raises(sps.SpsError):
        sps.sps_server_create(1 << 30, 17)


def test_timed_run_then_continue(sps):
    # 2 streams, chunks of ~0.1 s / 0.2 s, compressed 4x: every scheduled
    # chunk is searched in order; afterwards the rings still hold the right
    # overlap, so a pushed chunk equals the oracle on the concatenated series
    wa = _wl(128, 96, 150.0, 98.304e-6, 31)
    wb = _wl(64, 40, 400.0, 196.608e-6, 32)
    La, Lb = 4096, 4096
    nsrc = 3
    run_s, comp = 1.5, 4.0
    with sps.sps_server_create(8 << 30, 2) as server:
        ia, ib = _add(sps, server, wa, La), _add(sps, server, wb, Lb)
        srcs = [_series(wa, nsrc, La), _series(wb, nsrc, Lb)]
        feeds = []
        for Xs, L in zip(srcs, (La, Lb)):
            stacked = np.concatenate([Xs[:, k * L:(k + 1) * L] for k in range(nsrc)], axis=0)
            feeds.append(dict(host=torch.from_numpy(np.ascontiguousarray(stacked)).pin_memory(),
                              nsrc=nsrc, first=1))
        recs = sps.sps_server_run(server, feeds, run_s, comp)
        assert np.all(recs["status"] == 0)
        for sid, wl, L in ((ia, wa, La), (ib, wb, Lb)):
            T = L * wl.tsamp_s / comp
            phase = T * sid / 2
            nexp = int(np.floor((run_s - phase) / T + 1e-9))
            r = recs[recs["stream"] == sid]
            assert len(r) == nexp and list(r["index"]) == list(range(nexp))
            assert np.allclose(r["arrival_s"], phase + (np.arange(nexp) + 1) * T)
            assert np.all(r["start_s"] >= r["arrival_s"]) and np.all(r["end_s"] > r["start_s"])
            assert np.all(r["upload_s"] >= r["start_s"]) and np.all(r["compute_s"] >= r["upload_s"])
            assert np.all(r["end_s"] >= r["compute_s"])
            assert np.all(np.diff(r["start_s"]) > 0)
        # continue: the run searched chunks first, first+1, ... of the sources
        for sid, wl, L, Xs in ((ia, wa, La, srcs[0]), (ib, wb, Lb, srcs[1])):
            nrun = int((recs["stream"] == sid).sum())
            order = [(1 + k) % nsrc for k in range(nrun + 1)]
            full = np.concatenate([Xs[:, j * L:(j + 1) * L] for j in order], axis=1)
            Y = torch.zeros((wl.ndm, L), dtype=torch.int32, device="cuda")
            cands, n = sps.sps_server_push(server, sid, full[:, nrun * L:], Y_copy=Y)
            torch.cuda.synchronize()
            info = sps.sps_server_stream_info(server, sid)
            ref = _oracle_chunk(wl, full, info["overlap"], nrun, L)
            _check_chunk(Y.cpu().numpy().view(np.uint32), cands, n, ref, wl.widths)


def _net(sps, max_batch, seed):
    from paper_2511_02328_amd import detector
    p = detector.init_params(seed)
    p[-3] = 0.0  # objectness bias 0: a fair share of cells near the threshold
    net = sps.sps_cnn_create(max_batch)
    sps.sps_cnn_set_params(net, p)
    return net, p


def _oracle_cell_count(ncnn, snr, p, thr):
    """The server's count of flagged cells against the detector oracle on the
    same S/N plane (pooled by the oracle, network in the oracle's rounding
    points): every cell whose oracle logit clears the threshold by more than
    the FP32-accumulation drift bound of the head (1e-2 of its largest value)
    must be counted, and none below it by that margin."""
    cnn = oracle.cnn()
    params = cnn.init_params(7)
    params["bh"][0] = 0.0
    assert np.array_equal(np.concatenate([params[k].ravel() for k in cnn.param_names()]), p)
    tiles = np.stack([cnn.pool_tiles(snr[512 * i:512 * (i + 1), 4096 * j:4096 * (j + 1)], 0.125)
                      for i in range(snr.shape[0] // 512) for j in range(snr.shape[1] // 4096)])
    head, _ = cnn.forward(params, tiles)
    logit = head[:, 0]
    lt = np.log(thr / (1.0 - thr))
    delta = 1e-2 * np.abs(head).max()
    sure, maybe = int((logit >= lt + delta).sum()), int((logit >= lt - delta).sum())
    assert sure <= ncnn <= maybe, (sure, ncnn, maybe)


def test_detector_in_server(sps):
    # 1024 trials x 8192 samples per chunk = 2 x 2 tiles; the server's network
    # takes 3 tiles a batch, so each chunk needs two batches
    wl = _wl(64, 1024, 400.0, 196.608e-6, 41)
    L, nchunks, thr = 8192, 3, 0.6
    Xs = _series(wl, nchunks, L)
    net, p = _net(sps, 3, 7)
    ref_net = sps.sps_cnn_create(4)
    sps.sps_cnn_set_params(ref_net, p)
    plan = sps.plan_for(wl)
    with sps.sps_server_create(8 << 30, 1) as server:
        sid = _add(sps, server, wl, L)
        before = sps.sps_server_memory(server)["used"]
        sps.sps_server_set_detector(server, net, thr)
        assert sps.sps_server_memory(server)["used"] == before + 4 * 256 * 512 * 2
        counts = []
        for k in range(nchunks):
            Y = torch.zeros((wl.ndm, L), dtype=torch.int32, device="cuda")
            host = np.ascontiguousarray(Xs[:, k * L:(k + 1) * L])
            cands, n, ncnn = sps.sps_server_push(server, sid, host, Y_copy=Y, with_cnn=True)
            snr = torch.empty((wl.ndm, L), dtype=torch.float32, device="cuda")
            best = torch.empty((wl.ndm, L), dtype=torch.uint8, device="cuda")
            st = torch.empty((wl.ndm, 2), dtype=torch.int32, device="cuda")
            sps.sps_boxcar_snr(plan, Y, L, wl.widths, snr, best, st)
            tiles = torch.empty((4, 256, 512), dtype=torch.int16, device="cuda")
            assert sps.sps_cnn_pool_tile_grid(snr, L, 0.125, tiles) == 4
            _, want = sps.sps_cnn_detect(ref_net, tiles, 4, thr, cap=0, allow_truncated=True)
            torch.cuda.synchronize()
            assert ncnn == want, k
            if k == 0:
                _oracle_cell_count(ncnn, snr.cpu().numpy(), p, thr)
            counts.append(ncnn)
            info = sps.sps_server_stream_info(server, sid)
            ref = _oracle_chunk(wl, Xs, info["overlap"], k, L)
            _check_chunk(Y.cpu().numpy().view(np.uint32), cands, n, ref, wl.widths)
        assert 0 < sum(counts) < nchunks * 4 * 128
        # a timed run carries the counts in its records
        feed = dict(host=torch.from_numpy(np.ascontiguousarray(Xs[:, :L])).pin_memory(), nsrc=1)
        recs = sps.sps_server_run(server, [feed], 0.5, 4.0)
        assert len(recs) > 0 and np.all(recs["status"] == 0)
        assert np.all((recs["n_cnn"] >= 0) & (recs["n_cnn"] <= 4 * 128))
        sps.sps_server_set_detector(server, None)
        _, _, ncnn = sps.sps_server_push(server, sid, np.ascontiguousarray(Xs[:, :L]),
                                         with_cnn=True)
        assert ncnn == 0
    net.close()
    ref_net.close()
    plan.close()


def test_detector_budget(sps):
    wl = _wl(64, 1024, 400.0, 196.608e-6, 42)
    with sps.sps_server_create(1 << 40, 1) as probe:
        _add(sps, probe, wl, 8192)
        one = sps.sps_server_memory(probe)["used"]
    net, _ = _net(sps, 2, 8)
    with sps.sps_server_create(one + 4 * 256 * 512 * 2 - 1, 1) as server:
        _add(sps, server, wl, 8192)
        with pytest.raises(sps.SpsError) as e:
            sps.sps_server_set_detector(server, net, 0.9)
        assert e.value.name == "SPS_ERR_NOMEM"
        assert sps.sps_server_memory(server)["used"] == one
        with pytest.raises(sps.SpsError):
            sps.sps_server_set_detector(server, net, 1.5)
    with sps.sps_server_create(one + 4 * 256 * 512 * 2, 1) as server:
        sps.sps_server_set_detector(server, net, 0.9)   # no streams yet: no tiles
        assert sps.sps_server_memory(server)["used"] == 0
        _add(sps, server, wl, 8192)                     # the stream brings its tiles
        assert sps.sps_server_memory(server)["used"] == one + 4 * 256 * 512 * 2
        with pytest.raises(sps.SpsError):
            _add(sps, server, _wl(64, 2048, 400.0, 196.608e-6, 43), 8192)
    net.close()


def test_detector_on_planes_without_whole_tiles(sps):
    # fewer than 512 trials: no whole tile, so the network never runs and the
    # count is 0; the search itself is unchanged
    wl = _wl(128, 96, 150.0, 98.304e-6, 44)
    L = 4096
    Xs = _series(wl, 2, L)
    net, _ = _net(sps, 2, 9)
    with sps.sps_server_create(8 << 30, 1) as server:
        sps.sps_server_set_detector(server, net, 0.5)
        sid = _add(sps, server, wl, L)
        for k in range(2):
            Y = torch.zeros((wl.ndm, L), dtype=torch.int32, device="cuda")
            cands, n, ncnn = sps.sps_server_push(server, sid, np.ascontiguousarray(Xs[:, k * L:(k + 1) * L]),
                                                 Y_copy=Y, with_cnn=True)
            torch.cuda.synchronize()
            assert ncnn == 0
            info = sps.sps_server_stream_info(server, sid)
            ref = _oracle_chunk(wl, Xs, info["overlap"], k, L)
            _check_chunk(Y.cpu().numpy().view(np.uint32), cands, n, ref, wl.widths)
    net.close()
