"""GPU parity of the detector tiles written straight from the boxcar pass
(sps_boxcar_pool, and batches in tile mode): bit for bit the tiles that
pooling the S/N plane gives (sps_cnn_pool_tile_grid, and the oracle's
pooling of the GPU plane), and against the oracle's own S/N within one
bfloat16 step exactly where a rounding boundary lies within the S/N
tolerance of the oracle's pooled value."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from _checks import SNR_RTOL, check_snr  # noqa: E402
from sps_inputs.workloads import Workload  # noqa: E402

pytestmark = pytest.mark.gpu

cnn = oracle.cnn()
SCALE = 0.125


@pytest.fixture(scope="module")
def sps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_02328_amd import sps as mod
    mod.library()
    return mod


def _grid_tiles(plane, scale):
    """Oracle pooling of the whole 512 x 4096 tiles of a plane, row-major."""
    nd, nt = plane.shape
    out = []
    for i in range(nd // 512):
        for j in range(nt // 4096):
            out.append(cnn.pool_tiles(plane[512 * i:512 * (i + 1), 4096 * j:4096 * (j + 1)], scale))
    return np.array(out)


def _check_against_oracle_snr(got, snro, scale):
    """got (bf16 values) against the oracle S/N pooled: equal, or one bf16
    step apart where the oracle's pooled value lies within the S/N tolerance
    of the boundary between them."""
    want = _grid_tiles(snro.astype(np.float32), scale)
    diff = got != want
    if not diff.any():
        return
    # the unrounded pooled values of the oracle plane at the differing cells
    nd, nt = snro.shape
    k, i, j = np.nonzero(diff)
    ncols = nt // 4096
    ti, tj = k // ncols, k % ncols
    vals = []
    for a, b, c, d in zip(ti, tj, i, j):
        blk = snro[512 * a + 2 * c:512 * a + 2 * c + 2, 4096 * b + 8 * d:4096 * b + 8 * d + 8]
        vals.append(float(blk.max()) * scale)
    vals = np.array(vals)
    g, w = got[diff].astype(np.float64), want[diff].astype(np.float64)
    mid = 0.5 * (g + w)
    tol = SNR_RTOL * np.maximum(1.0, np.abs(vals) / scale) * scale
    assert np.all(np.abs(g - w) <= 2.0 ** (np.floor(np.log2(np.abs(w) + 1e-38)) - 7) + 1e-38)
    assert np.all(np.abs(vals - mid) <= tol)


@pytest.mark.parametrize("case", [
    dict(ndm=1100, nout=9000, widths=(1, 2, 4, 8, 16, 32, 64)),   # 2 x 2 whole tiles + ragged rest
    dict(ndm=512, nout=4096, widths=(1, 3, 5, 12)),               # generic widths, one tile
    dict(ndm=1024, nout=8192, widths=(1, 2, 4, 8, 16, 32, 64, 128, 256)),
])
def test_boxcar_pool_matches_pooled_planes(sps, case):
    ndm, nout, widths = case["ndm"], case["nout"], case["widths"]
    rng = np.random.Generator(np.random.PCG64(ndm + nout))
    nchan = 256
    Y = rng.integers(0, 255 * nchan + 1, size=(ndm, nout)).astype(np.uint32)
    Y[5] = 77              # MAD 0: S/N 0 in its pair
    Y[6] = rng.integers(1000, 1003, size=nout)
    for _ in range(10):    # bright windows
        d, t = int(rng.integers(0, ndm)), int(rng.integers(0, nout - 64))
        Y[d, t:t + 32] = 255 * nchan
    wl = Workload("pool", nchan, 1000.0, 1500.0, 1e-4, nout, ndm, 0.0, 1.0, widths)
    ntiles = (ndm // 512) * (nout // 4096)
    print(f"case sps_boxcar_pool {case}", flush=True)
    with sps.plan_for(wl) as plan:
        Yd = torch.from_numpy(Y.view(np.int32)).cuda()
        tiles = torch.full((ntiles + 1, 256, 512), 0x7FC0, dtype=torch.int16, device="cuda")
        st = torch.empty((ndm, 2), dtype=torch.int32, device="cuda")
        n = sps.sps_boxcar_pool(plan, Yd, nout, widths, st, SCALE, tiles)
        snr = torch.empty((ndm, nout), dtype=torch.float32, device="cuda")
        best = torch.empty((ndm, nout), dtype=torch.uint8, device="cuda")
        sps.sps_boxcar_snr(plan, Yd, nout, widths, snr, best)
        grid = torch.zeros_like(tiles)
        ng = sps.sps_cnn_pool_tile_grid(snr, nout, SCALE, grid)
        torch.cuda.synchronize()
    assert n == ntiles and ng == ntiles
    got_bits = tiles.cpu().numpy().view(np.uint16)
    assert np.all(got_bits[ntiles] == 0x7FC0)  # nothing past the whole tiles
    got_bits = got_bits[:ntiles]
    # bit for bit the pooling of the S/N plane the boxcar call writes
    assert np.array_equal(got_bits, grid.cpu().numpy().view(np.uint16)[:ntiles])
    got = cnn.from_bf16_bits(got_bits)
    snr_g = snr.cpu().numpy()
    assert np.array_equal(got, _grid_tiles(snr_g, SCALE))
    # against the oracle's statistics and S/N
    sto = oracle.stats(Y)
    assert np.array_equal(st.cpu().numpy().astype(np.int64), sto)
    snro, _ = check_snr(Y, sto, widths, snr_g, best.cpu().numpy(), str(case))
    _, _, s64 = oracle.boxcar(Y, sto, widths, want_f64=True)
    _check_against_oracle_snr(got, s64, SCALE)


def test_batch_tile_mode(sps):
    # beams of one plan with 1, 2 and 1 whole tile columns (one ragged); the
    # tile mode's tiles equal the pooling of the search mode's planes, in
    # eager runs and graph replays
    from sps_inputs import synth
    nchan, ndm = 64, 512
    wl = Workload("poolbatch", nchan, 1000.0, 1500.0, 2e-4, 8192, ndm, 0.0, 100.0,
                  (1, 2, 4, 8, 16))
    nouts = [4096, 8192, 5000]
    with sps.plan_for(wl) as plan:
        _, dmax = sps.sps_plan_delays(plan)
        beams = []
        for i, nout in enumerate(nouts):
            nsamp = nout + dmax
            pitch = (nsamp + 255) // 256 * 256
            X, _ = synth.make_filterbank(wl, nsamp, seed=40 + i, device="cuda", pitch=pitch)
            beams.append(dict(X=X, nsamp_in=nsamp, nout=nout,
                              Y=torch.empty((ndm, nout), dtype=torch.int32, device="cuda"),
                              snr=torch.empty((ndm, nout), dtype=torch.float32, device="cuda"),
                              best_w=torch.empty((ndm, nout), dtype=torch.uint8, device="cuda"),
                              stats=torch.empty((ndm, 2), dtype=torch.int32, device="cuda")))
        with sps.sps_batch_create(plan, beams, list(wl.widths), 8.0, 64, 4096, 16, 64) as b:
            stream = torch.cuda.Stream()
            sps.sps_batch_enqueue(b, stream)
            stream.synchronize()
            want = []
            for bm in beams:
                g = torch.zeros((2, 256, 512), dtype=torch.int16, device="cuda")
                k = sps.sps_cnn_pool_tile_grid(bm["snr"], bm["nout"], SCALE, g)
                want.append(g[:k])
            want = torch.cat(want)
            tiles = torch.zeros((want.shape[0], 256, 512), dtype=torch.int16, device="cuda")
            assert sps.sps_batch_set_tiles(b, tiles, SCALE) == want.shape[0] == 4
            for rep in range(3):
                tiles.zero_()
                stream.wait_stream(torch.cuda.current_stream())
                if rep == 0:
                    sps.sps_batch_enqueue(b, stream)
                else:
                    sps.sps_batch_launch_graph(b, stream)
                stream.synchronize()
                assert torch.equal(tiles, want), rep
            with pytest.raises(sps.SpsError):
                sps.sps_batch_candidates(b, 0)
            # back to the search mode: candidates again
            sps.sps_batch_set_tiles(b, None)
            sps.sps_batch_launch_graph(b, stream)
            stream.synchronize()
            full = [sps.sps_batch_candidates(b, i) for i in range(len(beams))]
        # a batch without planes: the same tiles in tile mode, the same
        # candidates when switched back
        bare = [dict(bm, snr=None, best_w=None) for bm in beams]
        with sps.sps_batch_create(plan, bare, list(wl.widths), 8.0, 64, 4096, 16, 64) as b:
            stream = torch.cuda.Stream()
            assert sps.sps_batch_set_tiles(b, tiles, SCALE) == 4
            tiles.zero_()
            stream.wait_stream(torch.cuda.current_stream())
            sps.sps_batch_launch_graph(b, stream)
            stream.synchronize()
            assert torch.equal(tiles, want), "tiles without planes"
            sps.sps_batch_set_tiles(b, None)
            sps.sps_batch_launch_graph(b, stream)
            stream.synchronize()
            for i in range(len(beams)):
                c, n = sps.sps_batch_candidates(b, i)
                assert n == full[i][1] and np.array_equal(c, full[i][0]), f"beam {i}"
