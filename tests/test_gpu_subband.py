"""GPU parity for the paper's own method and its pre-processing, through the
C ABI: subband tables and two-stage dedispersion bit-exact against the
oracle (and against brute force when N0 = 1), zero-DM filter and square-law
downsampling bit-exact."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from sps_inputs import synth  # noqa: E402
from sps_inputs.workloads import SINGLE_BEAM  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_02328_amd import sps as mod
    mod.library()
    return mod


def pitched(X, nsamp, pad=1):
    p = ((nsamp + 15) // 16) * 16 + 16 * pad
    t = torch.full((X.shape[0], max(p, 16)), 0x5A, dtype=torch.uint8, device="cuda")
    t[:, :nsamp] = torch.from_numpy(np.ascontiguousarray(X[:, :nsamp])).cuda()
    return t


def _plan(sps, wl, ndm, n0, nsub):
    ddm = (wl.dm_hi - wl.dm_lo) / (wl.ndm - 1)
    return sps.sps_subband_plan_create(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, ndm, wl.dm_lo, ddm,
                                       n0, nsub), ddm


@pytest.mark.parametrize("ndm,n0,nsub,nout,zero_pad", [
    (512, 8, 32, 4096, False), (96, 4, 16, 777, False), (100, 3, 5, 1281, True),
    (64, 1, 8, 2000, False), (33, 16, 1, 5, True), (40, 2, 256, 300, False)])
def test_subband_matches_oracle(sps, ndm, n0, nsub, nout, zero_pad):
    wl = SINGLE_BEAM
    plan, ddm = _plan(sps, wl, ndm, n0, nsub)
    with plan:
        Dc, R, F, mx = sps.sps_subband_tables(plan)
        sub = oracle.equal_subbands(wl.nchan, nsub)
        Ro, Fo, dmc = oracle.subband_residuals(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, sub, ndm,
                                               wl.dm_lo, ddm, n0)
        Dco = oracle.delays(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, dmc)
        assert np.array_equal(Dc, Dco) and np.array_equal(R, Ro) and np.array_equal(F, Fo)
        nsamp = nout + mx - (500 if zero_pad else 0)
        X = synth.random_bytes(wl.nchan, max(nsamp, 1), seed=ndm + n0)
        Xd = pitched(X, max(nsamp, 1))
        Y = torch.empty((ndm, nout), dtype=torch.int32, device="cuda")
        sps.sps_dedisperse_subband(plan, Xd, max(nsamp, 1), Y, nout,
                                   sps.SPS_ZERO_PAD if zero_pad else 0)
        torch.cuda.synchronize()
        Yo = oracle.subband_dedisperse(X, Dco, sub, Ro, n0, nout, max(nsamp, 1))
        assert np.array_equal(Y.cpu().numpy().view(np.uint32), Yo)
        if n0 == 1:
            Yb = torch.empty_like(Y)
            sps.sps_dedisperse(plan, Xd, max(nsamp, 1), Yb, nout)
            torch.cuda.synchronize()
            assert torch.equal(Y, Yb)


def test_subband_pulse_and_strict_check(sps):
    wl = SINGLE_BEAM
    plan, ddm = _plan(sps, wl, wl.ndm, 8, 32)
    with plan:
        _, _, _, mx = sps.sps_subband_tables(plan)
        X, truth = synth.make_filterbank(wl, wl.nout + mx)
        Xd = pitched(X, wl.nout + mx)
        Y = torch.empty((wl.ndm, wl.nout), dtype=torch.int32, device="cuda")
        with pytest.raises(sps.SpsError):
            sps.sps_dedisperse_subband(plan, Xd, wl.nout + mx - 1, Y, wl.nout)
        sps.sps_dedisperse_subband(plan, Xd, wl.nout + mx, Y, wl.nout)
        snr = torch.empty((wl.ndm, wl.nout), dtype=torch.float32, device="cuda")
        best = torch.empty((wl.ndm, wl.nout), dtype=torch.uint8, device="cuda")
        sps.sps_boxcar_snr(plan, Y, wl.nout, wl.widths, snr, best)
        cands, n = sps.sps_detect(plan, snr, best, wl.nout, wl.widths, 8.0, 64, 4096, 16, 128)
    assert n >= 1 and abs(cands[0]["dm"] - 300) < 20 and abs(cands[0]["toa_s"] - truth.pulses[0].toa_s) < 0.2


@pytest.mark.parametrize("nchan,nsamp,inplace", [(256, 4096, False), (37, 1001, False),
                                                 (4096, 333, True), (1, 64, False)])
def test_zero_dm(sps, nchan, nsamp, inplace):
    X = synth.random_bytes(nchan, nsamp, seed=nchan)
    X[:, 10:14] = 250
    Xd = pitched(X, nsamp)
    Xo = Xd if inplace else torch.zeros_like(Xd)
    sps.sps_zero_dm(Xd, nsamp, Xo)
    torch.cuda.synchronize()
    assert np.array_equal(Xo[:, :nsamp].cpu().numpy(), oracle.zero_dm(X, nsamp))


@pytest.mark.parametrize("factor,nsamp", [(1, 100), (2, 4096), (3, 1000), (8, 27460), (64, 6000)])
def test_downsample(sps, factor, nsamp):
    X = synth.random_bytes(64, nsamp, seed=factor)
    X[3] = 255
    X[4] = 0
    Xd = pitched(X, nsamp)
    nb = nsamp // factor
    Xo = torch.zeros((64, ((nb + 15) // 16) * 16 + 16), dtype=torch.uint8, device="cuda")
    sps.sps_downsample_sqrt(Xd, nsamp, factor, Xo)
    torch.cuda.synchronize()
    assert np.array_equal(Xo[:, :nb].cpu().numpy(), oracle.downsample_sqrt(X, factor, nsamp))


@pytest.mark.parametrize("nsub", [32, 8])
def test_autotuned_stage1_form_identical(sps, nsub):
    # the autotuner times both stage-1 forms and keeps the faster; the output
    # is the same either way
    wl = SINGLE_BEAM
    plan, _ = _plan(sps, wl, wl.ndm, 8, nsub)
    with plan:
        _, _, _, mx = sps.sps_subband_tables(plan)
        nsamp = wl.nout + mx
        X = synth.random_bytes(wl.nchan, nsamp, seed=77)
        Xd = pitched(X, nsamp)
        Y0 = torch.empty((wl.ndm, wl.nout), dtype=torch.int32, device="cuda")
        sps.sps_dedisperse_subband(plan, Xd, nsamp, Y0, wl.nout)
        sps.sps_plan_autotune(plan, 4096, 2)
        Y1 = torch.empty_like(Y0)
        sps.sps_dedisperse_subband(plan, Xd, nsamp, Y1, wl.nout)
        torch.cuda.synchronize()
        assert torch.equal(Y0, Y1)
