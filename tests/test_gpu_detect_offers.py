"""GPU parity of detection with any number of offers: planes whose tile
maxima above the threshold number well beyond what the selection kernel
keeps in LDS (8192), and suppression radii beyond the plane, against the
oracle's tile / threshold / greedy-suppression rule (candidate record of
Sec. 2), candidate for candidate and in order."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from sps_inputs.workloads import Workload  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_02328_amd import sps as mod
    mod.library()
    return mod


def _plane(seed, ndm, nout, ties=200):
    rng = np.random.Generator(np.random.PCG64(seed))
    snr = rng.uniform(1.0, 60.0, (ndm, nout)).astype(np.float32)
    # exact ties across tiles: the order falls to t, then d
    snr[rng.integers(0, ndm, ties), rng.integers(0, nout, ties)] = 61.0
    best = rng.integers(0, 4, (ndm, nout)).astype(np.uint8)
    return snr, best


def _plan(sps, ndm):
    return sps.plan_for(Workload("d", 8, 1000.0, 1500.0, 1e-4, 16, ndm, 0.0, 10.0, (1,)))


def _compare(sps, snr, best, thr, td, tt, rd, rt, label, plan=None):
    ndm, nout = snr.shape
    widths = [1, 2, 4, 8]
    co = oracle.detect(snr, best, thr, td, tt, rd, rt, cap=1 << 20)
    print(f"case {label}: plane {ndm}x{nout}, tiles {td}x{tt}, radius {rd}x{rt}", flush=True)
    own = plan is None
    if own:
        plan = _plan(sps, ndm)
    try:
        cands, n = sps.sps_detect(plan, torch.from_numpy(snr).cuda(),
                                  torch.from_numpy(best).cuda(), nout, widths, thr, td, tt, rd,
                                  rt, cap=1 << 20)
    finally:
        if own:
            sps.sps_plan_destroy(plan)
    assert n == co["n_found"], label
    assert np.array_equal(cands["dm_idx"], co["d"]), label
    assert np.array_equal(cands["t_idx"], co["t"]), label
    assert np.array_equal(cands["snr"], co["snr"]), label
    assert list(cands["width"]) == [widths[i] for i in co["w"]], label
    return n


# offers: 20,000 (4 LDS blocks of the sort); 12,000 (2 blocks); 9,000 tiles
# with a few hundred offers (global tile map, sort within one LDS block)
@pytest.mark.parametrize("case", [
    dict(ndm=200, nout=20000, td=2, tt=100, rd=1, rt=50, thr=0.5),
    dict(ndm=120, nout=10000, td=1, tt=100, rd=2, rt=150, thr=0.5),
    dict(ndm=90, nout=10000, td=1, tt=100, rd=3, rt=300, thr=57.0),
])
def test_many_offers_match_oracle(sps, case):
    snr, best = _plane(7 + case["ndm"], case["ndm"], case["nout"])
    n = _compare(sps, snr, best, case["thr"], case["td"], case["tt"], case["rd"], case["rt"],
                 str(case))
    assert n > 0


def test_radius_beyond_the_plane(sps):
    # radii of INT_MAX trials and 2^62 samples act as the plane's extent:
    # exactly one candidate, the plane's maximum, from 20,000 offers
    snr, best = _plane(11, 200, 20000, ties=0)
    n = _compare(sps, snr, best, 0.5, 2, 100, 2**31 - 1, 2**62, "radius beyond the plane")
    assert n == 1


def test_offer_count_grows_and_shrinks(sps):
    # one plan, scratch grown for the large plane, then reused for a small one
    big, bb = _plane(21, 100, 30000, ties=50)
    small, sb = _plane(22, 100, 700, ties=5)
    with _plan(sps, 100) as plan:
        _compare(sps, big, bb, 0.5, 1, 100, 1, 100, "30,000 offers", plan)
        _compare(sps, small, sb, 0.5, 1, 100, 1, 100, "700 offers", plan)
        _compare(sps, big, bb, 0.5, 1, 100, 1, 100, "30,000 offers again", plan)
