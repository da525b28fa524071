"""GPU test of sps_detect_noalloc, detection on the library's fixed device
scratch: through the C ABI its candidates equal those of sps_detect (and of
the oracle's tile / threshold / greedy-suppression rule) on two calls in a
row, the second on a smaller plane, with no device memory taken by the
calls; a plane whose scratch would exceed the fixed array is refused before
anything is enqueued."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from sps_inputs.workloads import Workload  # noqa: E402

pytestmark = pytest.mark.gpu

WIDTHS = [1, 2, 4, 8]


@pytest.fixture(scope="module")
def sps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_02328_amd import sps as mod
    mod.library()
    return mod


def _plane(seed, ndm, nout, ties):
    rng = np.random.Generator(np.random.PCG64(seed))
    snr = rng.uniform(1.0, 60.0, (ndm, nout)).astype(np.float32)
    snr[rng.integers(0, ndm, ties), rng.integers(0, nout, ties)] = 61.0
    best = rng.integers(0, len(WIDTHS), (ndm, nout)).astype(np.uint8)
    return snr, best


def _same(a, b, label):
    (ca, na), (cb, nb) = a, b
    assert na == nb, label
    for f in ("dm_idx", "t_idx", "width", "snr", "dm", "toa_s"):
        assert np.array_equal(ca[f], cb[f]), f"{label}: field {f}"


def _against_oracle(cands, n, snr, best, args, label):
    co = oracle.detect(snr, best, *args, cap=1 << 20)
    assert n == co["n_found"], label
    assert np.array_equal(cands["dm_idx"], co["d"]), label
    assert np.array_equal(cands["t_idx"], co["t"]), label
    assert np.array_equal(cands["snr"], co["snr"]), label
    assert list(cands["width"]) == [WIDTHS[i] for i in co["w"]], label


def test_noalloc_equals_detect_on_two_calls(sps):
    # first: 30,000 tiles (offers beyond what the selection keeps in LDS, so
    # the global arrays of the scratch are used); second: a smaller plane of
    # 700 tiles, which must not see the first call's contents
    cases = [
        ("30,000 tiles", _plane(31, 100, 30000, 50), (0.5, 1, 100, 1, 100)),
        ("700 tiles", _plane(32, 100, 700, 5), (0.5, 1, 100, 1, 100)),
    ]
    planes = [(label, torch.from_numpy(s).cuda(), torch.from_numpy(b).cuda(), s, b, a)
              for label, (s, b), a in cases]
    wl = Workload("noalloc", 8, 1000.0, 1500.0, 1e-4, 16, 100, 0.0, 10.0, (1,))
    with sps.plan_for(wl) as plan:
        # the process's first launch loads the library's code object (device
        # memory of its own); a one-tile call does that before measuring
        tiny = torch.ones((100, 16), dtype=torch.float32, device="cuda")
        tiny_w = torch.zeros((100, 16), dtype=torch.uint8, device="cuda")
        sps.sps_detect_noalloc(plan, tiny, tiny_w, 16, WIDTHS, 0.5, 100, 16, 1, 1)
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        got = []
        for label, sd, bd, s, b, a in planes:
            print(f"case sps_detect_noalloc {label}: plane {s.shape}", flush=True)
            got.append(sps.sps_detect_noalloc(plan, sd, bd, s.shape[1], WIDTHS, *a,
                                              cap=1 << 20))
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        # sps_detect on this fresh plan would take ~1.6 MB for the first plane
        assert free0 - free1 < (1 << 20), "the no-alloc calls took device memory"
        for (label, sd, bd, s, b, a), g in zip(planes, got):
            ref = sps.sps_detect(plan, sd, bd, s.shape[1], WIDTHS, *a, cap=1 << 20)
            _same(g, ref, label)
            _against_oracle(g[0], g[1], s, b, a, label)
            assert g[1] > 0, label


def test_noalloc_refuses_planes_beyond_the_fixed_scratch(sps):
    # 200 x 70,000 samples in 1 x 100 tiles: 140,000 tiles, beyond the 4 MiB array
    wl = Workload("noalloc", 8, 1000.0, 1500.0, 1e-4, 16, 200, 0.0, 10.0, (1,))
    snr = torch.zeros((200, 70000), dtype=torch.float32, device="cuda")
    best = torch.zeros((200, 70000), dtype=torch.uint8, device="cuda")
    with sps.plan_for(wl) as plan:
        with pytest.raises(sps.SpsError, match="fixed scratch"):
            sps.sps_detect_noalloc(plan, snr, best, 70000, WIDTHS, 1.0, 1, 100, 1, 100)
        # near the stated size it runs: 200 x 326 = 65,200 tiles, all below threshold
        c, n = sps.sps_detect_noalloc(plan, snr, best, 70000, WIDTHS, 1.0, 1, 215, 1, 100)
        assert n == 0 and len(c) == 0
