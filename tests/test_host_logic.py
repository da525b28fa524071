"""Host-side logic that needs no GPU: the benchmark's refusal of several
GPUs and its counter-summary guard, the workload descriptions the
benchmark and the tests share, and the detector-versus-boxcar judging rule
on hand-made head outputs."""
import math
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from sps_inputs import workloads  # noqa: E402


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line


def test_bench_counter_guard():
    # the counter figures are used only for the workload, tiling and kernel
    # source they were taken on
    import hashlib

    import bench
    wl = workloads.FULL_SCALE
    default = dict(m=5, dpw=1, nw=16, cs=16, waves_per_eu=8)
    src = os.path.join(ROOT, "paper_2511_02328_amd", "csrc", "dedisperse.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    summary = open(os.path.join(ROOT, "profiles", "full_scale_path_counters.txt")).read()
    got = bench.measured_counters(wl, default)
    if f"dedisperse_source_sha256_16: {sha}" in summary:
        assert got is not None and got["traffic"] > 1e10 and 0.5 < got["ops_per_add"] < 1.2
    else:
        assert got is None
    assert bench.measured_counters(wl, dict(default, waves_per_eu=4)) is None
    assert bench.measured_counters(workloads.SINGLE_BEAM, default) is None


def test_full_scale_workload_figures():
    wl = workloads.FULL_SCALE
    assert (wl.nchan, wl.ndm, wl.nout) == (4096, 2048, 1 << 20)
    assert wl.sample_adds() == 2048 * 4096 * (1 << 20) == 8796093022208
    assert wl.dm_time_samples() == 2048 * (1 << 20)
    f = wl.freqs_mhz()
    # channel centres, channel 0 at the top, reference at the upper band edge
    assert f[0] == pytest.approx(1500.0 - 0.5 * 500.0 / 4096)
    assert np.all(np.diff(f) < 0) and wl.fref_mhz == 1500.0
    dms = wl.dms()
    assert dms[0] == 0.0 and dms[-1] == 2047.0 and np.allclose(np.diff(dms), 1.0)
    assert list(wl.widths) == [1 << i for i in range(9)]


def test_batched_and_streaming_compositions():
    bw = workloads.BATCHED
    lengths = bw.beam_lengths()
    assert len(lengths) == 19 and set(lengths) <= {1 << 18, 1 << 19, 1 << 20}
    assert lengths == bw.beam_lengths()  # seeded
    sw = workloads.STREAMING
    streams = sw.streams()
    assert len(streams) == 24
    counts = {}
    for s in streams:
        counts[(s.nchan, s.ndm, s.nout)] = counts.get((s.nchan, s.ndm, s.nout), 0) + 1
    assert counts == {(1024, 1024, 1 << 18): 8, (4096, 2048, 1 << 20): 12,
                      (8192, 4096, 1 << 18): 4}


def test_paper_sweep_shapes():
    """The two dedispersion timing sweeps of Sec. 3.1 (channel count) and
    Sec. 3.2 (trial DMs): 40 us sampling, 500 MHz around 1250 MHz, DMs 0-1024."""
    ch, dm = workloads.SWEEPS["sweep_channels"], workloads.SWEEPS["sweep_dms"]
    assert [w.nchan for w in ch] == [512, 1024, 2048, 4096, 8192]
    assert {(w.ndm, w.nout) for w in ch} == {(1500, 550000)}   # 22 s span
    assert [w.ndm for w in dm] == [512, 1024, 2048, 4096, 8192]
    assert {(w.nchan, w.nout) for w in dm} == {(2048, 500000)}  # 20 s span
    for w in ch + dm:
        assert w.tsamp_s == 40e-6 and (w.f_lo_mhz + w.f_hi_mhz) / 2 == 1250.0
        assert w.f_hi_mhz - w.f_lo_mhz == 500.0
        assert w.dms()[0] == 0.0 and w.dms()[-1] == pytest.approx(1024.0)


def _meta(n_pos, n_neg):
    n = n_pos + n_neg
    meta = {
        "positive": np.array([True] * n_pos + [False] * n_neg),
        "pulse_snr": np.full(n, 12.0),
        "fwhm_s": np.full(n, 1e-3),
        "d_star": np.full(n, 100.0),
        "t_star": np.full(n, 1000.0),
        "pseudo_d": np.full(n, 300.0),
        "pseudo_t": np.full(n, 3000.0),
        "pseudo_fws": np.full(n, 10.0),
        "boxcar_hit": np.array([True] * n_pos + [False] * n_neg),
        "boxcar_any": np.array([True] * n_pos + [False] * n_neg),
        "boxcar_chance": np.zeros(n, bool),
    }
    return meta


def test_judging_rule_on_hand_made_heads():
    from paper_2511_02328_amd import detector
    n_pos, n_neg = 3, 2
    meta = _meta(n_pos, n_neg)
    head = np.full((n_pos + n_neg, 3, 8, 16), -20.0, np.float32)  # nothing fires
    # tile 0: a confident cell whose offsets put the detection on the pulse
    # (row 100 of 512 trials = cell row 1 + 36/64, sample 1000 = cell 3 + 232/256)
    cell_rows = detector.CELL[0] * detector.POOL[0]
    cell_cols = detector.CELL[1] * detector.POOL[1]
    gy, gx = 100 // cell_rows, 1000 // cell_cols
    head[0, 0, gy, gx] = 5.0
    head[0, 1, gy, gx] = 100 / cell_rows - gy
    head[0, 2, gy, gx] = 1000 / cell_cols - gx
    # tile 1: confident but placed 40 trials away (outside the matching rule)
    head[1, 0, gy, gx] = 5.0
    head[1, 1, gy, gx] = (100 + 40) / cell_rows - gy
    head[1, 2, gy, gx] = 1000 / cell_cols - gx
    # tile 3 (pulse-free): a false alarm far from its pseudo pulse
    head[3, 0, 0, 0] = 5.0
    r = detector.compare_with_boxcar(head, meta, 0.5)
    assert r["n_positive_snr_ge_min"] == 3 and r["n_negative"] == 2
    assert r["cnn_recall"] == pytest.approx(1 / 3)
    assert r["cnn_false_alarm_rate"] == pytest.approx(0.5)
    assert r["cnn_chance_match_rate"] == 0.0
    assert r["boxcar_recall"] == 1.0 and r["boxcar_false_alarm_rate"] == 0.0
    # the threshold is a probability: logit 5 fires at p = 0.99, not at 0.999
    p = 1 / (1 + math.exp(-5.0))
    assert detector.compare_with_boxcar(head, meta, p - 1e-6)["cnn_recall"] == pytest.approx(1 / 3)
    assert detector.compare_with_boxcar(head, meta, 0.999)["cnn_recall"] == 0.0
