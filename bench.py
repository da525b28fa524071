"""Throughput of the single-pulse search hot path on one GPU.

One step = one chunk of the full-scale workload through the whole path:
brute-force dedispersion (4096 channels, 2048 trial DMs, 2^20 output
samples), per-row median/MAD, boxcar S/N for widths 1..256 and candidate
detection, with the filterbank already resident in device memory.  Prints
one JSON line: DM x time samples per second, the real-time factor
R = t_obs / t_c (t_obs = dedispersed span, t_c = GPU time per chunk), chunk
latency percentiles, the dedispersion kernel's position against the integer
ALU roof (HIP events on the launch stream), and the CPU oracle timed on a
bounded sample of the same chunk.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X vector ALU: 256 CUs x 64 lanes x 2.4 GHz, two 32-bit lane-ops per
# lane per clock -- the rate behind the published 157.3 TFLOP/s FP32 vector
# peak (two FMAs = four flops per lane per clock).  Two-operand integer ops
# (v_add_u32) reach it; three-operand ops (v_add3_u32, v_perm_b32) issue at
# half of it (sps_probe_peaks measures both on the device).
ALU_PEAK_TOPS = 256 * 64 * 2 * 2.4e9 / 1e12
# LDS reads: 256 B per clock per CU with 16-byte reads (CDNA4 doubled CDNA3's
# 128 B; the probe sustains about 0.92 of this).  The dedispersion kernel's
# window reads are 4-byte, for which the probe finds about half of it.
LDS_PEAK_BPS = 256 * 256 * 2.4e9
# Dense BF16 matrix cores.
BF16_PEAK_TFLOPS = 2500.0
# HBM3E.
HBM_PEAK_BPS = 8.0e12
# True-positive rule of the paper's evaluation (Sec. 5.1): a candidate
# matches an injected pulse when its DM is within 20 pc cm^-3 and its arrival
# time at the top of the band within 0.2 s.
TP_RULE = {"abs_ddm_lt": 20.0, "abs_dtoa_lt_s": 0.2}


def injection_recovery(cands, n_found, pulses):
    """Injected pulses with at least one matching candidate, and candidates
    that match no injected pulse (RFI and noise), under TP_RULE."""
    dm = np.asarray(cands["dm"], np.float64)
    toa = np.asarray(cands["toa_s"], np.float64)
    hit = np.zeros(len(dm), bool)
    rec = 0
    for p in pulses:
        m = (np.abs(dm - p.dm) < TP_RULE["abs_ddm_lt"]) & \
            (np.abs(toa - p.toa_s) < TP_RULE["abs_dtoa_lt_s"])
        rec += bool(m.any())
        hit |= m
    return {"recovered": int(rec), "recall": rec / max(1, len(pulses)),
            "candidates": int(n_found), "read_back": int(len(dm)),
            "unmatched_candidates": int((~hit).sum())}


def measured_counters(wl, tiling):
    """Figures of the committed counter summary (calibrated HBM bytes per
    dedispersion launch, VALU lane-ops per sample-add), if it was taken on
    this workload, tiling and kernel source; otherwise None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "full_scale_path_counters.txt")
    src = os.path.join(ROOT, "paper_2511_02328_amd", "csrc", "dedisperse.hip")
    if wl.name != "full_scale_4096ch_2p20t_2048dm" or not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if vals.get("dedisperse_source_sha256_16") != sha:
        return None
    args = vals.get("dedisperse_kernel_name", "").split("<")[-1].rstrip(">").split(",")
    if len(args) < 6 or [int(a) for a in (args[0], args[1], args[2], args[3], args[5])] != [
            tiling["m"], tiling["dpw"], tiling["nw"], tiling["cs"], tiling["waves_per_eu"]]:
        return None
    return {"traffic": float(vals["dedisperse_hbm_bytes_calibrated"]),
            "ops_per_add": float(vals["dedisperse_valu_lane_ops_per_sample_add"])}


# Vector instructions per 16-channel slab of the dedispersion kernel's inner
# loop, per lane (320 sample-adds: 20 outputs x 16 channels), read from its
# ISA: byte permutes, three-input adds and address adds.  The first two are
# three-operand ops, which take two of the ALU's lane-op issue slots.
SLAB_PERMS, SLAB_ADD3S, SLAB_ADDS, SLAB_SAMPLE_ADDS = 160, 80, 18, 320
SLAB_SLOTS_PER_ADD = (2 * SLAB_PERMS + 2 * SLAB_ADD3S + SLAB_ADDS) / SLAB_SAMPLE_ADDS


def measured_peaks(sps, achieved_tops, lds_bytes_per_add=None):
    """The device's sustained instruction and LDS read rates from the
    library's probes (run after the timed region), the sample-add rate the
    dedispersion slab loop's instruction mix would reach at them with every
    issue slot used, and the kernel's fraction of each."""
    p = sps.sps_probe_peaks(0)
    mix = SLAB_SAMPLE_ADDS / (SLAB_PERMS / p["valu_perm_ops_per_s"]
                              + SLAB_ADD3S / p["valu_add3_ops_per_s"]
                              + SLAB_ADDS / p["valu_add_ops_per_s"])
    out = {"valu_add_tops": p["valu_add_ops_per_s"] / 1e12,
           "valu_add3_tops": p["valu_add3_ops_per_s"] / 1e12,
           "valu_perm_tops": p["valu_perm_ops_per_s"] / 1e12,
           "lds_read_tbps": p["lds_read_bytes_per_s"] / 1e12,
           "lds_read32_tbps": p["lds_read32_bytes_per_s"] / 1e12,
           "slab_mix_tops": mix / 1e12,
           "frac_of_valu_add": achieved_tops * 1e12 / p["valu_add_ops_per_s"],
           "frac_of_slab_mix": achieved_tops * 1e12 / mix}
    if lds_bytes_per_add:  # against the 4-byte read rate, the kernel's access width
        out["lds_read_frac"] = (achieved_tops * 1e12 * lds_bytes_per_add
                                / p["lds_read32_bytes_per_s"])
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="full_scale_4096ch_2p20t_2048dm")
    ap.add_argument("--cpu-rows", type=int, default=128,
                    help="DM rows of the chunk the CPU oracle processes (0 = skip)")
    ap.add_argument("--tiling", default="", help="m,dpw,nw,cs[,waves_per_eu] override of the dedispersion tiling")
    ap.add_argument("--method", default="brute", choices=["brute", "subband"],
                    help="dedispersion method for the single-filterbank workloads")
    ap.add_argument("--n0", type=int, default=8, help="subband method: coarse DM step in fine steps")
    ap.add_argument("--nsub", type=int, default=32, help="subband method: number of subbands")
    ap.add_argument("--compression", type=float, default=8.0,
                    help="streaming: chunks arrive this many times faster than real time")
    ap.add_argument("--run-s", type=float, default=40.0, help="streaming: wall-clock run length")
    ap.add_argument("--workers", type=int, default=2, help="streaming: worker threads/HIP streams")
    ap.add_argument("--hbm-budget-gb", type=float, default=200.0,
                    help="streaming: device memory the server may hold (GB)")
    ap.add_argument("--nsrc", type=int, default=2,
                    help="streaming: distinct synthetic chunks per set-up, cycled by its streams")
    ap.add_argument("--stream-detector-tiles", type=int, default=32768,
                    help="streaming: tiles the learned detector every stream runs is trained on "
                         "before serving (0 = no detector)")
    ap.add_argument("--stream-detector-epochs", type=int, default=3)
    ap.add_argument("--stream-detector-threshold", type=float, default=0.9)
    ap.add_argument("--train-tiles", type=int, default=200000,
                    help="detector: training tiles generated by the search")
    ap.add_argument("--val-tiles", type=int, default=10000, help="detector: held-out tiles")
    ap.add_argument("--epochs", type=int, default=6, help="detector: passes over the training set")
    ap.add_argument("--batch", type=int, default=256, help="detector: tiles per training step")
    ap.add_argument("--lr", type=float, default=2e-3, help="detector: peak Adam learning rate")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (reference "
                         "dispatch for scaling hardware byte counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the hot path is measured per GPU "
              "(see the design notes for how it shards); --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2511_02328_amd import sps

    from sps_inputs import synth
    from sps_inputs.workloads import BATCH_WORKLOADS, STREAMING_WORKLOADS, SWEEPS, WORKLOADS

    if args.workload == "detector":
        return bench_detector(args)
    if args.workload in STREAMING_WORKLOADS:
        return bench_streaming(args, STREAMING_WORKLOADS[args.workload])
    if args.workload in BATCH_WORKLOADS:
        return bench_batched(args, BATCH_WORKLOADS[args.workload])
    if args.workload in SWEEPS:
        return bench_sweep(args, args.workload, SWEEPS[args.workload])
    if args.method == "subband":
        return bench_subband(args, WORKLOADS[args.workload])
    wl = WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    dev = "cuda"
    plan = sps.plan_for(wl)
    if args.tiling:
        sps.sps_plan_set_tiling(plan, *[int(x) for x in args.tiling.split(",")])
    tiling = sps.sps_plan_get_tiling(plan)
    _, dmax = sps.sps_plan_delays(plan)
    nsamp = wl.nout + dmax
    pitch = (nsamp + 255) // 256 * 256
    print(f"[bench] {wl.name}: nsamp_in {nsamp}, tiling {tiling}; generating input", flush=True)
    X, truth = synth.make_filterbank(wl, nsamp, device=dev, pitch=pitch)
    Y = torch.empty((wl.ndm, wl.nout), dtype=torch.int32, device=dev)
    snr = torch.empty((wl.ndm, wl.nout), dtype=torch.float32, device=dev)
    best = torch.empty((wl.ndm, wl.nout), dtype=torch.uint8, device=dev)
    st = torch.empty((wl.ndm, 2), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    det = dict(threshold=8.0, tile_dm=64, tile_t=4096, nms_dm=16, nms_t=2 * max(wl.widths))

    def step(ev=None, Xin=None, cap=4096):
        if ev is not None:
            ev[0].record(stream)
        sps.sps_dedisperse(plan, X if Xin is None else Xin, nsamp, Y, wl.nout, stream=stream)
        if ev is not None:
            ev[1].record(stream)
        # statistics, boxcar S/N and detection in one call: the boxcar pass
        # gathers the tile maxima, so detection does not re-read the S/N plane
        cands, n = sps.sps_search(plan, Y, wl.nout, wl.widths, snr, best, st, cap=cap,
                                  stream=stream, allow_truncated=True, **det)
        if ev is not None:
            ev[2].record(stream)
        return cands, n

    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib << 20
        a = torch.ones(n, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        print(f"[bench] calibration copy of {args.copy_calibration_mib} MiB done", flush=True)
    torch.cuda.synchronize()
    print(f"[bench] warmup {args.warmup}", flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        cands, n = step(events[k])  # detect synchronises: the chunk is done on return
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dd = np.array([e[0].elapsed_time(e[1]) for e in events]) / 1e3
    sr = np.array([e[1].elapsed_time(e[2]) for e in events]) / 1e3
    ms_step = wall / args.steps * 1e3
    t_obs = wl.nout * wl.tsamp_s
    print(f"[bench] {args.steps} steps: {ms_step:.2f} ms/step, dedisperse {dd.mean()*1e3:.2f} ms, "
          f"statistics+boxcar+detection {sr.mean()*1e3:.2f} ms, {n} candidates", flush=True)
    # the same search of the last step's plane without S/N or width planes
    # (candidates only): statistics, boxcar and detection at 4 B per output
    wp = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    for k in range(args.steps):
        wp[k][0].record(stream)
        c_np, n_np = sps.sps_search(plan, Y, wl.nout, wl.widths, None, None, st, cap=4096,
                                    stream=stream, allow_truncated=True, **det)
        wp[k][1].record(stream)
    torch.cuda.synchronize()
    sr_np = np.array([e[0].elapsed_time(e[1]) for e in wp]) / 1e3
    same_np = n_np == n and bool(np.array_equal(c_np, cands))
    print(f"[bench] without planes: statistics+boxcar+detection {sr_np.mean()*1e3:.2f} ms, "
          f"same candidates {same_np}", flush=True)

    # injected pulses recovered (outside the timed region), with and without
    # the zero-DM filter in front of the search
    recovery = None
    if truth is not None and truth.pulses:
        recovery = {"rule": TP_RULE, "pulses": len(truth.pulses)}
        cands_all, n_all = step(cap=1 << 17)
        recovery["plain"] = injection_recovery(cands_all, n_all, truth.pulses)
        Xz = torch.empty_like(X)
        sps.sps_zero_dm(X, nsamp, Xz, stream=stream)
        cands_z, n_z = step(Xin=Xz, cap=1 << 17)
        recovery["zero_dm"] = injection_recovery(cands_z, n_z, truth.pulses)
        del Xz
        step()  # the plane of the unfiltered chunk again, for the CPU baseline's row check
        torch.cuda.synchronize()
        print(f"[bench] injected pulses recovered: {recovery['plain']['recovered']} of "
              f"{len(truth.pulses)} ({n_all} candidates); with zero-DM "
              f"{recovery['zero_dm']['recovered']} ({n_z} candidates)", flush=True)

    # host link: the chunk's upload from pinned host memory, timed on the stream
    h2d_ms = None
    try:
        host = torch.empty(X.shape, dtype=torch.uint8, pin_memory=True)
        host.copy_(X)
        torch.cuda.synchronize()
        hx = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        reps = 3
        hx[0].record(stream)
        for _ in range(reps):
            X.copy_(host, non_blocking=True)
        hx[1].record(stream)
        hx[1].synchronize()
        h2d_ms = hx[0].elapsed_time(hx[1]) / reps
        del host
    except RuntimeError as e:  # pinned allocation refused: report without it
        print(f"[bench] host-link timing skipped: {e}", flush=True)

    adds = wl.sample_adds()
    achieved = adds / dd.mean() / 1e12
    counters = measured_counters(wl, tiling)
    rec = {
        "metric": "DM×time samples/s dedispersed+searched",
        "value": wl.dm_time_samples() / (wall / args.steps),
        "unit": "DM-time samples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": wl.name, "nchan": wl.nchan, "ndm": wl.ndm, "nout": wl.nout,
                   "nsamp_in": nsamp, "tsamp_us": wl.tsamp_s * 1e6, "band_mhz": [wl.f_lo_mhz, wl.f_hi_mhz],
                   "widths": list(wl.widths), "seed": wl.seed, "tiling": tiling, "detect": det},
        "real_time_factor": t_obs / (wall / args.steps),
        "real_time_factor_dedisperse_kernel": t_obs / dd.mean(),
        "host_link": None if h2d_ms is None else {
            "h2d_ms": h2d_ms, "gb_per_s": X.numel() / (h2d_ms / 1e3) / 1e9,
            "real_time_factor_with_h2d_serial": t_obs / (wall / args.steps + h2d_ms / 1e3)},
        "chunk_latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                             "p99": float(np.percentile(lat, 99) * 1e3),
                             "chunk_duration_ms": t_obs * 1e3},
        "breakdown_ms": {"dedisperse": dd.mean() * 1e3, "stats_boxcar_detect": sr.mean() * 1e3},
        # the scan stages against 8 TB/s, at their algorithmic bytes:
        # statistics read the plane once (4 B per output), the boxcar reads
        # it and writes S/N and width (4 + 4 + 1 B) and gathers the tile
        # maxima on the way; selection reads only the tile records
        "hbm_stages": {
            "stats_boxcar_detect": {"bytes": 13 * wl.ndm * wl.nout,
                                    "gb_per_s": 13 * wl.ndm * wl.nout / sr.mean() / 1e9,
                                    "frac": 13 * wl.ndm * wl.nout / sr.mean() / HBM_PEAK_BPS},
            # the search writing no planes: statistics and boxcar each read
            # the plane once (4 + 4 B per output)
            "without_planes": {"ms": sr_np.mean() * 1e3, "bytes": 8 * wl.ndm * wl.nout,
                               "gb_per_s": 8 * wl.ndm * wl.nout / sr_np.mean() / 1e9,
                               "frac": 8 * wl.ndm * wl.nout / sr_np.mean() / HBM_PEAK_BPS,
                               "same_candidates": same_np}},
        "candidates": n,
        "injection_recovery": recovery,
        "roofline": {"kernel": "dedisperse_kernel", "bound": "alu", "achieved": achieved,
                     "peak": ALU_PEAK_TOPS, "unit": "TOP/s", "frac": achieved / ALU_PEAK_TOPS,
                     "traffic": counters["traffic"] if counters else None,
                     "traffic_unit": "bytes per launch (FETCH_SIZE x2.0 + WRITE_SIZE x1.0, "
                                     "scaled by a 1 GiB copy)",
                     "work_per_launch": f"{adds} sample-adds (ndm x nout x nchan)",
                     # the packed (SWAR) kernel spends 0.82 VALU lane-ops per
                     # sample-add, mostly three-operand ops that take two issue
                     # slots each: its own ceilings are the ALU's issue slots at
                     # the slab loop's slots per add, and the LDS read rate at
                     # (m+1)/m bytes per add
                     "valu_lane_ops_per_add": counters["ops_per_add"] if counters else None,
                     "issue_slots_per_add": SLAB_SLOTS_PER_ADD,
                     "valu_issue_frac": achieved * SLAB_SLOTS_PER_ADD / ALU_PEAK_TOPS,
                     "lds_read_frac": (achieved * 1e12 * (tiling["m"] + 1) / tiling["m"]
                                       / LDS_PEAK_BPS if tiling["m"] else None),
                     "measured_peaks": measured_peaks(
                         sps, achieved, (tiling["m"] + 1) / tiling["m"] if tiling["m"] else None)},
    }

    if args.cpu_rows > 0:
        rec["cpu_baseline"] = cpu_baseline(wl, X, nsamp, Y, args.cpu_rows, det)
    print(json.dumps(rec), flush=True)
    plan.close()


def bench_batched(args, bw):
    """Many beams of one receiver, one chunk each, replayed from a HIP graph."""
    import torch

    from paper_2511_02328_amd import sps

    from sps_inputs import synth
    wl0 = bw.base
    torch.cuda.set_device(0)
    plan = sps.plan_for(wl0)
    _, dmax = sps.sps_plan_delays(plan)
    lengths = bw.beam_lengths()
    print(f"[bench] {bw.name}: {bw.nbeams} beams, lengths {lengths}", flush=True)
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
    det = dict(threshold=8.0, tile_dm=64, tile_t=4096, nms_dm=16, nms_t=2 * max(wl0.widths))
    batch = sps.sps_batch_create(plan, beams, list(wl0.widths), **det)
    stream = torch.cuda.Stream()
    # the batch times its own batched launch with every tiling (untimed
    # set-up, like the warm-up)
    ms = sps.sps_batch_autotune(batch, 3, stream)
    t_dd, best_i = min((m, i) for i, m in enumerate(ms) if m > 0)
    tiling = sps.sps_tiling_describe(best_i)
    print(f"[bench] batch autotuner: {[round(m, 2) for m in ms]} ms, keeps {tiling}", flush=True)

    def step():
        sps.sps_batch_launch_graph(batch, stream)
        return sum(k for _, k in sps.sps_batch_candidates_all(batch, cap=4096, stream=stream,
                                                              allow_truncated=True))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        n = step()
        lat.append(time.perf_counter() - ts)
    wall = time.perf_counter() - t0
    # GPU time of the four batched launches alone (graph replays, HIP events
    # on the launch stream)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        sps.sps_batch_launch_graph(batch, stream)
    ev1.record(stream)
    ev1.synchronize()
    t_graph = ev0.elapsed_time(ev1) / args.steps / 1e3
    # the same search without S/N or width planes (candidates only; each
    # tile key carries its peak's width): its own autotuned tiling, the same
    # candidates
    bare = sps.sps_batch_create(plan, [dict(b, snr=None, best_w=None) for b in beams],
                                list(wl0.widths), **det)
    sps.sps_batch_autotune(bare, 3, stream)
    sps.sps_batch_launch_graph(batch, stream)
    sps.sps_batch_launch_graph(bare, stream)
    same = True
    for i in range(bw.nbeams):
        cf, nf = sps.sps_batch_candidates(batch, i, cap=4096, stream=stream, allow_truncated=True)
        cb, nb = sps.sps_batch_candidates(bare, i, cap=4096, stream=stream, allow_truncated=True)
        same = same and nf == nb and bool(np.array_equal(cf, cb))

    def step_bare():
        sps.sps_batch_launch_graph(bare, stream)
        return sum(k for _, k in sps.sps_batch_candidates_all(bare, cap=4096, stream=stream,
                                                              allow_truncated=True))

    for _ in range(args.warmup):
        step_bare()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step_bare()
    wall_bare = time.perf_counter() - t0
    ev0.record(stream)
    for _ in range(args.steps):
        sps.sps_batch_launch_graph(bare, stream)
    ev1.record(stream)
    ev1.synchronize()
    t_graph_bare = ev0.elapsed_time(ev1) / args.steps / 1e3
    bare.close()
    samples = sum(wl0.ndm * n for n in lengths)
    adds = samples * wl0.nchan
    durations = [n * wl0.tsamp_s for n in lengths]
    rec = {
        "metric": "DM×time samples/s dedispersed+searched", "value": samples / (wall / args.steps),
        "unit": "DM-time samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": bw.name, "nbeams": bw.nbeams, "nchan": wl0.nchan, "ndm": wl0.ndm,
                   "beam_lengths": lengths, "tsamp_us": wl0.tsamp_s * 1e6,
                   "widths": list(wl0.widths), "tiling": tiling, "autotune_ms": ms,
                   "launch": "one HIP graph per step: batched dedispersion (one workgroup per item) + "
                             "batched stats, boxcar, detection; every beam's candidates read back "
                             "in one call (sps_batch_candidates_all)", "detect": det},
        "chunk_latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                             "p99": float(np.percentile(lat, 99) * 1e3),
                             "shortest_chunk_duration_ms": min(durations) * 1e3},
        "real_time_factor_vs_shortest_chunk": min(durations) / float(np.percentile(lat, 99)),
        "real_time_sustained": bool(np.percentile(lat, 99) < min(durations)),
        "candidates": n,
        "without_planes": {"value": samples / (wall_bare / args.steps),
                           "ms_per_step": wall_bare / args.steps * 1e3,
                           "graph_ms": t_graph_bare * 1e3, "same_candidates": same,
                           "note": "the same search writing no S/N or width plane"},
        # the dominant kernel, timed by the batch autotuner with HIP events on
        # the launch stream (mean of its timed launches of the kept tiling);
        # the whole step's four launches beside it
        "roofline": {"kernel": "dedisperse_batch_kernel", "bound": "alu",
                     "achieved": adds / (t_dd / 1e3) / 1e12, "peak": ALU_PEAK_TOPS, "unit": "TOP/s",
                     "frac": adds / (t_dd / 1e3) / 1e12 / ALU_PEAK_TOPS, "traffic": None,
                     "kernel_ms": t_dd, "graph_ms": t_graph * 1e3,
                     "step_frac": adds / t_graph / 1e12 / ALU_PEAK_TOPS,
                     "work_per_launch": f"{adds} sample-adds (sum over beams of ndm x nout x nchan)",
                     "measured_peaks": measured_peaks(sps, adds / (t_dd / 1e3) / 1e12)},
    }
    print(json.dumps(rec), flush=True)
    batch.close()
    plan.close()


def bench_streaming(args, sw):
    """Mixed real-time streams served by the native streaming runtime: chunks
    arrive on a wall-clock schedule compressed `compression` times, each
    stream keeps its dispersion overlap on the device, every chunk runs
    dedispersion, statistics, boxcar S/N, detection and the learned detector,
    and every chunk's latency (search finished minus arrival) is recorded."""
    import torch

    from paper_2511_02328_amd import sps

    from sps_inputs import synth
    torch.cuda.set_device(0)
    streams = sw.streams()
    setups = []
    for wl in streams:
        if wl not in setups:
            setups.append(wl)
    # host feeds: nsrc distinct chunks per set-up in pinned memory, made on the GPU
    pools = {}
    for wl in setups:
        pool = torch.empty((args.nsrc * wl.nchan, wl.nout), dtype=torch.uint8, pin_memory=True)
        for j in range(args.nsrc):
            X, _ = synth.make_filterbank(wl, wl.nout, seed=wl.seed + 1000 * j, device="cuda")
            pool[j * wl.nchan:(j + 1) * wl.nchan].copy_(X)
            del X
        pools[wl.name] = pool
        print(f"[bench] {wl.name}: {args.nsrc} host chunks of {wl.nchan} x {wl.nout} ready",
              flush=True)
    # the learned detector every stream runs after its boxcar search, trained
    # briefly on tiles the search itself makes
    net, det_info = None, None
    if args.stream_detector_tiles > 0:
        from paper_2511_02328_amd import detector
        fac = detector.TileFactory(batch=64)
        tiles, labels, _ = fac.make(args.stream_detector_tiles, seed=101)
        fac.close()
        net = sps.sps_cnn_create(args.batch)
        sps.sps_cnn_set_params(net, detector.init_params(7))
        losses = detector.train(net, tiles, labels, args.stream_detector_epochs, args.batch,
                                args.lr)
        del tiles, labels
        det_info = {"train_tiles": args.stream_detector_tiles,
                    "epochs": args.stream_detector_epochs,
                    "threshold": args.stream_detector_threshold,
                    "loss_last20": float(np.mean(losses[-20:]))}
        print(f"[bench] detector trained: loss {losses[0]:.4f} -> {det_info['loss_last20']:.4f}",
              flush=True)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    det = dict(threshold=8.0, tile_dm=64, tile_t=4096, nms_dm=16, nms_t=512)
    budget = int(args.hbm_budget_gb * 1e9)
    server = sps.sps_server_create(budget, args.workers)
    if net is not None:  # attached first, so admission counts each stream's tiles
        sps.sps_server_set_detector(server, net, args.stream_detector_threshold,
                                    detector.TILE_SCALE)
    admitted, refused, feeds = [], [], []
    for i, wl in enumerate(streams):
        try:
            sid = sps.sps_server_add_stream(server, wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s,
                                            wl.dms(), wl.widths, chunk_len=wl.nout, **det)
        except sps.SpsError as e:
            if e.name != "SPS_ERR_NOMEM":
                raise
            refused.append(i)
            continue
        admitted.append(wl)
        feeds.append(dict(host=pools[wl.name], nsrc=args.nsrc, first=len(admitted) % args.nsrc))
    mem = sps.sps_server_memory(server)
    print(f"[bench] admitted {len(admitted)} of {len(streams)} streams, "
          f"{mem['used'] / 1e9:.1f} of {mem['budget'] / 1e9:.1f} GB", flush=True)
    # warm-up: one chunk of each set-up on worker 0 (module load, detection scratch)
    for wl in setups:
        if wl in admitted:
            sps.sps_server_push(server, admitted.index(wl), pools[wl.name][:wl.nchan],
                                allow_truncated=True)
    print(f"[bench] serving for {args.run_s:.0f} s at {args.compression:g}x real time", flush=True)
    recs = sps.sps_server_run(server, feeds, args.run_s, args.compression)
    lat = recs["end_s"] - recs["arrival_s"]
    sid = recs["stream"]
    dur = np.array([admitted[s].nout * admitted[s].tsamp_s for s in sid])
    period = dur / args.compression
    samples = float(sum(admitted[s].ndm * admitted[s].nout for s in sid))
    adds = float(sum(admitted[s].sample_adds() for s in sid))
    span = float(recs["end_s"].max() - recs["arrival_s"].min())
    # union of the intervals in which at least one chunk was being searched
    iv = sorted(zip(recs["start_s"], recs["end_s"]))
    busy, cur0, cur1 = 0.0, None, None
    for a, b in iv:
        if cur1 is None or a > cur1:
            if cur1 is not None:
                busy += cur1 - cur0
            cur0, cur1 = a, b
        else:
            cur1 = max(cur1, b)
    busy += cur1 - cur0
    per_setup = {}
    for wl in setups:
        m = np.array([admitted[s].name == wl.name for s in sid])
        if m.any():
            per_setup[wl.name] = {
                "streams": sum(1 for a in admitted if a.name == wl.name), "chunks": int(m.sum()),
                "chunk_duration_s": wl.nout * wl.tsamp_s,
                "mean_queue_ms": float(np.mean(recs["start_s"][m] - recs["arrival_s"][m]) * 1e3),
                "mean_upload_ms": float(np.mean(recs["upload_s"][m] - recs["start_s"][m]) * 1e3),
                "mean_lock_wait_ms": float(np.mean(recs["compute_s"][m] - recs["upload_s"][m]) * 1e3),
                "mean_compute_ms": float(np.mean(recs["end_s"][m] - recs["compute_s"][m]) * 1e3),
                "p50_ms": float(np.percentile(lat[m], 50) * 1e3),
                "p99_ms": float(np.percentile(lat[m], 99) * 1e3),
                "max_ms": float(lat[m].max() * 1e3)}
    rec = {
        "metric": "DM×time samples/s dedispersed+searched", "value": samples / span,
        "unit": "DM-time samples/s", "n_gpus": 1, "steps": int(len(recs)), "warmup": len(setups),
        "ms_per_step": float(np.mean(recs["end_s"] - recs["start_s"]) * 1e3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": sw.name, "streams": [[n, wl.name] for n, wl in sw.groups],
                   "admitted": len(admitted), "refused": refused,
                   "hbm_used_gb": mem["used"] / 1e9, "hbm_budget_gb": mem["budget"] / 1e9,
                   "workers": args.workers, "compression": args.compression,
                   "run_s": args.run_s, "host_chunks_per_setup": args.nsrc, "detect": det,
                   "learned_detector": det_info},
        "chunk_latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                             "p99": float(np.percentile(lat, 99) * 1e3),
                             "max": float(lat.max() * 1e3)},
        "latency_below_chunk_duration": bool(np.all(lat < dur)),
        "real_time_sustained": bool(np.all(lat < period)),
        "busy_fraction": busy / span,
        "real_time_factor": args.compression * span / busy,
        "sample_adds_per_s_busy": adds / busy,
        "alu_frac_over_busy_time": adds / busy / (ALU_PEAK_TOPS * 1e12),
        "per_setup": per_setup,
        "candidates": int(recs["n_cand"].sum()),
        "detector_cells": int(recs["n_cnn"].sum()),
        "roofline": {"kernel": "all chunk work over the GPU's busy time", "bound": "alu",
                     "achieved": adds / busy / 1e12, "peak": ALU_PEAK_TOPS, "unit": "TOP/s",
                     "frac": adds / busy / (ALU_PEAK_TOPS * 1e12), "traffic": None,
                     "work_per_launch": "sample-adds of every searched chunk"},
    }
    print(json.dumps(rec), flush=True)
    server.close()
    if net is not None:
        net.close()


def cnn_flops_per_tile():
    """Multiply-adds x 2 of one tile through the six 3x3 layers (forward)."""
    layers = ((1, 16, 128, 256), (16, 32, 64, 128), (32, 64, 32, 64), (64, 128, 16, 32),
              (128, 128, 8, 16), (128, 128, 8, 16))
    return sum(2 * 9 * ci * co * h * w for ci, co, h, w in layers)


def bench_detector(args):
    """The learned detector: training set made by the search, BF16-MFMA
    training, comparison with the boxcar search on held-out tiles, and
    inference rate beside the plain search's."""
    import torch

    from paper_2511_02328_amd import detector, sps
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    fac = detector.TileFactory(batch=64)
    t0 = time.perf_counter()
    tr_tiles, tr_labels, tr_meta = fac.make(args.train_tiles, seed=101)
    gen_s = time.perf_counter() - t0
    print(f"[bench] {args.train_tiles} training tiles in {gen_s:.1f} s", flush=True)
    va_tiles, va_labels, va_meta = fac.make(args.val_tiles, seed=202)
    print(f"[bench] {args.val_tiles} held-out tiles", flush=True)
    net = sps.sps_cnn_create(args.batch)
    sps.sps_cnn_set_params(net, detector.init_params(7))
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    losses = detector.train(net, tr_tiles, tr_labels, args.epochs, args.batch, args.lr,
                            stream=stream)
    e1.record(stream)
    e1.synchronize()
    train_ms = e0.elapsed_time(e1)
    steps = len(losses)
    tiles_trained = steps * args.batch
    print(f"[bench] trained {steps} steps in {train_ms / 1e3:.1f} s, loss {losses[0]:.4f} -> "
          f"{np.mean(losses[-20:]):.4f}", flush=True)
    head = detector.cnn_scores(net, va_tiles, args.batch, stream=stream)
    judged = [detector.compare_with_boxcar(head, va_meta, th)
              for th in (0.02, 0.05, 0.1, 0.2, 0.3, 0.5, 0.9, 0.97, 0.99, 0.995, 0.999)]
    by_rfi = {th: detector.compare_by_rfi(head, va_meta, th) for th in (0.1, 0.5, 0.9, 0.99)}
    # operating point: the highest threshold at which the network's recall
    # still matches the boxcar search's
    ok = [j for j in judged if j["cnn_recall"] is not None and j["boxcar_recall"] is not None
          and j["cnn_recall"] >= j["boxcar_recall"]]
    operating = ok[-1] if ok else None
    # inference rate: inference passes of full batches (layer 0 fused into
    # layer 1, its activation not kept)
    for _ in range(3):
        sps.sps_cnn_infer(net, va_tiles[:args.batch], args.batch, stream=stream)
    reps = 20
    e0.record(stream)
    for _ in range(reps):
        sps.sps_cnn_infer(net, va_tiles[:args.batch], args.batch, stream=stream)
    e1.record(stream)
    e1.synchronize()
    fwd_ms = e0.elapsed_time(e1) / reps
    # the plain search on the same GPU: one 64-beam batch (dedispersion,
    # statistics, boxcar, detection) and the pooling of its planes
    for _ in range(2):
        sps.sps_batch_launch_graph(fac.handle, stream)
    e0.record(stream)
    for _ in range(reps):
        sps.sps_batch_launch_graph(fac.handle, stream)
    e1.record(stream)
    e1.synchronize()
    search_ms = e0.elapsed_time(e1) / reps / fac.batch
    # the plain search writing no S/N or width planes (candidates only), on
    # the same beams
    bare = sps.sps_batch_create(
        fac.plan, [dict(X=fac.X[i], nsamp_in=fac.nsamp, nout=fac.wl.nout, Y=fac.Y[i],
                        stats=fac.stats[i], snr=None, best_w=None) for i in range(fac.batch)],
        list(fac.wl.widths), **detector.SEARCH)
    sps.sps_batch_autotune(bare, 3, stream)
    for _ in range(2):
        sps.sps_batch_launch_graph(bare, stream)
    e0.record(stream)
    for _ in range(reps):
        sps.sps_batch_launch_graph(bare, stream)
    e1.record(stream)
    e1.synchronize()
    bare_ms = e0.elapsed_time(e1) / reps / fac.batch
    bare.close()
    # the detector path on the same batch: dedispersion, statistics and the
    # boxcar pass writing the network's tiles directly (no S/N or width
    # planes, no threshold search), then the network on those tiles
    det_tiles = torch.empty((fac.batch, 256, 512), dtype=torch.int16, device="cuda")
    ntl = sps.sps_batch_set_tiles(fac.handle, det_tiles, detector.TILE_SCALE)
    assert ntl == fac.batch

    def detector_path():
        sps.sps_batch_launch_graph(fac.handle, stream)
        sps.sps_cnn_infer(net, det_tiles, fac.batch, stream=stream)

    for _ in range(2):
        detector_path()
    e0.record(stream)
    for _ in range(reps):
        detector_path()
    e1.record(stream)
    e1.synchronize()
    det_path_ms = e0.elapsed_time(e1) / reps / fac.batch
    # the same tiles as the search mode's planes pooled (what the network was
    # trained and judged on)
    sps.sps_batch_set_tiles(fac.handle, None)
    sps.sps_batch_launch_graph(fac.handle, stream)
    ref = torch.empty_like(det_tiles)
    for i in range(fac.batch):
        sps.sps_cnn_pool_tiles(fac.snr[i], fac.wl.nout, detector.TILE_SCALE, ref[i], stream=stream)
    stream.synchronize()
    sps.sps_batch_set_tiles(fac.handle, det_tiles, detector.TILE_SCALE)
    sps.sps_batch_launch_graph(fac.handle, stream)
    stream.synchronize()
    tiles_identical = bool(torch.equal(ref, det_tiles))
    sps.sps_batch_set_tiles(fac.handle, None)
    dm_t_per_tile = fac.wl.ndm * fac.wl.nout
    flops = cnn_flops_per_tile()
    rec = {
        "metric": "detector training tiles/s", "value": tiles_trained / (train_ms / 1e3),
        "unit": "tiles/s", "n_gpus": 1, "steps": steps, "warmup": 0,
        "ms_per_step": train_ms / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "detector_tiles_256x512_bf16", "train_tiles": args.train_tiles,
                   "val_tiles": args.val_tiles, "epochs": args.epochs, "batch": args.batch,
                   "lr": args.lr, "tile_generation_s": gen_s,
                   "search_autotune_ms": [round(x, 3) for x in fac.autotune_ms],
                   "positives_train": int(tr_meta["positive"].sum())},
        "loss_first": float(losses[0]), "loss_last20": float(np.mean(losses[-20:])),
        "train_tflops_mfma_conv": 3 * flops * tiles_trained / (train_ms / 1e3) / 1e12,
        "inference_tiles_per_s": args.batch / (fwd_ms / 1e3),
        "inference_tflops": flops * args.batch / (fwd_ms / 1e3) / 1e12,
        "roofline": {"kernel": "forward pass (six 3x3 conv layers, BF16 MFMA for five)",
                     "bound": "mfma", "achieved": flops * args.batch / (fwd_ms / 1e3) / 1e12,
                     "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": flops * args.batch / (fwd_ms / 1e3) / 1e12 / BF16_PEAK_TFLOPS,
                     "traffic": None,
                     "work_per_launch": f"{flops * args.batch} FLOP per batch of {args.batch} tiles"},
        "search_ms_per_tile": search_ms, "cnn_ms_per_tile": fwd_ms / args.batch,
        # end to end, one 64-beam batch of single-beam filterbanks per step
        "end_to_end": {
            "plain_search": {"ms_per_tile": search_ms, "tiles_per_s": 1e3 / search_ms,
                             "dm_time_samples_per_s": dm_t_per_tile * 1e3 / search_ms},
            "detector_path": {"ms_per_tile": det_path_ms, "tiles_per_s": 1e3 / det_path_ms,
                              "dm_time_samples_per_s": dm_t_per_tile * 1e3 / det_path_ms},
            "detector_path_over_plain": search_ms / det_path_ms,
            "plain_search_without_planes": {"ms_per_tile": bare_ms, "tiles_per_s": 1e3 / bare_ms,
                                            "dm_time_samples_per_s": dm_t_per_tile * 1e3 / bare_ms},
            "detector_path_over_plain_without_planes": bare_ms / det_path_ms,
            "tiles_identical_to_pooled_planes": tiles_identical},
        "operating_point": operating,
        "vs_boxcar_by_rfi": {str(th): {g: {k: (round(v, 4) if isinstance(v, float) else v)
                                        for k, v in r.items()}
                                    for g, r in grp.items()} for th, grp in by_rfi.items()},
        "vs_boxcar_snr_ge_8": judged,
    }
    print(json.dumps(rec), flush=True)
    net.close()
    fac.close()


def bench_subband(args, wl):
    """The paper's two-stage subband dedispersion on the same chunk, against
    brute force: time per chunk and S/N kept at the injected pulses."""
    import torch

    from paper_2511_02328_amd import sps

    from sps_inputs import synth
    torch.cuda.set_device(0)
    ddm = (wl.dm_hi - wl.dm_lo) / (wl.ndm - 1)
    plan = sps.sps_subband_plan_create(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, wl.ndm, wl.dm_lo,
                                       ddm, args.n0, args.nsub)
    _, _, _, emax = sps.sps_subband_tables(plan)
    _, dmax = sps.sps_plan_delays(plan)
    nsamp = wl.nout + max(emax, dmax)
    # the autotuner also picks the stage-1 form (one segmented launch or one
    # launch per subband) on a probe
    sps.sps_plan_autotune(plan, 1 << 18, 2)
    pitch = (nsamp + 255) // 256 * 256
    print(f"[bench] {wl.name}: subband n0={args.n0} nsub={args.nsub}, generating input", flush=True)
    X, truth = synth.make_filterbank(wl, nsamp, device="cuda", pitch=pitch)
    Y = torch.empty((wl.ndm, wl.nout), dtype=torch.int32, device="cuda")
    snr = torch.empty((wl.ndm, wl.nout), dtype=torch.float32, device="cuda")
    best = torch.empty((wl.ndm, wl.nout), dtype=torch.uint8, device="cuda")

    def timed(fn, n):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        torch.cuda.synchronize()
        a.record()
        for _ in range(n):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / n / 1e3

    def peak_snrs():
        sps.sps_boxcar_snr(plan, Y, wl.nout, wl.widths, snr, best)
        torch.cuda.synchronize()
        out = []
        dms = wl.dms()
        for p in truth.pulses:
            d = int(np.argmin(np.abs(dms - p.dm)))
            t = int(round(p.toa_s / wl.tsamp_s))
            d0, d1 = max(0, d - 8), min(wl.ndm, d + 9)
            t0, t1 = max(0, t - 4096), min(wl.nout, t + 4096)
            out.append(float(snr[d0:d1, t0:t1].max()))
        return np.array(out)

    t_sub = timed(lambda: sps.sps_dedisperse_subband(plan, X, nsamp, Y, wl.nout), args.steps)
    s_sub = peak_snrs()
    t_bf = timed(lambda: sps.sps_dedisperse(plan, X, nsamp, Y, wl.nout), max(2, args.steps // 2))
    s_bf = peak_snrs()
    keep = s_sub / np.maximum(s_bf, 1e-9)
    # integer adds of the method: stage 1 (coarse trials x channels x
    # stage-1 row length) + stage 2 (trials x subbands x outputs)
    ncoarse = (wl.ndm + args.n0 - 1) // args.n0
    Dc, R, _, _ = sps.sps_subband_tables(plan)
    len1 = (wl.nout + int(R.max()) + 3) // 4 * 4
    adds = ncoarse * wl.nchan * len1 + wl.ndm * args.nsub * wl.nout
    rec = {
        "metric": "DM×time samples/s dedispersed (subband method)",
        "value": wl.dm_time_samples() / t_sub, "unit": "DM-time samples/s", "n_gpus": 1,
        "steps": args.steps, "dtype": "u8", "data": "synthetic",
        "config": {"workload": wl.name, "method": "subband", "n0": args.n0, "nsub": args.nsub},
        "ms_per_chunk": {"subband": t_sub * 1e3, "brute_force": t_bf * 1e3},
        "speedup_vs_brute_force": t_bf / t_sub,
        "pulse_snr_kept": {"median": float(np.median(keep)), "min": float(keep.min()),
                           "n_pulses": int(keep.size)},
        "roofline": {"kernel": "sps_dedisperse_subband (stage 1 + stage 2)", "bound": "alu",
                     "achieved": adds / t_sub / 1e12, "peak": ALU_PEAK_TOPS, "unit": "TOP/s",
                     "frac": adds / t_sub / 1e12 / ALU_PEAK_TOPS, "traffic": None,
                     "work_per_launch": f"{adds} integer adds (stage 1 + stage 2)"},
    }
    print(json.dumps(rec), flush=True)
    plan.close()


# Dedispersion kernel times the paper prints for its own code at the two
# ends of each sweep (RTX 4090, Sec. 3.1 and 3.2), in seconds: context from
# other hardware, never a target of this line.
PAPER_SWEEP_KERNEL_S = {"sweep_channels": {512: 0.11, 8192: 0.96},
                        "sweep_dms": {512: 0.091, 8192: 1.295}}


def bench_sweep(args, name, points):
    """The paper's dedispersion timing sweeps: kernel time against the number
    of channels (Sec. 3.1, 1500 trials, 22 s span) or of trial DMs (Sec. 3.2,
    2048 channels, 20 s span), with R = span / kernel time at each point.
    The kernel alone is timed (HIP events around `--steps` calls, at most 5,
    after one untimed call), its input resident on the device, each point
    with the tiling the autotuner keeps for it."""
    import torch

    from paper_2511_02328_amd import sps
    from sps_inputs import synth
    torch.cuda.set_device(0)
    reps = max(2, min(args.steps, 5))
    subband = args.method == "subband"
    rows = []
    for wl in points:
        if subband:
            plan = sps.sps_subband_plan_create(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, wl.ndm,
                                               wl.dm_lo, (wl.dm_hi - wl.dm_lo) / (wl.ndm - 1),
                                               args.n0, args.nsub)
            _, rtab, _, emax = sps.sps_subband_tables(plan)
            # the method's own integer adds: stage 1 (coarse trials x channels
            # x stage-1 row length) + stage 2 (trials x subbands x outputs)
            adds = (-(-wl.ndm // args.n0) * wl.nchan * ((wl.nout + int(rtab.max()) + 3) // 4 * 4)
                    + wl.ndm * args.nsub * wl.nout)
        else:
            plan, emax, adds = sps.plan_for(wl), 0, wl.sample_adds()
        nsamp = wl.nout + max(emax, sps.sps_plan_delays(plan)[1])
        sps.sps_plan_autotune(plan, 1 << 18, 2)
        X, _ = synth.make_filterbank(wl, nsamp, device="cuda", pitch=(nsamp + 255) // 256 * 256)
        Y = torch.empty((wl.ndm, wl.nout), dtype=torch.int32, device="cuda")
        if subband:
            def fn():
                sps.sps_dedisperse_subband(plan, X, nsamp, Y, wl.nout)
        else:
            def fn():
                sps.sps_dedisperse(plan, X, nsamp, Y, wl.nout)
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        b.synchronize()
        t = a.elapsed_time(b) / reps / 1e3
        span = wl.nout * wl.tsamp_s
        row = {"workload": wl.name, "nchan": wl.nchan, "ndm": wl.ndm, "nout": wl.nout,
               "nsamp_in": nsamp, "kernel_s": t, "R": span / t,
               "dm_time_samples_per_s": wl.dm_time_samples() / t,
               "integer_adds_per_s": adds / t}
        if not subband:
            row["tiling"] = sps.sps_plan_get_tiling(plan)
        rows.append(row)
        print(f"[bench] {wl.name}: {t * 1e3:.1f} ms, R = {span / t:.0f}", flush=True)
        del X, Y
        plan.close()
        torch.cuda.empty_cache()
    key = "nchan" if name == "sweep_channels" else "ndm"
    paper = PAPER_SWEEP_KERNEL_S[name]
    last = rows[-1]
    rec = {
        "metric": "DM×time samples/s dedispersed" + (" (subband method)" if subband else ""),
        "value": last["dm_time_samples_per_s"], "unit": "DM-time samples/s", "n_gpus": 1,
        "steps": reps, "warmup": 1, "ms_per_step": last["kernel_s"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": name, "method": args.method, "value_at": last["workload"]},
        "points": rows,
        # linear in the swept size: time per unit of it, first and last point
        "kernel_s_per_unit": {str(r[key]): r["kernel_s"] / r[key] for r in (rows[0], last)},
        "paper_kernel_s_rtx4090": {str(k): v for k, v in paper.items()},
        "kernel_time_ratio_paper_over_this": {
            str(k): v / r["kernel_s"] for k, v in paper.items() for r in rows if r[key] == k},
        "roofline": {"kernel": "sps_dedisperse_subband" if subband else "dedisperse_kernel",
                     "bound": "alu", "unit": "TOP/s", "peak": ALU_PEAK_TOPS,
                     "achieved": last["integer_adds_per_s"] / 1e12,
                     "frac": last["integer_adds_per_s"] / 1e12 / ALU_PEAK_TOPS, "traffic": None,
                     "work_per_launch": (f"{last['integer_adds_per_s'] * last['kernel_s']:.4g} "
                                         "integer adds (stage 1 + stage 2)") if subband else
                                        f"{last['ndm']} x {last['nout']} x {last['nchan']} sample-adds"},
    }
    print(json.dumps(rec), flush=True)


def host_cpu():
    """The host the CPU baseline ran on: CPU model (lscpu / /proc/cpuinfo),
    nproc (CPUs this process may use) and the logical CPU count."""
    model = None
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    if model is None:
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        model = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    return {"model": model, "nproc": len(os.sched_getaffinity(0)), "logical_cpus": os.cpu_count()}


def cpu_baseline(wl, X, nsamp, Y, nrows, det):
    """The oracle on a bounded sample: every (ndm / nrows)-th DM row of the same
    chunk at full length, through dedispersion, statistics, boxcar and
    detection.  Also confirms those rows of the GPU plane bit for bit."""
    import oracle
    rows = np.linspace(0, wl.ndm - 1, nrows).round().astype(np.int64)
    print(f"[bench] cpu baseline: copying the chunk to the host, {nrows} rows", flush=True)
    Xh = X[:, :nsamp].cpu().numpy()
    Yg = Y[rows].cpu().numpy().view(np.uint32)
    D = oracle.delays(wl.freqs_mhz(), wl.fref_mhz, wl.tsamp_s, wl.dms())[rows]
    t0 = time.perf_counter()
    Yo = oracle.dedisperse(Xh, D, wl.nout, nsamp)
    sto = oracle.stats(Yo)
    snro, besto = oracle.boxcar(Yo, sto, wl.widths)
    oracle.detect(snro, besto, det["threshold"], det["tile_dm"], det["tile_t"], det["nms_dm"],
                  det["nms_t"])
    sec = time.perf_counter() - t0
    ok = bool(np.array_equal(Yo, Yg))
    print(f"[bench] cpu baseline: {sec:.1f} s, sampled rows bit-exact: {ok}", flush=True)
    return {"value": nrows * wl.nout / sec, "unit": "DM-time samples/s",
            "cores": oracle.threads(), "kind": "oracle",
            "host": host_cpu(),
            "sample": f"{nrows} of {wl.ndm} DM rows (evenly spaced) of one chunk at full length "
                      f"({wl.nout} samples): dedisperse + stats + boxcar + detect; {sec:.1f} s",
            "sampled_rows_match_gpu": ok}


if __name__ == "__main__":
    main()
