"""The learned candidate detector around the HIP library: its training set
made by the search itself, the training loop and the comparison with the
plain boxcar search.

Tiles come from the single-beam set-up (256 channels, 98.304 us, 512 trial
DMs 0-1000, 4096 output samples): seeded synthetic filterbanks, half of them
with persistent narrow-band sinusoids, half (independently) with broadband
impulses, and for the positive half one dispersed pulse whose amplitude aims
at a boxcar S/N drawn from 5-50.  The library dedisperses them, forms the S/N planes,
runs the boxcar search (the yardstick) and pools the planes into bfloat16 tiles;
the labels are the injected pulses' positions.  Python only draws the
events, marshals buffers and keeps the books.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace
from typing import Optional

import numpy as np

from sps_inputs import synth
from sps_inputs.workloads import PulseModel, RfiModel, Workload

TILE_WORKLOAD = Workload(
    name="detector_tiles_256ch_4096t_512dm", nchan=256, f_lo_mhz=1000.0, f_hi_mhz=1500.0,
    tsamp_s=98.304e-6, nout=4096, ndm=512, dm_lo=0.0, dm_hi=1000.0,
    widths=(1, 2, 4, 8, 16, 32, 64), pulses=PulseModel(),
    rfi=RfiModel(chan_fraction=0.05, n_impulses=4), seed=0)

TILE_SCALE = 0.125                 # tile value = bf16(S/N / 8)
POOL = (2, 8)                      # trials x samples per tile pixel
CELL = (32, 32)                    # tile pixels per output cell
SEARCH = dict(threshold=8.0, tile_dm=32, tile_t=512, nms_dm=16, nms_t=128)


@dataclass
class TileSpec:
    snr_range: tuple = (5.0, 50.0)
    fwhm_range_s: tuple = (0.5e-3, 10e-3)     # log-uniform
    dm_range: tuple = (50.0, 950.0)
    sine_prob: float = 0.5
    impulse_prob: float = 0.5
    pos_frac: float = 0.5


# A detection matches an injected pulse when it lies within MATCH_DM trials
# and within MATCH_T + 3 FWHM samples of it (the same rule for both searches).
MATCH_DM = 16
MATCH_T = 64


def _boxcar_gain(sigma: float, widths) -> float:
    """max over widths and window starts of (sum of a unit Gaussian profile in
    the window) / sqrt(width): the matched-filter S/N per unit amplitude and
    unit noise of one channel-summed series."""
    h = int(math.ceil(6 * sigma)) + max(widths)
    t = np.arange(-h, h + 1, dtype=np.float64)
    best = 0.0
    for off in (0.0, 0.5):
        g = np.exp(-0.5 * ((t - off) / sigma) ** 2)
        c = np.concatenate([[0.0], np.cumsum(g)])
        for w in widths:
            best = max(best, float((c[w:] - c[:-w]).max()) / math.sqrt(w))
    return best


def draw_truth(rng: np.random.Generator, wl: Workload, nsamp_in: int, positive: bool,
               spec: TileSpec):
    """Events of one tile (numpy PCG64): with probability sine_prob sinusoids
    on 5% of channels, with probability impulse_prob broadband impulses, and
    for a positive tile one pulse.  Returns (Truth, pulse parameters or None)."""
    sig = wl.noise_sigma
    rm = wl.rfi
    sines = []
    n_rfi = int(round(rm.chan_fraction * wl.nchan)) if rng.random() < spec.sine_prob else 0
    for c in np.sort(rng.choice(wl.nchan, size=n_rfi, replace=False)):
        per = math.exp(rng.uniform(math.log(rm.sine_period_range_s[0]),
                                   math.log(rm.sine_period_range_s[1])))
        sines.append(synth.Sine(int(c), per, rng.uniform(0, 2 * math.pi), rm.sine_amp_sigma * sig))
    impulses = []
    if rng.random() < spec.impulse_prob:
        for _ in range(int(rng.integers(1, rm.n_impulses + 1))):
            ln = int(rng.integers(rm.impulse_len[0], rm.impulse_len[1] + 1))
            impulses.append(synth.Impulse(int(rng.integers(0, nsamp_in - ln)), ln,
                                          rm.impulse_amp_sigma * sig))
    pulses, info = [], None
    if positive:
        dm = rng.uniform(*spec.dm_range)
        fw = math.exp(rng.uniform(math.log(spec.fwhm_range_s[0]), math.log(spec.fwhm_range_s[1])))
        target = rng.uniform(*spec.snr_range)
        span = wl.nout * wl.tsamp_s
        toa = rng.uniform(3 * fw + 0.01, span - 3 * fw - 0.01)
        # width seen by the search: the pulse plus the smearing of a DM error
        # of a quarter trial step across the band
        ddm = (wl.dm_hi - wl.dm_lo) / (wl.ndm - 1)
        f = wl.freqs_mhz()
        smear = synth.SKY_K_DM * 0.25 * ddm * (1 / f.min() ** 2 - 1 / f.max() ** 2) / wl.tsamp_s
        s_t = math.sqrt((fw * synth.FWHM_TO_SIGMA / wl.tsamp_s) ** 2 + smear ** 2 / 12.0)
        amp = target * sig / (math.sqrt(wl.nchan) * _boxcar_gain(s_t, wl.widths))
        pulses.append(synth.Pulse(dm, fw, amp, toa))
        info = (dm, toa, fw, target)
    return synth.Truth(pulses, impulses, sines), info


class TileFactory:
    """Makes labelled tiles on the GPU with the library's own search: the
    filterbanks of a batch are dedispersed, searched (boxcar S/N + detection)
    and pooled in one pass."""

    def __init__(self, batch: int = 64, device: str = "cuda"):
        import torch

        from . import sps
        self.torch, self.sps = torch, sps
        self.wl = TILE_WORKLOAD
        self.batch = batch
        self.device = device
        self.plan = sps.plan_for(self.wl)
        _, self.dmax = sps.sps_plan_delays(self.plan)
        self.nsamp = self.wl.nout + self.dmax
        self.pitch = (self.nsamp + 255) // 256 * 256
        wl = self.wl
        self.X = torch.zeros((batch, wl.nchan, self.pitch), dtype=torch.uint8, device=device)
        self.Y = torch.empty((batch, wl.ndm, wl.nout), dtype=torch.int32, device=device)
        self.snr = torch.empty((batch, wl.ndm, wl.nout), dtype=torch.float32, device=device)
        self.best = torch.empty((batch, wl.ndm, wl.nout), dtype=torch.uint8, device=device)
        self.stats = torch.empty((batch, wl.ndm, 2), dtype=torch.int32, device=device)
        beams = [dict(X=self.X[i], nsamp_in=self.nsamp, nout=wl.nout, Y=self.Y[i],
                      snr=self.snr[i], best_w=self.best[i], stats=self.stats[i])
                 for i in range(batch)]
        self.handle = sps.sps_batch_create(self.plan, beams, list(wl.widths), **SEARCH)
        self.stream = torch.cuda.Stream()
        # the dedispersion tiling: the fastest on this batch's own launch
        # (4096 outputs fit some time tiles better than others)
        self.autotune_ms = sps.sps_batch_autotune(self.handle, 3, self.stream)

    def close(self):
        self.handle.close()
        self.plan.close()

    def make(self, n: int, seed: int, spec: Optional[TileSpec] = None):
        """n labelled tiles: (tiles int16 [n][256][512] on the device, labels
        float32 [n][3][8][16] on the device, meta dict of numpy arrays)."""
        torch, sps, wl = self.torch, self.sps, self.wl
        spec = spec or TileSpec()
        rng = np.random.Generator(np.random.PCG64(seed))
        tiles = torch.empty((n, wl.ndm // POOL[0], wl.nout // POOL[1]), dtype=torch.int16,
                            device=self.device)
        labels = np.zeros((n, 3, 8, 16), np.float32)
        meta = {k: np.full(n, np.nan) for k in ("dm", "toa_s", "fwhm_s", "target_snr",
                                                "pulse_snr", "row", "col", "d_star", "t_star")}
        meta["positive"] = np.zeros(n, bool)
        meta["sines"] = np.zeros(n, bool)
        meta["impulses"] = np.zeros(n, bool)
        meta["boxcar_any"] = np.zeros(n, bool)
        meta["boxcar_hit"] = np.zeros(n, bool)
        meta["plane_max_snr"] = np.zeros(n)
        # a pseudo pulse per pulse-free tile, drawn like the real ones from a
        # separate stream: how often a search "finds" a pulse by chance
        for k in ("pseudo_d", "pseudo_t", "pseudo_fws"):
            meta[k] = np.full(n, np.nan)
        meta["boxcar_chance"] = np.zeros(n, bool)
        prng = np.random.Generator(np.random.PCG64([seed, 7]))
        ddm = (wl.dm_hi - wl.dm_lo) / (wl.ndm - 1)
        for b0 in range(0, n, self.batch):
            nb = min(self.batch, n - b0)
            truths, infos = [], []
            for i in range(self.batch):
                pos = i < nb and rng.random() < spec.pos_frac
                tr, info = draw_truth(rng, wl, self.nsamp, pos, spec)
                truths.append(tr)
                infos.append(info)
            with torch.cuda.stream(self.stream):
                synth.render_filterbanks(wl, self.nsamp, truths, int(rng.integers(1 << 62)),
                                         self.device, self.pitch, out=self.X)
            sps.sps_batch_launch_graph(self.handle, self.stream)
            for i in range(nb):
                sps.sps_cnn_pool_tiles(self.snr[i], wl.nout, TILE_SCALE, tiles[b0 + i],
                                       stream=self.stream)
            with torch.cuda.stream(self.stream):
                pmax = self.snr[:nb].amax(dim=(1, 2)).cpu().numpy()
            for i in range(nb):
                j = b0 + i
                meta["plane_max_snr"][j] = pmax[i]
                meta["sines"][j] = len(truths[i].sines) > 0
                meta["impulses"][j] = len(truths[i].impulses) > 0
                cands, _ = sps.sps_batch_candidates(self.handle, i, cap=4096, stream=self.stream,
                                                    allow_truncated=True)
                meta["boxcar_any"][j] = len(cands) > 0
                info = infos[i]
                if info is None:
                    pdm = prng.uniform(*spec.dm_range)
                    pfw = math.exp(prng.uniform(math.log(spec.fwhm_range_s[0]),
                                                math.log(spec.fwhm_range_s[1])))
                    ptoa = prng.uniform(3 * pfw + 0.01, wl.nout * wl.tsamp_s - 3 * pfw - 0.01)
                    pd, pt, pf = (pdm - wl.dm_lo) / ddm, ptoa / wl.tsamp_s, pfw / wl.tsamp_s
                    meta["pseudo_d"][j], meta["pseudo_t"][j], meta["pseudo_fws"][j] = pd, pt, pf
                    meta["boxcar_chance"][j] = bool(
                        ((np.abs(cands["dm_idx"] - pd) <= MATCH_DM) &
                         (np.abs(cands["t_idx"] - pt) <= MATCH_T + 3 * pf)).any())
                    continue
                dm, toa, fw, target = info
                d_star = (dm - wl.dm_lo) / ddm
                t_star = toa / wl.tsamp_s
                row, col = d_star / POOL[0], t_star / POOL[1]
                meta["positive"][j] = True
                for k, v in (("dm", dm), ("toa_s", toa), ("fwhm_s", fw), ("target_snr", target),
                             ("row", row), ("col", col), ("d_star", d_star), ("t_star", t_star)):
                    meta[k][j] = v
                gy, gx = int(row // CELL[0]), int(col // CELL[1])
                labels[j, 0, gy, gx] = 1.0
                labels[j, 1, gy, gx] = row / CELL[0] - gy
                labels[j, 2, gy, gx] = col / CELL[1] - gx
                # S/N of the injected pulse: the plane's maximum near it
                fws = fw / wl.tsamp_s
                d0, d1 = max(0, int(d_star) - 8), min(wl.ndm, int(d_star) + 9)
                t0 = max(0, int(t_star - 3 * fws) - max(wl.widths))
                t1 = min(wl.nout, int(t_star + 3 * fws) + 8)
                with torch.cuda.stream(self.stream):
                    meta["pulse_snr"][j] = float(self.snr[i, d0:d1, t0:t1].max().cpu())
                tol_t = MATCH_T + 3 * fws
                near = (np.abs(cands["dm_idx"] - d_star) <= MATCH_DM) & \
                       (np.abs(cands["t_idx"] - t_star) <= tol_t)
                meta["boxcar_hit"][j] = bool(near.any())
        self.stream.synchronize()
        return tiles, torch.from_numpy(labels).to(self.device), meta


CNN_LAYERS = ((1, 16), (16, 32), (32, 64), (64, 128), (128, 128), (128, 128))


def init_params(seed: int) -> np.ndarray:
    """Initial parameters in the library's order (per 3x3 layer weights
    [cout][cin][3][3] then biases, then head weights [3][128] and biases):
    He-normal weights, zero biases, head weights N(0, 1/128), head biases
    (-4, 0.5, 0.5) so that training starts from a low objectness."""
    specs = []
    for i, (ci, co) in enumerate(CNN_LAYERS):
        specs += [(f"w{i}", (co, ci, 3, 3), math.sqrt(2.0 / (9 * ci))), (f"b{i}", (co,), 0.0)]
    specs += [("wh", (3, 128), math.sqrt(1.0 / 128)), ("bh", (3,), 0.0)]
    p = synth.seeded_weights(seed, specs)
    p["bh"] = np.array([-4.0, 0.5, 0.5], np.float32)
    return np.concatenate([p[name].ravel() for name, _, _ in specs])


def train(net, tiles, labels, epochs: int, batch: int, lr: float, stream=None,
          lr_min_frac: float = 0.05):
    """Adam over the tile set in order (the tiles are i.i.d. draws), cosine
    learning-rate decay; returns the per-step losses (numpy)."""
    import torch

    from . import sps
    n = int(tiles.shape[0])
    steps = n // batch
    total = steps * epochs
    losses = torch.zeros(max(total, 1), dtype=torch.float32, device=tiles.device)
    k = 0
    for _ in range(epochs):
        for s in range(steps):
            frac = k / max(total - 1, 1)
            lr_k = lr * (lr_min_frac + (1 - lr_min_frac) * 0.5 * (1 + math.cos(math.pi * frac)))
            sps.sps_cnn_train_step(net, tiles[s * batch:(s + 1) * batch],
                                   labels[s * batch:(s + 1) * batch], batch, lr_k,
                                   losses[k:k + 1], stream=stream)
            k += 1
    if stream is not None:
        stream.synchronize()
    return losses.cpu().numpy()


def cnn_scores(net, tiles, batch: int, stream=None):
    """Head outputs of every tile: float32 numpy [n][3][8][16]."""
    import torch

    from . import sps
    n = int(tiles.shape[0])
    out = torch.empty((n, 3, 8, 16), dtype=torch.float32, device=tiles.device)
    for b0 in range(0, n, batch):
        nb = min(batch, n - b0)
        sps.sps_cnn_forward(net, tiles[b0:b0 + nb], nb, out[b0:b0 + nb], stream=stream)
    if stream is not None:
        stream.synchronize()
    return out.cpu().numpy()


def compare_by_rfi(head: np.ndarray, meta: dict, threshold: float, snr_min: float = 8.0) -> dict:
    """compare_with_boxcar() on all tiles and separately on tiles without RFI, with
    sinusoids only and with impulses (any)."""
    groups = {"all": np.ones(len(meta["positive"]), bool),
              "clean": ~meta["sines"] & ~meta["impulses"],
              "sines_only": meta["sines"] & ~meta["impulses"],
              "impulses": meta["impulses"]}
    out = {}
    for g, m in groups.items():
        sub = {k: v[m] for k, v in meta.items()}
        out[g] = compare_with_boxcar(head[m], sub, threshold, snr_min)
    return out


def compare_with_boxcar(head: np.ndarray, meta: dict, threshold: float,
                        snr_min: float = 8.0) -> dict:
    """Recall on positive tiles whose injected pulse reaches snr_min in the
    boxcar plane, and false-alarm rate on pulse-free tiles, for the network
    and for the boxcar search.  A network detection is a cell at or above
    the probability threshold, placed where its offset heads put it; it
    matches the pulse under the same rule as a boxcar candidate (within
    MATCH_DM trials and MATCH_T + 3 FWHM samples).  A false alarm is any
    detection on a pulse-free tile; the chance-match rate is how often a
    pulse-free tile has a detection matching a pseudo pulse drawn like the
    real ones (the part of a recall that coincidence alone would give)."""
    logit = math.log(threshold / (1 - threshold))
    fire = head[:, 0] >= logit
    pos = meta["positive"]
    strong = pos & (meta["pulse_snr"] >= snr_min)
    gy = np.arange(head.shape[2])[:, None]
    gx = np.arange(head.shape[3])[None, :]
    hit = np.zeros(len(pos), bool)
    for j in np.flatnonzero(pos):
        d_pred = (gy + head[j, 1]) * CELL[0] * POOL[0]
        t_pred = (gx + head[j, 2]) * CELL[1] * POOL[1]
        fws = meta["fwhm_s"][j] / TILE_WORKLOAD.tsamp_s
        ok = fire[j] & (np.abs(d_pred - meta["d_star"][j]) <= MATCH_DM) & \
             (np.abs(t_pred - meta["t_star"][j]) <= MATCH_T + 3 * fws)
        hit[j] = bool(ok.any())
    neg = ~pos
    chance = np.zeros(len(pos), bool)
    for j in np.flatnonzero(neg):
        d_pred = (gy + head[j, 1]) * CELL[0] * POOL[0]
        t_pred = (gx + head[j, 2]) * CELL[1] * POOL[1]
        ok = fire[j] & (np.abs(d_pred - meta["pseudo_d"][j]) <= MATCH_DM) & \
             (np.abs(t_pred - meta["pseudo_t"][j]) <= MATCH_T + 3 * meta["pseudo_fws"][j])
        chance[j] = bool(ok.any())
    return {
        "threshold": threshold,
        "cnn_chance_match_rate": float(chance[neg].mean()) if neg.any() else None,
        "boxcar_chance_match_rate": float(meta["boxcar_chance"][neg].mean()) if neg.any() else None,
        "n_positive_snr_ge_min": int(strong.sum()), "n_negative": int(neg.sum()),
        "cnn_recall": float(hit[strong].mean()) if strong.any() else None,
        "boxcar_recall": float(meta["boxcar_hit"][strong].mean()) if strong.any() else None,
        "cnn_false_alarm_rate": float(fire[neg].any(axis=(1, 2)).mean()) if neg.any() else None,
        "boxcar_false_alarm_rate": float(meta["boxcar_any"][neg].mean()) if neg.any() else None,
        "cnn_recall_below_min": float(hit[pos & ~strong].mean()) if (pos & ~strong).any() else None,
        "boxcar_recall_below_min": (float(meta["boxcar_hit"][pos & ~strong].mean())
                                    if (pos & ~strong).any() else None),
    }
