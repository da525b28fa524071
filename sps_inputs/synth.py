"""Seeded synthetic filterbanks (the only module both the GPU path and the
oracle-based checks draw inputs from).

It simulates the sky and the receiver, not the search: Gaussian noise of the
workload's mean and sigma, dispersed pulses placed on the continuous
cold-plasma sweep (the pulse arrives at the top of the band at its TOA and
at t + K DM (f^-2 - f_ref^-2) in channel f, unrounded, with no intra-channel
smearing and a flat spectrum), persistent narrow-band sinusoids and broadband
zero-DM impulses.  The float sum is rounded to nearest and clipped to 0..255.
None of the search's arithmetic (integer delay table, shift-and-sum,
statistics, boxcar, detection) appears here.

Random draws: ``SeedSequence(seed).spawn(2)`` gives one stream for the event
parameters (numpy PCG64, identical on every device) and one for the noise.
On the CPU the noise is numpy PCG64; on a GPU it is torch's seeded device
generator, so the two devices give different (each reproducible) noise
realisations of the same events.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

from .workloads import Workload

# Cold-plasma dispersion constant of the simulated sky, s MHz^2 pc^-1 cm^3.
SKY_K_DM = 4.148808e3
FWHM_TO_SIGMA = 1.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)))


@dataclass
class Pulse:
    dm: float
    fwhm_s: float
    amp: float        # counts added at the peak, per channel
    toa_s: float      # arrival time at the top of the band, from sample 0


@dataclass
class Impulse:
    start: int
    length: int
    amp: float


@dataclass
class Sine:
    chan: int
    period_s: float
    phase: float
    amp: float


@dataclass
class Truth:
    pulses: List[Pulse]
    impulses: List[Impulse]
    sines: List[Sine]


def draw_events(wl: Workload, nsamp_in: int, seed: Optional[int] = None) -> Truth:
    """Event parameters for one chunk (numpy PCG64, device independent)."""
    seed = wl.seed if seed is None else seed
    ev_seq, _ = np.random.SeedSequence(seed).spawn(2)
    rng = np.random.Generator(np.random.PCG64(ev_seq))
    sig = wl.noise_sigma
    span = wl.nout * wl.tsamp_s
    pulses = [Pulse(dm, fw, a * sig, toa) for dm, fw, a, toa in wl.pulses.fixed]
    pm = wl.pulses
    for _ in range(pm.count):
        dm = rng.uniform(*pm.dm_range)
        fw = math.exp(rng.uniform(math.log(pm.fwhm_range_s[0]), math.log(pm.fwhm_range_s[1])))
        amp = rng.uniform(*pm.amp_range_sigma) * sig
        lo = min(3 * fw, span / 2)
        toa = rng.uniform(lo, max(span - 3 * fw, lo))
        pulses.append(Pulse(dm, fw, amp, toa))
    rm = wl.rfi
    sines = []
    n_rfi = int(round(rm.chan_fraction * wl.nchan))
    if n_rfi:
        chans = np.sort(rng.choice(wl.nchan, size=n_rfi, replace=False))
        for c in chans:
            per = math.exp(rng.uniform(math.log(rm.sine_period_range_s[0]),
                                       math.log(rm.sine_period_range_s[1])))
            sines.append(Sine(int(c), per, rng.uniform(0, 2 * math.pi), rm.sine_amp_sigma * sig))
    impulses = []
    for _ in range(rm.n_impulses):
        ln = int(rng.integers(rm.impulse_len[0], rm.impulse_len[1] + 1))
        impulses.append(Impulse(int(rng.integers(0, max(1, nsamp_in - ln))), ln,
                                rm.impulse_amp_sigma * sig))
    return Truth(pulses, impulses, sines)


def _pulse_windows(wl: Workload, p: Pulse, c0: int, c1: int, nsamp_in: int):
    """Per-channel sample windows and Gaussian values for pulse p (numpy)."""
    f = wl.freqs_mhz()[c0:c1]
    fref = wl.fref_mhz
    centre = (p.toa_s + SKY_K_DM * p.dm * (1.0 / (f * f) - 1.0 / (fref * fref))) / wl.tsamp_s
    s = p.fwhm_s * FWHM_TO_SIGMA / wl.tsamp_s
    h = int(math.ceil(6.0 * s)) + 1
    idx = np.floor(centre).astype(np.int64)[:, None] + np.arange(-h, h + 1)[None, :]
    val = p.amp * np.exp(-0.5 * ((idx - centre[:, None]) / s) ** 2)
    ok = (idx >= 0) & (idx < nsamp_in)
    return idx, val, ok


def make_filterbank(wl: Workload, nsamp_in: int, seed: Optional[int] = None,
                    device: str = "cpu", pitch: Optional[int] = None,
                    chan_block: int = 256):
    """Channel-major uint8 filterbank [nchan][pitch] (first nsamp_in valid, rest 0).

    ``device='cpu'`` returns a numpy array, anything else a torch tensor on
    that device.  Returns (X, truth).
    """
    seed = wl.seed if seed is None else seed
    pitch = nsamp_in if pitch is None else pitch
    if pitch < nsamp_in:
        raise ValueError("pitch < nsamp_in")
    truth = draw_events(wl, nsamp_in, seed)
    _, noise_seq = np.random.SeedSequence(seed).spawn(2)
    on_cpu = device == "cpu"
    if on_cpu:
        rng = np.random.Generator(np.random.PCG64(noise_seq))
        X = np.zeros((wl.nchan, pitch), dtype=np.uint8)
    else:
        import torch
        gen = torch.Generator(device=device)
        gen.manual_seed(int(noise_seq.generate_state(1, np.uint64)[0] & 0x7FFFFFFFFFFFFFFF))
        X = torch.zeros((wl.nchan, pitch), dtype=torch.uint8, device=device)
    t_s = None
    for c0 in range(0, wl.nchan, chan_block):
        c1 = min(wl.nchan, c0 + chan_block)
        nb = c1 - c0
        if on_cpu:
            blk = rng.normal(wl.noise_mean, wl.noise_sigma, size=(nb, nsamp_in))
        else:
            blk = torch.randn((nb, nsamp_in), generator=gen, device=device, dtype=torch.float32)
            blk.mul_(wl.noise_sigma).add_(wl.noise_mean)
        for p in truth.pulses:
            idx, val, ok = _pulse_windows(wl, p, c0, c1, nsamp_in)
            rows = np.broadcast_to(np.arange(nb)[:, None], idx.shape)
            if on_cpu:
                np.add.at(blk, (rows[ok], idx[ok]), val[ok])
            else:
                flat = torch.from_numpy((rows[ok] * nsamp_in + idx[ok]).astype(np.int64)).to(device)
                blk.view(-1).index_add_(0, flat, torch.from_numpy(val[ok].astype(np.float32)).to(device))
        for s in truth.sines:
            if c0 <= s.chan < c1:
                if t_s is None:
                    t_s = (np.arange(nsamp_in, dtype=np.float64) * wl.tsamp_s) if on_cpu else \
                        torch.arange(nsamp_in, device=device, dtype=torch.float64) * wl.tsamp_s
                arg = 2 * math.pi * t_s / s.period_s + s.phase
                if on_cpu:
                    blk[s.chan - c0] += s.amp * np.sin(arg)
                else:
                    blk[s.chan - c0] += (s.amp * torch.sin(arg)).to(torch.float32)
        for im in truth.impulses:
            blk[:, im.start:im.start + im.length] += im.amp
        if on_cpu:
            X[c0:c1, :nsamp_in] = np.clip(np.rint(blk), 0, 255).astype(np.uint8)
        else:
            X[c0:c1, :nsamp_in] = blk.round_().clamp_(0, 255).to(torch.uint8)
        del blk
    return X, truth


def render_filterbanks(wl: Workload, nsamp_in: int, truths, seed: int, device: str = "cuda",
                       pitch: Optional[int] = None, out=None):
    """Many filterbanks at once: truths[b] (events of filterbank b) rendered over
    fresh Gaussian noise into uint8 [B][nchan][pitch] (torch, on `device`).
    Same sky model as make_filterbank; the noise comes from one torch
    generator seeded with `seed` for the whole batch."""
    import torch
    pitch = nsamp_in if pitch is None else pitch
    B, nc = len(truths), wl.nchan
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed) & 0x7FFFFFFFFFFFFFFF)
    blk = torch.randn((B * nc, nsamp_in), generator=gen, device=device, dtype=torch.float32)
    blk.mul_(wl.noise_sigma).add_(wl.noise_mean)
    flat_idx, flat_val = [], []
    rows = np.arange(nc)[:, None]
    for b, tr in enumerate(truths):
        for p in tr.pulses:
            idx, val, ok = _pulse_windows(wl, p, 0, nc, nsamp_in)
            r = np.broadcast_to(rows, idx.shape)
            flat_idx.append(((b * nc + r[ok]) * nsamp_in + idx[ok]).astype(np.int64))
            flat_val.append(val[ok].astype(np.float32))
    if flat_idx:
        blk.view(-1).index_add_(0, torch.from_numpy(np.concatenate(flat_idx)).to(device),
                                torch.from_numpy(np.concatenate(flat_val)).to(device))
    srow, sper, sph, samp = [], [], [], []
    for b, tr in enumerate(truths):
        for sn in tr.sines:
            srow.append(b * nc + sn.chan)
            sper.append(sn.period_s)
            sph.append(sn.phase)
            samp.append(sn.amp)
    if srow:
        t_s = torch.arange(nsamp_in, device=device, dtype=torch.float64) * wl.tsamp_s
        per = torch.tensor(sper, device=device, dtype=torch.float64)[:, None]
        ph = torch.tensor(sph, device=device, dtype=torch.float64)[:, None]
        amp = torch.tensor(samp, device=device, dtype=torch.float64)[:, None]
        wave = (amp * torch.sin(2 * math.pi * t_s[None, :] / per + ph)).to(torch.float32)
        blk.index_add_(0, torch.tensor(srow, device=device, dtype=torch.int64), wave)
        del wave
    for b, tr in enumerate(truths):
        for im in tr.impulses:
            blk[b * nc:(b + 1) * nc, im.start:im.start + im.length] += im.amp
    if out is None:
        out = torch.zeros((B, nc, pitch), dtype=torch.uint8, device=device)
    out[:, :, :nsamp_in] = blk.round_().clamp_(0, 255).to(torch.uint8).view(B, nc, nsamp_in)
    del blk
    return out


def seeded_weights(seed: int, specs) -> dict:
    """Initial weights, an input of training: specs is a list of
    (name, shape, std); each entry is drawn N(0, std^2) in order from one
    numpy PCG64 stream (std 0 gives zeros).  float32 arrays."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = {}
    for name, shape, std in specs:
        out[name] = (rng.normal(0.0, std, shape) if std > 0 else np.zeros(shape)).astype(np.float32)
    return out


def random_bytes(nchan: int, nsamp_in: int, seed: int, pitch: Optional[int] = None,
                 lo: int = 0, hi: int = 256) -> np.ndarray:
    """Uniform random bytes [nchan][pitch] (first nsamp_in valid, rest 0)."""
    pitch = nsamp_in if pitch is None else pitch
    rng = np.random.Generator(np.random.PCG64(seed))
    X = np.zeros((nchan, pitch), dtype=np.uint8)
    X[:, :nsamp_in] = rng.integers(lo, hi, size=(nchan, nsamp_in), dtype=np.uint8)
    return X
