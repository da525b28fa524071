"""Workload descriptions: observing set-ups shaped like the paper's searches.

A workload names the band, the sampling, the chunk length, the trial-DM grid
and the boxcar widths, plus the sky model the synthetic generator draws from.
Nothing here computes any step of the search: the two helpers give the
channel centre frequencies and the trial-DM values, which are inputs to the
search, not part of it.

* ``single_beam``: 256 channels over 1000-1500 MHz, 98.304 us, a 4096-sample
  dedispersed span, 512 trial DMs 0-1000, widths 1..64, one injected pulse at
  DM 300 (FWHM 1 ms, +6 sigma per channel).  Small enough for the CPU oracle
  to run in full in seconds.
* ``full_scale``: 4096 channels over 1000-1500 MHz, 49.152 us, 2^20-sample
  chunks plus the dispersion overlap, 2048 trial DMs 0..2047 in steps of 1,
  widths 1..256; 20 injected pulses and RFI per chunk.  The throughput
  workload: one chunk is 2048 x 2^20 DM-time samples.
* ``batched_19beams_256ch_512dm``: 19 beams of the single-beam receiver with
  uneven chunk lengths (2^18, 2^19 or 2^20 samples), searched together.
* ``streaming_24_mixed``: 24 real-time streams of three set-ups (1024, 4096
  and 8192 channels) served together.

Channel order follows the common 8-bit filterbank convention: channel 0 is
the top of the band, and the reference frequency of the delays is the upper
band edge (arrival times are quoted at the top of the band, Sec. 2).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Tuple

import numpy as np


@dataclass(frozen=True)
class PulseModel:
    """Sky model of injected dispersed pulses (flat spectrum, Gaussian profile)."""
    count: int = 0
    fixed: Tuple[Tuple[float, float, float, float], ...] = ()  # (dm, fwhm_s, amp_sigma, toa_s)
    dm_range: Tuple[float, float] = (50.0, 2000.0)
    fwhm_range_s: Tuple[float, float] = (0.1e-3, 20e-3)       # log-uniform
    amp_range_sigma: Tuple[float, float] = (0.5, 5.0)         # per-channel peak


@dataclass(frozen=True)
class RfiModel:
    """Persistent narrow-band sinusoids and broadband zero-DM impulses."""
    chan_fraction: float = 0.0
    sine_amp_sigma: float = 8.0
    sine_period_range_s: Tuple[float, float] = (1e-3, 100e-3)  # log-uniform
    n_impulses: int = 0
    impulse_len: Tuple[int, int] = (1, 4)
    impulse_amp_sigma: float = 10.0


@dataclass(frozen=True)
class Workload:
    name: str
    nchan: int
    f_lo_mhz: float
    f_hi_mhz: float
    tsamp_s: float
    nout: int
    ndm: int
    dm_lo: float
    dm_hi: float
    widths: Tuple[int, ...]
    noise_mean: float = 128.0
    noise_sigma: float = 16.0
    pulses: PulseModel = field(default_factory=PulseModel)
    rfi: RfiModel = field(default_factory=RfiModel)
    seed: int = 1

    @property
    def fref_mhz(self) -> float:
        return self.f_hi_mhz

    def freqs_mhz(self) -> np.ndarray:
        """Channel centres, channel 0 at the top: f_hi - (c + 1/2) * B / nchan."""
        bw = (self.f_hi_mhz - self.f_lo_mhz) / self.nchan
        return self.f_hi_mhz - (np.arange(self.nchan, dtype=np.float64) + 0.5) * bw

    def dms(self) -> np.ndarray:
        """Trial DMs, evenly spaced with both ends included."""
        if self.ndm == 1:
            return np.array([self.dm_lo], dtype=np.float64)
        step = (self.dm_hi - self.dm_lo) / (self.ndm - 1)
        return self.dm_lo + np.arange(self.ndm, dtype=np.float64) * step

    def dm_time_samples(self) -> int:
        return self.ndm * self.nout

    def sample_adds(self) -> int:
        return self.ndm * self.nout * self.nchan


SINGLE_BEAM = Workload(
    name="single_beam_256ch_4096t_512dm",
    nchan=256, f_lo_mhz=1000.0, f_hi_mhz=1500.0, tsamp_s=98.304e-6,
    nout=4096, ndm=512, dm_lo=0.0, dm_hi=1000.0,
    widths=(1, 2, 4, 8, 16, 32, 64),
    pulses=PulseModel(fixed=((300.0, 1e-3, 6.0, 2000 * 98.304e-6),)),
    seed=1,
)

FULL_SCALE = Workload(
    name="full_scale_4096ch_2p20t_2048dm",
    nchan=4096, f_lo_mhz=1000.0, f_hi_mhz=1500.0, tsamp_s=49.152e-6,
    nout=1 << 20, ndm=2048, dm_lo=0.0, dm_hi=2047.0,
    widths=(1, 2, 4, 8, 16, 32, 64, 128, 256),
    pulses=PulseModel(count=20),
    rfi=RfiModel(chan_fraction=0.05, n_impulses=10),
    seed=2,
)

@dataclass(frozen=True)
class BatchWorkload:
    """Many beams of one receiver searched together: each beam has the base
    workload's band, sampling and DM grid, its own chunk length (drawn from
    `lengths`, seeded) and its own noise, pulses and RFI."""
    name: str
    base: Workload
    nbeams: int
    lengths: Tuple[int, ...]
    seed: int

    def beam_lengths(self) -> list:
        rng = np.random.Generator(np.random.PCG64(self.seed))
        return [int(x) for x in rng.choice(self.lengths, size=self.nbeams)]

    def beam_seeds(self) -> list:
        return [int(s.generate_state(1)[0] & 0x7FFFFFFF)
                for s in np.random.SeedSequence(self.seed).spawn(self.nbeams)]

    def beam_workload(self, i: int, nout: int) -> Workload:
        from dataclasses import replace
        return replace(self.base, name=f"{self.name}_beam{i}", nout=nout, seed=self.beam_seeds()[i])


# 19 beams shaped like the single-beam set-up (256 channels, 98.304 us,
# 512 DMs 0-1000, widths 1..64), chunks of 2^18, 2^19 or 2^20 samples, each
# with its own pulses (DM 50-1000) and RFI.
BATCHED = BatchWorkload(
    name="batched_19beams_256ch_512dm",
    base=Workload(name="batched_beam", nchan=256, f_lo_mhz=1000.0, f_hi_mhz=1500.0,
                  tsamp_s=98.304e-6, nout=1 << 18, ndm=512, dm_lo=0.0, dm_hi=1000.0,
                  widths=(1, 2, 4, 8, 16, 32, 64),
                  pulses=PulseModel(count=4, dm_range=(50.0, 1000.0)),
                  rfi=RfiModel(chan_fraction=0.05, n_impulses=4)),
    nbeams=19, lengths=(1 << 18, 1 << 19, 1 << 20), seed=3)

@dataclass(frozen=True)
class StreamingWorkload:
    """Concurrent real-time streams of mixed observing set-ups: `groups` holds
    (count, workload) pairs, the workload's nout being the chunk length."""
    name: str
    groups: Tuple[Tuple[int, Workload], ...]

    def streams(self) -> list:
        return [wl for n, wl in self.groups for _ in range(n)]


_STREAM_A = Workload(
    name="stream_1024ch_64us_2p18t_1024dm", nchan=1024, f_lo_mhz=1000.0, f_hi_mhz=1500.0,
    tsamp_s=64e-6, nout=1 << 18, ndm=1024, dm_lo=0.0, dm_hi=1000.0,
    widths=(1, 2, 4, 8, 16, 32, 64, 128, 256), pulses=PulseModel(count=4),
    rfi=RfiModel(chan_fraction=0.05, n_impulses=4), seed=11)
_STREAM_C = Workload(
    name="stream_8192ch_196us_2p18t_4096dm", nchan=8192, f_lo_mhz=1000.0, f_hi_mhz=1500.0,
    tsamp_s=196.608e-6, nout=1 << 18, ndm=4096, dm_lo=0.0, dm_hi=4095.0,
    widths=(1, 2, 4, 8, 16, 32, 64, 128, 256), pulses=PulseModel(count=4),
    rfi=RfiModel(chan_fraction=0.05, n_impulses=4), seed=13)

# 24 streams: 8 x (1024 channels, 64 us, 2^18-sample chunks, 1024 DMs 0-1000),
# 12 x the full-scale set-up (4096 channels, 49.152 us, 2^20, 2048 DMs) and
# 4 x (8192 channels, 196.608 us, 2^18, 4096 DMs 0-4095).
STREAMING = StreamingWorkload(
    name="streaming_24_mixed",
    groups=((8, _STREAM_A), (12, FULL_SCALE), (4, _STREAM_C)))


def _sweep_point(name: str, nchan: int, ndm: int, span_s: float) -> Workload:
    return Workload(
        name=name, nchan=nchan, f_lo_mhz=1000.0, f_hi_mhz=1500.0, tsamp_s=40e-6,
        nout=int(round(span_s / 40e-6)), ndm=ndm, dm_lo=0.0, dm_hi=1024.0, widths=(1,),
        pulses=PulseModel(count=4, dm_range=(50.0, 1000.0)), seed=21)


# The paper's two dedispersion timing sweeps (Sec. 3.1 and 3.2): 8-bit data
# at 40 us over 1000-1500 MHz (centre 1250 MHz), DMs 0-1024.  Channel sweep:
# 1500 trials over a 22 s dedispersed span, 512..8192 channels.  DM sweep:
# 2048 channels over a 20 s span, 512..8192 trials.
SWEEPS = {
    "sweep_channels": tuple(_sweep_point(f"sweep_{c}ch_1500dm_22s", c, 1500, 22.0)
                            for c in (512, 1024, 2048, 4096, 8192)),
    "sweep_dms": tuple(_sweep_point(f"sweep_2048ch_{d}dm_20s", 2048, d, 20.0)
                       for d in (512, 1024, 2048, 4096, 8192)),
}

WORKLOADS = {w.name: w for w in (SINGLE_BEAM, FULL_SCALE)}
BATCH_WORKLOADS = {BATCHED.name: BATCHED}
STREAMING_WORKLOADS = {STREAMING.name: STREAMING}
