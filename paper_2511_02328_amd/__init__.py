"""MI355X-native single-pulse search hot path: brute-force incoherent
dedispersion of a channelised 8-bit filterbank over a trial-DM grid, then a
boxcar matched-filter S/N search over the DM-time plane and candidate
detection (ASTROFLOW, arXiv:2511.02328, Sec. 1 and Sec. 2.3).

The computation lives in a HIP shared library behind a C ABI
(``include/sps.h``); :mod:`paper_2511_02328_amd.sps` is its ctypes binding.
The workload descriptions and the seeded input generators live in the
separate package ``sps_inputs``, which holds no step of the search.
"""
__all__ = ["sps", "detector"]
