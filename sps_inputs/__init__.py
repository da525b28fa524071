"""Seeded inputs shared by the GPU path's tests and benchmark and by the
oracle-based checks: workload descriptions (band, sampling, trial-DM grid,
widths, sky model) and the synthetic filterbank and weight generators.

This package holds no step of the search.  It imports neither the HIP
library's binding (``paper_2511_02328_amd``) nor the oracle, so both sides
can draw their inputs from it without sharing any of the method's code.
"""
__all__ = ["synth", "workloads"]
