"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

Nothing in this package computes any part of the search method (no traveltime
operator fit, no semblance, no evolution).  It only draws reproducible inputs:
Ricker-wavelet CMP-sorted gathers with exact constant-velocity kinematics, and
random candidate parameter vectors.
"""
from .gathers import (  # noqa: F401
    Gather,
    WORKLOADS,
    make_gather,
    make_workload,
    random_candidates,
    base_bounds,
)
