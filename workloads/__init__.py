"""Seeded synthetic inputs for the sliding-window correlation.

This module only draws random numbers and shapes test images; it holds none of
the correlation arithmetic.  Both the CPU oracle's tests and the GPU path's
tests and benchmark take their inputs from here.
"""
from .gen import (  # noqa: F401
    CONFIGS,
    batched_pairs,
    cloud_pair,
    paper_shaped_u16,
    precision_pair,
    series_1d,
    volume_3d,
    random_pair,
)
