"""Seeded synthetic input generators shared by the CPU oracle and the GPU path.

This package holds input generation only; none of the search method's
arithmetic lives here.
"""
from . import patch_mixture
from .configs import (WORKLOADS, SMALL_10K, SCALE_1M, PRECISION_1M, ZIPF_10M, SIFTLIKE_1M, SIFTLIKE_20K,
                      Workload)

__all__ = ["patch_mixture", "WORKLOADS", "SMALL_10K", "SCALE_1M", "PRECISION_1M", "ZIPF_10M", "SIFTLIKE_1M",
           "SIFTLIKE_20K", "Workload"]
