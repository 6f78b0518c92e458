"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package holds random-field generators and workload descriptions only.  It
contains none of the multiscale method's arithmetic, so both the CPU oracle and
the HIP path may consume what it produces without sharing any solver code.
"""
from .fields import gaussian_logk, channel_logk, layered_logk
from .workloads import Workload, make_workload, WORKLOADS

__all__ = ["gaussian_logk", "channel_logk", "layered_logk", "Workload",
           "make_workload", "WORKLOADS"]
