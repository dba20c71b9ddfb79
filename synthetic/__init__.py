"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package holds no arithmetic of the method: it only draws velocity models,
initial wavefields, source/receiver positions and the workload definitions.
The damping profiles, the operator, the Faber/Krylov coefficients and the
source wavelet are computed separately by the oracle and by the native library.
"""
from .models import layered_velocity, smooth_state, homogeneous_velocity, smoothed
from .workloads import WORKLOADS, Workload, get_workload

__all__ = ["layered_velocity", "smooth_state", "homogeneous_velocity",
           "WORKLOADS", "Workload", "get_workload"]
