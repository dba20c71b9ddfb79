"""Workload definitions: grid, medium, damping layer, source, receivers, steps.

Each workload is plain data. `velocity()` draws the seeded medium;
`source_node()` and `receiver_nodes()` return flat indices into the pressure
field (x fastest). Nothing here computes any part of the method.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .models import homogeneous_velocity, layered_velocity


@dataclass(frozen=True)
class Workload:
    name: str
    n: tuple                  # (nx, nz) or (nx, ny, nz)
    h: float                  # grid spacing (m)
    abc_cells: int            # damping-layer thickness in cells
    sigma_max: float          # peak damping (1/s)
    f_peak: float             # Ricker peak frequency (Hz)
    t_delay: float            # Ricker delay (s)
    T: float                  # final time (s)
    src: tuple                # source node (i, [j,] k)
    medium: str = "layered"   # "homogeneous" or "layered"
    c_homog: float = 2000.0
    seed: int = 0
    faber_m: int = 16
    dt: float = 4e-3
    taylor_p: int = 8
    receivers: str = "none"   # "none", "surface_row", "nodes"
    rec_nodes: tuple = ()     # receiver nodes for receivers == "nodes"
    extra: dict = field(default_factory=dict)

    @property
    def ndim(self):
        return len(self.n)

    @property
    def npts(self):
        return int(np.prod(self.n))

    def velocity(self):
        if self.medium == "homogeneous":
            return homogeneous_velocity(self.n, self.c_homog)
        return layered_velocity(self.n, self.h, self.seed)

    def c2(self):
        """c^2 (float64 array) with values representable in FP32: the FP32
        and FP64 runs of a workload then see exactly the same medium."""
        return (self.velocity() ** 2).astype(np.float32).astype(np.float64)

    def flat_index(self, node):
        idx = 0
        stride = 1
        for a, v in enumerate(node):
            idx += int(v) * stride
            stride *= int(self.n[a])
        return idx

    def source_node(self):
        return self.flat_index(self.src)

    def receiver_nodes(self):
        if self.receivers == "none":
            return np.zeros(0, dtype=np.int64)
        if self.receivers == "surface_row":
            row = self.abc_cells + 2
            if self.ndim == 2:
                return np.array([self.flat_index((i, row)) for i in range(self.n[0])],
                                dtype=np.int64)
            j = self.n[1] // 2
            return np.array([self.flat_index((i, j, row)) for i in range(self.n[0])],
                            dtype=np.int64)
        if self.receivers == "nodes":
            return np.array([self.flat_index(v) for v in self.rec_nodes], dtype=np.int64)
        raise ValueError(self.receivers)


WORKLOADS = {
    # 101x101 homogeneous, FP64; the small case the oracle finishes in seconds
    "homog2d_101": Workload(
        name="homog2d_101", n=(101, 101), h=10.0, abc_cells=20, sigma_max=300.0,
        f_peak=15.0, t_delay=0.18, T=0.4, src=(50, 50), medium="homogeneous",
        c_homog=2000.0, faber_m=16, dt=4e-3, taylor_p=8),
    # 1001x501 layered, 40-cell layer, surface receiver line, T = 2 s
    "layered2d_1001x501": Workload(
        name="layered2d_1001x501", n=(1001, 501), h=10.0, abc_cells=40, sigma_max=300.0,
        f_peak=15.0, t_delay=0.18, T=2.0, src=(500, 42), medium="layered",
        seed=2000, faber_m=16, dt=2e-3, taylor_p=8, receivers="surface_row"),
    # 241x161 layered box without an absorbing layer (zero ghost values on
    # every side, so the wavefield keeps its energy): a grid small enough for
    # whole oracle runs of 1000 and more steps (long-run parity)
    "layered2d_241x161": Workload(
        name="layered2d_241x161", n=(241, 161), h=10.0, abc_cells=0, sigma_max=0.0,
        f_peak=15.0, t_delay=0.18, T=2.0, src=(120, 42), medium="layered",
        seed=2400, faber_m=16, dt=2e-3, taylor_p=8, receivers="surface_row"),
    # 8192x4096 layered: an added HBM-bound 2D shape (working set far above the
    # 256 MB Infinity Cache), same generator and layer as the 1001x501 medium
    "layered2d_8192x4096": Workload(
        name="layered2d_8192x4096", n=(8192, 4096), h=10.0, abc_cells=40, sigma_max=300.0,
        f_peak=15.0, t_delay=0.18, T=2.0, src=(4096, 42), medium="layered",
        seed=2100, faber_m=16, dt=2e-3, taylor_p=8, receivers="surface_row"),
    # single-signal experiment: homogeneous 6 km x 5 km at h = 10 m, c = 3 km/s,
    # no absorbing layer, source 10 m above the bottom edge, one receiver at
    # mid-depth, T = 1.3 s (the receiver is sampled uniformly over [0.6, 1.3] s)
    "homog2d_single_signal": Workload(
        name="homog2d_single_signal", n=(601, 501), h=10.0, abc_cells=0, sigma_max=0.0,
        f_peak=15.0, t_delay=0.18, T=1.3, src=(300, 499), medium="homogeneous",
        c_homog=3000.0, faber_m=16, dt=2e-3, taylor_p=8, receivers="nodes",
        rec_nodes=((300, 250),)),
    # inversion gradient: 601 x 301 layered (seed 5000) true model, start model =
    # the true model smoothed over 15 cells, 16 shots evenly spaced on row 42,
    # 601 receivers on row 42, T = 1.5 s, Faber degree 20, dt = 3 ms,
    # checkpoints every 10 steps
    "fwi2d_601x301": Workload(
        name="fwi2d_601x301", n=(601, 301), h=10.0, abc_cells=40, sigma_max=300.0,
        f_peak=15.0, t_delay=0.18, T=1.5, src=(300, 42), medium="layered",
        seed=5000, faber_m=20, dt=3e-3, taylor_p=8, receivers="surface_row",
        extra={"shots": 16, "checkpoint_every": 10, "smooth_cells": 15.0}),
    # 256^3 layered, 20-cell layer, centre source, T = 1 s, Faber degree 24
    "layered3d_256": Workload(
        name="layered3d_256", n=(256, 256, 256), h=10.0, abc_cells=20, sigma_max=300.0,
        f_peak=15.0, t_delay=0.18, T=1.0, src=(128, 128, 128), medium="layered",
        seed=3000, faber_m=24, dt=2.5e-3, taylor_p=8),
}


def get_workload(name):
    return WORKLOADS[name]
