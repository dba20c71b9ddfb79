"""Seeded velocity models and initial wavefields.

Arrays use the numpy shape (nz, nx) in 2D and (nz, ny, nx) in 3D, x fastest,
matching the canonical field layout of the library: node (i, k) of a 2D grid
is element [k, i]. Grid extents are given as n = (nx, nz) or (nx, ny, nz).

The paper's velocity models (Corner, Santos Basin, Marmousi, SEG/EAGE) are not
available here, so seeded smooth layered media of the same velocity range and
comparable shapes stand in for them.
"""
from __future__ import annotations

import numpy as np
from scipy.ndimage import gaussian_filter


def _numpy_shape(n):
    return tuple(int(v) for v in reversed(tuple(n)))


def homogeneous_velocity(n, c=2000.0):
    """Constant velocity c (m/s) on a grid of extents n."""
    return np.full(_numpy_shape(n), float(c))


def layered_velocity(n, h, seed, vmin=1500.0, vmax=4500.0, n_interfaces=8,
                     n_anomalies=3, smooth_cells=2.0):
    """Smooth layered velocity model (m/s), deterministic in `seed`.

    Recipe: `n_interfaces` undulating interfaces at sorted uniform depths in
    (0.05, 0.95) of the depth extent, each perturbed by A sin(2 pi x / lam + phi)
    (A <= 0.03 of the depth, lam in [0.3, 1] of the lateral extent; in 3D a
    second undulation along y); layer speeds sorted uniform in [vmin, vmax] with
    the top layer at vmin and the bottom layer at vmax; `n_anomalies` Gaussian
    anomalies of +-5..15 % with radii 5..15 % of the smallest extent; clipped to
    [vmin, vmax] and Gaussian-smoothed with a width of `smooth_cells` cells.
    """
    rng = np.random.default_rng(seed)
    n = tuple(int(v) for v in n)
    ndim = len(n)
    ext = [max(v - 1, 1) * h for v in n]     # physical extents per axis (x, [y,] z)
    lz = ext[-1]
    axes = [np.arange(v) * h for v in n]
    grids = np.meshgrid(*[axes[a] for a in reversed(range(ndim))], indexing="ij")
    # grids[0] is the slowest numpy axis = z; the last is x
    zc = grids[0]
    xc = grids[-1]
    yc = grids[1] if ndim == 3 else None

    depths = np.sort(rng.uniform(0.05, 0.95, n_interfaces)) * lz
    amp = rng.uniform(0.0, 0.03, n_interfaces) * lz
    lam_x = rng.uniform(0.3, 1.0, n_interfaces) * ext[0]
    phi_x = rng.uniform(0.0, 2.0 * np.pi, n_interfaces)
    if ndim == 3:
        lam_y = rng.uniform(0.3, 1.0, n_interfaces) * ext[1]
        phi_y = rng.uniform(0.0, 2.0 * np.pi, n_interfaces)
    speeds = np.sort(rng.uniform(vmin, vmax, n_interfaces + 1))
    speeds[0] = vmin
    speeds[-1] = vmax

    layer = np.zeros(zc.shape, dtype=np.int64)
    for q in range(n_interfaces):
        surf = depths[q] + amp[q] * np.sin(2.0 * np.pi * xc / lam_x[q] + phi_x[q])
        if ndim == 3:
            surf = surf + 0.5 * amp[q] * np.sin(2.0 * np.pi * yc / lam_y[q] + phi_y[q])
        layer += (zc > surf)
    c = speeds[layer]

    lmin = min(ext)
    for _ in range(n_anomalies):
        centre = [rng.uniform(0.0, e) for e in ext]
        radius = rng.uniform(0.05, 0.15) * lmin
        rel = rng.uniform(0.05, 0.15) * rng.choice([-1.0, 1.0])
        r2 = (xc - centre[0]) ** 2 + (zc - centre[-1]) ** 2
        if ndim == 3:
            r2 = r2 + (yc - centre[1]) ** 2
        c = c * (1.0 + rel * np.exp(-r2 / radius ** 2))

    c = np.clip(c, vmin, vmax)
    if smooth_cells > 0:
        c = gaussian_filter(c, smooth_cells, mode="nearest")
    return np.clip(c, vmin, vmax)


def smooth_state(n, seed, n_pulses=6, width_cells=6.0, v_scale=1e-3):
    """Seeded smooth wavefield [p | v_1 | ... | v_d] as one flat float64 vector.

    Each field is a sum of `n_pulses` Gaussian pulses with random centres,
    signs and amplitudes in [0.5, 1]; velocity fields are scaled by `v_scale`
    so that the state resembles an acoustic wavefield (|v| ~ |p| / (rho c)).
    Used as a non-trivial initial state for parity runs.
    """
    rng = np.random.default_rng(seed)
    n = tuple(int(v) for v in n)
    ndim = len(n)
    shape = _numpy_shape(n)
    idx = np.meshgrid(*[np.arange(v, dtype=np.float64) for v in shape], indexing="ij")
    fields = []
    for f in range(ndim + 1):
        acc = np.zeros(shape)
        for _ in range(n_pulses):
            centre = [rng.uniform(0.15, 0.85) * (s - 1) for s in shape]
            a = rng.uniform(0.5, 1.0) * rng.choice([-1.0, 1.0])
            w = rng.uniform(0.6, 1.4) * width_cells
            r2 = sum((idx[d] - centre[d]) ** 2 for d in range(len(shape)))
            acc += a * np.exp(-r2 / (2.0 * w * w))
        fields.append(acc * (1.0 if f == 0 else v_scale))
    return np.concatenate([fl.ravel() for fl in fields])


def smoothed(c, cells):
    """Gaussian-smoothed copy of a velocity model (a starting model for
    inversion), width `cells` grid cells."""
    return gaussian_filter(np.asarray(c, dtype=np.float64), cells, mode="nearest")
