"""Oracle: the paper's own spatial operator, the 2D acoustic PML system.

Test infrastructure only (see the package docstring).

Paper anchors:
- Sec. 2 (wave equation with PML): the 4-field first-order-in-time system for
  (u, v, w_x, w_y), with displacement u, its rate v = u_t and the PML
  auxiliaries w_x, w_y:
      u_t   = v
      v_t   = (-beta_x beta_y + c^2 (d_xx + d_yy)) u - (beta_x + beta_y) v
              + c^2 d_x w_x + c^2 d_y w_y + f
      w_x,t = (beta_y - beta_x) d_x u - beta_x w_x
      w_y,t = (beta_x - beta_y) d_y u - beta_y w_y
  with the quadratic profiles beta_z = beta_0 (1 - d/delta)^2 inside the layer;
  zero values on the two sides and the bottom, and no layer at the top
  (beta_y = 0 there), which is a free surface.
- Sec. 2.1 (spatial discretization): the 8th-order staggered first derivative
  1225/1024 (1, -1/15, 1/125, -1/1715) and the 8th-order centred second
  derivative; values outside the domain are zero.
- Sec. 2.2 (free surface) and the appendix on it: one-sided 8th-order
  stencils for d_yy u at the four rows nearest the surface and for d_y u at
  the three half rows nearest it, both built on u_y(0) = 0; d_y w_y near the
  surface by Fornberg's algorithm on points where w_y is known, using
  w_y(0) = 0.

Readings (the paper leaves these open or prints them garbled):
- Second derivative: the printed differences are read as sums and the
  missing 1/dx^2 is restored, i.e.
      d_xx u_i = (-205/72 u_i + sum_l b_l (u_{i+l} + u_{i-l})) / h^2,
      b = (8/5, -1/5, 8/315, -1/560)
  (exact to degree 9, pinned by a test; the printed form is not consistent).
- Grid: u, v and c at nodes (i, j), i = 0..nx-1 along x, j = 0..ny-1 downwards
  from the surface row j = 0 (y = -j h); w_x at (i + 1/2, j) and w_y at
  (i, j + 1/2), i.e. y = -(j + 1/2) h, as in the paper's staggered figure and
  its appendix notation w_i = w_y(x, -(i + 1/2) dx). Each field is an
  (ny, nx) array; the state is [u | v | w_x | w_y] flattened.
- Derivatives in y are taken with respect to the paper's upward y, so the
  staggered d_y u at half row j is (1/h) sum_l alpha_l (u_{j+1-l} - u_{j+l})
  and d_y w_y at row j is (1/h) sum_l alpha_l (w_{j-l} - w_{j+l-1}).
  The interior formulas are used wherever they need no point above the surface:
  d_yy u for j >= 4, d_y u for half rows j >= 3, d_y w_y for j >= 4.
- Fornberg's node set for d_y w_y at rows j = 0..3: the surface point (where
  w_y = 0) and the eight half rows w_0..w_7, nine nodes in all, so the
  formula is of order 8 like the interior one. The surface weight multiplies
  zero and drops out.
- Damping: beta_x from the distance to the nearer side (0 or (nx-1) h),
  beta_y from the distance to the bottom row only (no layer at the top),
  each evaluated where the field lives (half points for the staggered
  directions), with the profile of the p/v operator.
- Source: f enters the v equation at a node (strength amps / h^2 times the
  Ricker wavelet), and receivers record u.
"""
from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction as Fr

import numpy as np

from .operator import damping_profile, staggered_weights

# Sec. 2.1, 8th-order centred second derivative (read with sums and 1/h^2)
D2_CENTER = -205.0 / 72.0
D2_WEIGHTS = np.array([8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0])

# Appendix on the free surface: d_yy u at y = 0, -h, -2h, -3h from u_0..u_8
# (times 1/h^2), and d_y u at y = -h/2, -3h/2, -5h/2 from u_0..u_7 (times 1/h),
# with u_i = u(x, -i h) and y pointing up.
SURFACE_D2 = [
    [Fr(-3144919, 352800), Fr(16), Fr(-14), Fr(112, 9), Fr(-35, 4), Fr(112, 25), Fr(-14, 9),
     Fr(16, 49), Fr(-1, 32)],
    [Fr(271343, 156800), Fr(-1991, 630), Fr(57, 40), Fr(13, 60), Fr(-109, 288), Fr(6, 25),
     Fr(-11, 120), Fr(179, 8820), Fr(-9, 4480)],
    [Fr(-18519, 78400), Fr(58, 35), Fr(-251, 90), Fr(22, 15), Fr(-1, 16), Fr(-14, 225), Fr(1, 30),
     Fr(-2, 245), Fr(17, 20160)],
    [Fr(74801, 1411200), Fr(-37, 140), Fr(67, 40), Fr(-263, 90), Fr(53, 32), Fr(-23, 100),
     Fr(13, 360), Fr(-1, 245), Fr(1, 4480)],
]
SURFACE_D1 = [
    [Fr(5034629, 3763200), Fr(-23533, 15360), Fr(4259, 15360), Fr(-1103, 9216), Fr(151, 3072),
     Fr(-1171, 76800), Fr(139, 46080), Fr(-211, 752640)],
    [Fr(-363509, 3763200), Fr(6297, 5120), Fr(-6147, 5120), Fr(211, 3072), Fr(3, 1024),
     Fr(-153, 25600), Fr(29, 15360), Fr(-57, 250880)],
    [Fr(4631, 250880), Fr(-305, 3072), Fr(1245, 1024), Fr(-3725, 3072), Fr(275, 3072),
     Fr(-69, 5120), Fr(5, 3072), Fr(-5, 50176)],
]


def fornberg_weights(z0, nodes, m):
    """Finite-difference weights at z0 on arbitrary nodes (Fornberg's recursion).

    Returns c with c[k, i] the weight of f(nodes[i]) in the k-th derivative at
    z0, k = 0..m. Written from the published recursion: weights for the first
    n + 1 nodes are built from those for the first n by one new node at a time.
    Exact rational arithmetic when the inputs are Fractions.
    """
    nodes = list(nodes)
    n = len(nodes)
    c = [[0 * z0 for _ in range(n)] for _ in range(m + 1)]
    c[0][0] = 1 + 0 * z0
    c1 = 1 + 0 * z0
    c4 = nodes[0] - z0
    for i in range(1, n):
        mn = min(i, m)
        c2 = 1 + 0 * z0
        c5 = c4
        c4 = nodes[i] - z0
        for j in range(i):
            c3 = nodes[i] - nodes[j]
            c2 = c2 * c3
            if j == i - 1:
                for k in range(mn, 0, -1):
                    c[k][i] = c1 * (k * c[k - 1][i - 1] - c5 * c[k][i - 1]) / c2
                c[0][i] = -c1 * c5 * c[0][i - 1] / c2
            for k in range(mn, 0, -1):
                c[k][j] = (c4 * c[k][j] - k * c[k - 1][j]) / c3
            c[0][j] = c4 * c[0][j] / c3
        c1 = c2
    return c


def surface_dw_weights():
    """d_y w_y at y = -j h, j = 0..3, from w_0..w_7 (times 1/h): Fornberg on the
    surface point y = 0 plus the half rows y = -(i + 1/2) h, i = 0..7."""
    nodes = [Fr(0)] + [Fr(-(2 * i + 1), 2) for i in range(8)]
    rows = []
    for j in range(4):
        c = fornberg_weights(Fr(-j), nodes, 1)
        rows.append(c[1][1:])  # the surface node carries w_y = 0
    return rows


@dataclass(frozen=True)
class PMLGrid:
    nx: int
    ny: int
    h: float
    abc_cells: int = 0      # layer thickness delta = abc_cells * h (sides and bottom)
    beta0: float = 0.0      # beta_0 of the profile (1/s)

    ndim = 2
    order = 8

    @property
    def shape(self):
        return (self.ny, self.nx)

    @property
    def npts(self):
        return self.nx * self.ny

    @property
    def nfields(self):
        return 4

    @property
    def nstate(self):
        return 4 * self.npts


def bottom_profile(n, h, cells, beta0, half):
    """beta_y along depth: distance to the bottom row n-1 only (no layer at the
    surface); rows j (half: j + 1/2), clamped at 0 below the last row."""
    pos = np.arange(n, dtype=np.float64) + (0.5 if half else 0.0)
    d = np.maximum((n - 1) - pos, 0.0) * h
    delta = cells * h
    out = np.zeros(n)
    if cells > 0 and beta0 != 0.0:
        inside = d < delta
        out[inside] = beta0 * (1.0 - d[inside] / delta) ** 2
    return out


def betas(g):
    """(bx_node, bx_half, by_node, by_half): 1D profiles along x and depth."""
    bx = damping_profile(g.nx, g.h, g.abc_cells, g.beta0, False)
    bxh = damping_profile(g.nx, g.h, g.abc_cells, g.beta0, True)
    by = bottom_profile(g.ny, g.h, g.abc_cells, g.beta0, False)
    byh = bottom_profile(g.ny, g.h, g.abc_cells, g.beta0, True)
    return bx, bxh, by, byh


def _sx(f, s):
    """g[:, i] = f[:, i + s], zero outside."""
    g = np.zeros_like(f)
    n = f.shape[1]
    if s >= 0:
        g[:, : max(n - s, 0)] = f[:, s:]
    else:
        g[:, -s:] = f[:, : n + s]
    return g


def _sy(f, s):
    """g[j, :] = f[j + s, :], zero outside."""
    g = np.zeros_like(f)
    n = f.shape[0]
    if s >= 0:
        g[: max(n - s, 0), :] = f[s:, :]
    else:
        g[-s:, :] = f[: n + s, :]
    return g


def dx_plus(g, u):
    """d_x u at (i + 1/2, j)."""
    a = staggered_weights(8)
    return sum(a[l - 1] * (_sx(u, l) - _sx(u, 1 - l)) for l in range(1, 5)) / g.h


def dx_minus(g, w):
    """d_x w_x at nodes from the half points."""
    a = staggered_weights(8)
    return sum(a[l - 1] * (_sx(w, l - 1) - _sx(w, -l)) for l in range(1, 5)) / g.h


def dxx(g, u):
    return (D2_CENTER * u + sum(D2_WEIGHTS[l - 1] * (_sx(u, l) + _sx(u, -l)) for l in range(1, 5))) / g.h ** 2


def dyy(g, u):
    out = (D2_CENTER * u + sum(D2_WEIGHTS[l - 1] * (_sy(u, l) + _sy(u, -l)) for l in range(1, 5))) / g.h ** 2
    for j, row in enumerate(SURFACE_D2):
        out[j] = sum(float(cf) * u[i] for i, cf in enumerate(row)) / g.h ** 2
    return out


def dy_half(g, u):
    """d_y u (y up) at the half rows y = -(j + 1/2) h."""
    a = staggered_weights(8)
    out = sum(a[l - 1] * (_sy(u, 1 - l) - _sy(u, l)) for l in range(1, 5)) / g.h
    for j, row in enumerate(SURFACE_D1):
        out[j] = sum(float(cf) * u[i] for i, cf in enumerate(row)) / g.h
    return out


def dy_w(g, w):
    """d_y w_y (y up) at the rows y = -j h, with w_y = 0 at the surface."""
    a = staggered_weights(8)
    out = sum(a[l - 1] * (_sy(w, -l) - _sy(w, l - 1)) for l in range(1, 5)) / g.h
    for j, row in enumerate(surface_dw_weights()):
        out[j] = sum(float(cf) * w[i] for i, cf in enumerate(row)) / g.h
    return out


def split(g, U):
    return [U[k * g.npts:(k + 1) * g.npts].reshape(g.shape) for k in range(4)]


def apply_H_pml(g, c2, U):
    """H U for the 4-field PML system (Sec. 2), c2 of shape (ny, nx)."""
    if g.ny < 9:
        raise ValueError("the free-surface stencils need at least 9 rows")
    u, v, wx, wy = split(g, np.asarray(U, dtype=np.float64))
    bx, bxh, by, byh = betas(g)
    BX, BXH = bx[None, :], bxh[None, :]
    BY, BYH = by[:, None], byh[:, None]
    hu = v
    hv = (-BX * BY * u + c2 * (dxx(g, u) + dyy(g, u)) - (BX + BY) * v
          + c2 * (dx_minus(g, wx) + dy_w(g, wy)))
    hwx = (BY - BXH) * dx_plus(g, u) - BXH * wx
    hwy = (BX - BYH) * dy_half(g, u) - BYH * wy
    return np.concatenate([f.ravel() for f in (hu, hv, hwx, hwy)])


def assemble_H_pml(g, c2):
    """Dense H (small grids only), column by column."""
    n = g.nstate
    M = np.zeros((n, n))
    e = np.zeros(n)
    for k in range(n):
        e[k] = 1.0
        M[:, k] = apply_H_pml(g, c2, e)
        e[k] = 0.0
    return M


@dataclass(frozen=True)
class PMLSources:
    """Point sources on the v equation: node indices are grid points."""
    points: tuple
    amps: tuple
    f_peak: float
    t_delay: float

    def state_nodes(self, g):
        return [g.npts + int(p) for p in self.points]


class PMLProblem:
    """The interface the oracle steppers use (H, forcing, source columns)."""

    def __init__(self, g, c2, src=None, rect=None):
        from .source import PointSources
        self.grid = g
        self.c2 = np.asarray(c2, dtype=np.float64)
        self.rect = rect
        # the steppers' W and forcing take state indices: shift the points
        # onto the v field
        self.src = None if src is None else PointSources(
            tuple(src.state_nodes(g)), tuple(src.amps), src.f_peak, src.t_delay)

    def H(self, U):
        return apply_H_pml(self.grid, self.c2, U)

    def forcing(self, t):
        if self.src is None:
            return np.zeros(self.grid.nstate)
        return self.src.forcing(self.grid, t)

    def ellipse(self):
        from .spectrum import ellipse_from_rectangle
        x_lo, B = self.rect if self.rect is not None else spectrum_rectangle_pml(self.grid, self.c2)
        return ellipse_from_rectangle(x_lo, B)


# The one-sided surface rows raise the largest frequency of the discrete
# operator about 22 % above the interior symbol bound (dense eigenvalues of
# small grids, with and without the layer and for several media); B carries
# this margin so that the Faber ellipse through the rectangle's corners, whose
# height at Re = 0 is B, still encloses the spectrum.
SURFACE_MARGIN = 1.25


def spectrum_rectangle_pml(g, c2):
    """(x_lo, B) of the rectangle [x_lo, 0] x i[-B, B] around the spectrum of
    the PML operator (a reading; the paper gives no formula).

    B = SURFACE_MARGIN * c_max * sqrt(2 s) with s = (|D2_CENTER| + 2 sum |b_l|)
    / h^2 the largest symbol of the centred second derivative along one axis;
    x_lo = -(max beta_x + max beta_y), the real part of the u-v block's
    eigenvalues at zero wavenumber being -beta_x and -beta_y.
    """
    sym = (abs(D2_CENTER) + 2.0 * np.sum(np.abs(D2_WEIGHTS))) / g.h ** 2
    B = SURFACE_MARGIN * np.sqrt(np.max(c2)) * np.sqrt(2.0 * sym)
    bx, bxh, by, byh = betas(g)
    x_lo = -float(max(np.max(bx), np.max(bxh)) + max(np.max(by), np.max(byh)))
    return x_lo, float(B)
