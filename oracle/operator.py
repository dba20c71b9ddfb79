"""Oracle: grid, damping profiles and the semi-discrete acoustic operator H.

Test infrastructure only (see the package docstring).

Paper anchors:
- Sec. 2 (the wave equation): quadratic absorption profile
  beta(d) = beta_0 (1 - d/delta)^2 inside a layer of thickness delta, zero
  outside; values outside the domain are zero (Sec. 2.1, zero ghost rule).
- Sec. 2.1 (spatial discretization): staggered first-derivative stencil; the
  paper prints the 8th-order weights 1225/1024 (1, -1/15, 1/125, -1/1715).
- Sec. 3 (time integration methods): the semi-discrete system U' = H U + f.

Reading used for the operator (the paper's own operator is the 4-field PML
system; the operator here is the first-order pressure/velocity system with a
diagonal damping layer, rho = 1):

    (H U)_p   = -c^2 sum_a D-_a v_a - (sum_a sigma_a(x_a)) p
    (H U)_v_a = -D+_a p - sigma_a(x_a + h/2) v_a

with p at nodes, v_a half a cell forward along axis a, and
    (D+ f)[i] = (1/h) sum_l alpha_l (f[i+l] - f[i+1-l])      (at i + 1/2)
    (D- v)[i] = (1/h) sum_l alpha_l (v[i+l-1] - v[i-l])      (at i)

Layout: a field is a numpy array of shape (nz, nx) or (nz, ny, nx); logical
axis a (0 = x, 1 = y or z, 2 = z) is numpy axis ndim-1-a. The state vector is
the concatenation [p | v_0 | ... | v_{d-1}] of flattened fields.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


def staggered_weights(order):
    """Staggered first-derivative weights alpha_1..alpha_K (Sec. 2.1).

    order 8 is the stencil the paper prints; order 4 is the two-point member
    of the same family (exact for cubics, pinned by a polynomial test).
    """
    if order == 4:
        return np.array([9.0 / 8.0, -1.0 / 24.0])
    if order == 8:
        return 1225.0 / 1024.0 * np.array([1.0, -1.0 / 15.0, 1.0 / 125.0, -1.0 / 1715.0])
    raise ValueError("order must be 4 or 8")


@dataclass(frozen=True)
class Grid:
    n: tuple                 # (nx, nz) or (nx, ny, nz)
    h: float
    order: int = 4
    bc: str = "zero"         # "zero" ghost values, or "periodic" (closed-form tests)
    abc_cells: int = 0       # damping-layer thickness L in cells (delta = L h)
    sigma_max: float = 0.0   # beta_0 of the paper's profile (1/s)
    # optional caller-given 1D damping profiles (1/s), 2 * ndim arrays: axis a
    # at the integer points x_i = i h (entry 2a) and at the half points
    # (i + 1/2) h (entry 2a + 1), each of n[a] values >= 0; when given they
    # replace the quadratic profile of (abc_cells, sigma_max)
    profiles: tuple = None

    @property
    def ndim(self):
        return len(self.n)

    @property
    def shape(self):
        return tuple(int(v) for v in reversed(self.n))

    @property
    def npts(self):
        return int(np.prod(self.n))

    @property
    def nfields(self):
        return 1 + self.ndim

    @property
    def nstate(self):
        return self.nfields * self.npts

    def np_axis(self, a):
        return self.ndim - 1 - a


def damping_profile(n, h, cells, sigma_max, half):
    """1D damping values along one axis (Sec. 2, absorption profile).

    Points are x_i = i h (half=False) or x_i = (i + 1/2) h (half=True). The
    distance d to the domain boundary is measured to the nearest outer node
    (0 or n-1) and clamped at 0 for the half point beyond the last node;
    sigma = sigma_max (1 - d/delta)^2 for d < delta = cells * h, else 0.
    """
    pos = np.arange(n, dtype=np.float64) + (0.5 if half else 0.0)
    d = np.minimum(pos, (n - 1) - pos) * h
    d = np.maximum(d, 0.0)
    delta = cells * h
    out = np.zeros(n)
    if cells > 0 and sigma_max != 0.0:
        inside = d < delta
        out[inside] = sigma_max * (1.0 - d[inside] / delta) ** 2
    return out


def _broadcast_axis(grid, a, vec):
    shp = [1] * grid.ndim
    shp[grid.np_axis(a)] = grid.n[a]
    return vec.reshape(shp)


def axis_profiles(grid, a):
    """(integer-point, half-point) damping values along axis a."""
    if grid.profiles is not None:
        return (np.asarray(grid.profiles[2 * a], dtype=np.float64),
                np.asarray(grid.profiles[2 * a + 1], dtype=np.float64))
    return (damping_profile(grid.n[a], grid.h, grid.abc_cells, grid.sigma_max, False),
            damping_profile(grid.n[a], grid.h, grid.abc_cells, grid.sigma_max, True))


def damping_fields(grid):
    """sigma_p on nodes (sum over axes) and sigma_a at the v_a points."""
    sig_p = np.zeros(grid.shape)
    sig_v = []
    for a in range(grid.ndim):
        s_int, s_half = axis_profiles(grid, a)
        sig_p = sig_p + _broadcast_axis(grid, a, s_int)
        sig_v.append(np.broadcast_to(_broadcast_axis(grid, a, s_half), grid.shape))
    return sig_p, sig_v


def _shift(f, s, ax, bc):
    """g[i] = f[i + s] along numpy axis ax; zero outside (or wrapped)."""
    if bc == "periodic":
        return np.roll(f, -s, axis=ax)
    n = f.shape[ax]
    out = np.zeros_like(f)
    if abs(s) >= n:
        return out
    src = [slice(None)] * f.ndim
    dst = [slice(None)] * f.ndim
    if s >= 0:
        src[ax] = slice(s, n)
        dst[ax] = slice(0, n - s)
    else:
        src[ax] = slice(0, n + s)
        dst[ax] = slice(-s, n)
    out[tuple(dst)] = f[tuple(src)]
    return out


def d_plus(grid, f, a):
    """Forward staggered derivative of a node field along axis a (at i+1/2)."""
    alpha = staggered_weights(grid.order)
    ax = grid.np_axis(a)
    out = np.zeros_like(f)
    for l, al in enumerate(alpha, start=1):
        out += al * (_shift(f, l, ax, grid.bc) - _shift(f, 1 - l, ax, grid.bc))
    return out / grid.h


def d_minus(grid, v, a):
    """Backward staggered derivative of a half-point field along axis a (at i)."""
    alpha = staggered_weights(grid.order)
    ax = grid.np_axis(a)
    out = np.zeros_like(v)
    for l, al in enumerate(alpha, start=1):
        out += al * (_shift(v, l - 1, ax, grid.bc) - _shift(v, -l, ax, grid.bc))
    return out / grid.h


def split_state(grid, U):
    U = np.asarray(U)
    n = grid.npts
    return [U[f * n:(f + 1) * n].reshape(grid.shape) for f in range(grid.nfields)]


def join_state(fields):
    return np.concatenate([np.asarray(f).ravel() for f in fields])


def apply_H(grid, c2, U):
    """y = H U for the pressure/velocity system (Sec. 3, U' = H U + f)."""
    fields = split_state(grid, U)
    p, vs = fields[0], fields[1:]
    sig_p, sig_v = damping_fields(grid)
    div = np.zeros(grid.shape)
    for a in range(grid.ndim):
        div += d_minus(grid, vs[a], a)
    out = [-c2 * div - sig_p * p]
    for a in range(grid.ndim):
        out.append(-d_plus(grid, p, a) - sig_v[a] * vs[a])
    return join_state(out)


def _diff_matrix_1d(n, h, order, bc, kind):
    """1D staggered difference matrix written entry by entry from its definition."""
    alpha = staggered_weights(order)
    rows, cols, vals = [], [], []
    for i in range(n):
        for l, al in enumerate(alpha, start=1):
            if kind == "plus":
                pairs = ((i + l, al), (i + 1 - l, -al))
            else:
                pairs = ((i + l - 1, al), (i - l, -al))
            for j, w in pairs:
                if bc == "periodic":
                    j = j % n
                elif j < 0 or j >= n:
                    continue
                rows.append(i)
                cols.append(j)
                vals.append(w / h)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def _axis_operator(grid, a, mat1d):
    """Lift a 1D operator on axis a to the flat (x fastest) grid index."""
    out = None
    for b in reversed(range(grid.ndim)):          # slowest axis first
        blk = mat1d if b == a else sp.identity(grid.n[b], format="csr")
        out = blk if out is None else sp.kron(out, blk, format="csr")
    return out


def assemble_H(grid, c2):
    """H as a sparse matrix, built independently of `apply_H` from 1D blocks."""
    d = grid.ndim
    sig_p, sig_v = damping_fields(grid)
    C2 = sp.diags(np.asarray(c2, dtype=np.float64).ravel())
    blocks = [[None] * (d + 1) for _ in range(d + 1)]
    blocks[0][0] = -sp.diags(sig_p.ravel())
    for a in range(d):
        Dp = _axis_operator(grid, a, _diff_matrix_1d(grid.n[a], grid.h, grid.order, grid.bc, "plus"))
        Dm = _axis_operator(grid, a, _diff_matrix_1d(grid.n[a], grid.h, grid.order, grid.bc, "minus"))
        blocks[0][1 + a] = -(C2 @ Dm)
        blocks[1 + a][0] = -Dp
        blocks[1 + a][1 + a] = -sp.diags(np.ascontiguousarray(sig_v[a]).ravel())
    return sp.bmat(blocks, format="csr")


def energy(grid, c2, U):
    """Acoustic energy E = (h^d / 2) sum (p^2 / c^2 + |v|^2)."""
    fields = split_state(grid, U)
    e = np.sum(fields[0] ** 2 / c2)
    for v in fields[1:]:
        e += np.sum(v ** 2)
    return 0.5 * grid.h ** grid.ndim * e


def interior_mask(grid):
    """Nodes outside the damping layer (the paper's 'physical space')."""
    m = np.ones(grid.shape, dtype=bool)
    L = grid.abc_cells
    for a in range(grid.ndim):
        idx = np.arange(grid.n[a])
        inside = (idx >= L) & (idx <= grid.n[a] - 1 - L)
        m &= _broadcast_axis(grid, a, inside)
    return m


def rel_l2_pressure(grid, U_test, U_ref, interior=True):
    """Relative L2 error of the pressure field (optionally interior only)."""
    p_t = split_state(grid, U_test)[0]
    p_r = split_state(grid, U_ref)[0]
    if interior:
        msk = interior_mask(grid)
        p_t, p_r = p_t[msk], p_r[msk]
    den = np.linalg.norm(p_r)
    return float(np.linalg.norm(p_t - p_r) / den) if den > 0 else float(np.linalg.norm(p_t))
