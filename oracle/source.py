"""Oracle: Ricker source, its derivatives and the augmented-matrix tail.

Test infrastructure only (see the package docstring).

Paper anchors:
- Sec. 4 (single-signal experiment): a Ricker wavelet point source with a
  delay t0 (0.18 s in the paper's experiments).
- Sec. 3.2 (high order methods): expanding the source in a Taylor series
  turns the variation-of-constants formula into one exponential of the
  augmented matrix  H~ = [[H, W], [0, J]]  applied to [u; e_p], where the
  columns of W are the source and its first p-1 derivatives and J is the p x p
  matrix with ones on the superdiagonal.

Readings: g(t) = (1 - 2 a tau^2) exp(-a tau^2), a = (pi f)^2, tau = t - t0;
derivatives are exact (Hermite closed form) rather than approximated; the
source enters the pressure equation at node s with strength amp_s / h^d. The
columns of W are ordered [g^(p-1), ..., g', g] so that exp(t J) e_p holds the
Taylor monomials t^(p-c)/(p-c)! in entry c (1-based).
"""
from __future__ import annotations

from dataclasses import dataclass

from math import factorial

import numpy as np


def ricker(t, f_peak, t_delay):
    a = (np.pi * f_peak) ** 2
    tau = np.asarray(t, dtype=np.float64) - t_delay
    return (1.0 - 2.0 * a * tau * tau) * np.exp(-a * tau * tau)


def hermite_phys(nmax, x):
    """Physicists' Hermite polynomials H_0..H_nmax at x (three-term recurrence)."""
    x = np.asarray(x, dtype=np.float64)
    H = [np.ones_like(x), 2.0 * x]
    for n in range(1, nmax):
        H.append(2.0 * x * H[n] - 2.0 * n * H[n - 1])
    return H[: nmax + 1]


def ricker_derivatives(t, f_peak, t_delay, p):
    """[g(t), g'(t), ..., g^(p-1)(t)].

    g = -(1/(2a)) d^2/dtau^2 exp(-a tau^2) and
    d^n/dtau^n exp(-a tau^2) = (-1)^n a^(n/2) H_n(sqrt(a) tau) exp(-a tau^2),
    so g^(k) = -(1/(2a)) (-1)^k a^((k+2)/2) H_{k+2}(sqrt(a) tau) exp(-a tau^2).
    """
    a = (np.pi * f_peak) ** 2
    tau = float(t) - t_delay
    x = np.sqrt(a) * tau
    H = hermite_phys(p + 1, x)
    e = np.exp(-a * tau * tau)
    return np.array([-(1.0 / (2.0 * a)) * (-1.0) ** k * a ** ((k + 2) / 2.0) * H[k + 2] * e
                     for k in range(p)])


@dataclass(frozen=True)
class PointSources:
    """Point sources sharing one Ricker wavelet: flat pressure-node indices and amplitudes."""
    nodes: tuple
    amps: tuple
    f_peak: float
    t_delay: float

    def strengths(self, grid):
        return np.asarray(self.amps, dtype=np.float64) / grid.h ** grid.ndim

    def forcing(self, grid, t):
        """s(t): the forcing vector of U' = H U + s(t) (pressure entries only)."""
        s = np.zeros(grid.nstate)
        g = ricker(t, self.f_peak, self.t_delay)
        for node, st in zip(self.nodes, self.strengths(grid)):
            s[node] += st * g
        return s

    def w_columns(self, t, p):
        """Row vector G with W = e_src G: [g^(p-1)(t), ..., g(t)]."""
        return ricker_derivatives(t, self.f_peak, self.t_delay, p)[::-1].copy()


class TaylorTableSource:
    """Point sources with a tabulated time function: row n of table holds
    g^(k)(t_n), k = 0..p-1 (Sec. 3.2, augmented matrix: over a step the source
    is its Taylor polynomial). bind(n, t_n) selects the step; forcing evaluates
    the row's polynomial at t - t_n, and w_columns returns the row in the
    column order of W (highest derivative first)."""

    def __init__(self, nodes, amps, table):
        self.nodes = tuple(int(v) for v in nodes)
        self.amps = tuple(float(a) for a in amps)
        self.table = np.asarray(table, dtype=np.float64)
        self.step, self.t_n = 0, 0.0

    def bind(self, n, t_n):
        self.step, self.t_n = int(n), float(t_n)

    def strengths(self, grid):
        return np.asarray(self.amps, dtype=np.float64) / grid.h ** grid.ndim

    def value(self, t):
        tau = t - self.t_n
        row = self.table[self.step]
        return float(sum(row[k] * tau ** k / factorial(k) for k in range(row.size)))

    def forcing(self, grid, t):
        s = np.zeros(grid.nstate)
        g = self.value(t)
        for node, st in zip(self.nodes, self.strengths(grid)):
            s[node] += st * g
        return s

    def w_columns(self, t, p):
        return self.table[self.step, :p][::-1].copy()


def apply_W(grid, src, G, tau):
    """W tau as a state vector: strength_s * (G . tau) at each source node."""
    out = np.zeros(grid.nstate)
    val = float(np.dot(G, tau))
    for node, st in zip(src.nodes, src.strengths(grid)):
        out[node] += st * val
    return out


def apply_J(tau):
    """J tau with J the shift matrix (ones on the superdiagonal)."""
    out = np.zeros_like(tau)
    out[:-1] = tau[1:]
    return out


def e_p(p):
    v = np.zeros(p)
    v[-1] = 1.0
    return v
