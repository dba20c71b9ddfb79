"""Oracle: plain definitions used to pin the steppers.

Test infrastructure only (see the package docstring).

Paper anchor: Sec. 3.2, variation-of-constants formula
    U(t) = e^{(t - t0) H} U0 + int_{t0}^{t} e^{(t - tau) H} f(tau) dtau.
Here it is evaluated with library matrix exponentials (scipy.linalg.expm on
dense matrices, scipy.sparse.linalg.expm_multiply on sparse ones) and
Gauss-Legendre quadrature of the integral, independently of the augmented
matrix and of every stepper.

The periodic plane wave is the closed-form solution of the semi-discrete
system in a homogeneous medium without damping: with the staggered symbol
K(k) = (2/h) sum_l alpha_l sin((2l - 1) k h / 2) and omega = c |K|,
    p   = cos(k.x - omega t)
    v_a = (K_a / omega) cos(k.x_a - omega t),   x_a = x shifted h/2 along a.
"""
from __future__ import annotations

import numpy as np
from scipy.sparse.linalg import expm_multiply

from .operator import assemble_H, join_state, staggered_weights
from .source import ricker


class ExactPropagator:
    """Exact semi-discrete stepping U(t) -> U(t + dt) for a Problem."""

    def __init__(self, prob, nquad=24):
        self.prob = prob
        self.A = assemble_H(prob.grid, prob.c2).tocsc()
        self.nquad = nquad
        g = prob.grid
        self.b = np.zeros(g.nstate)
        if prob.src is not None:
            for node, st in zip(prob.src.nodes, prob.src.strengths(g)):
                self.b[node] += st

    def step(self, U, t, dt):
        out = expm_multiply(dt * self.A, np.asarray(U, dtype=np.float64))
        src = self.prob.src
        if src is not None:
            x, w = np.polynomial.legendre.leggauss(self.nquad)
            taus = t + 0.5 * dt * (x + 1.0)
            wts = 0.5 * dt * w
            for tq, wq in zip(taus, wts):
                gq = ricker(tq, src.f_peak, src.t_delay)
                out += wq * gq * expm_multiply((t + dt - tq) * self.A, self.b)
        return out

    def run(self, U0, t0, dt, nsteps):
        U = np.array(U0, dtype=np.float64)
        for n in range(nsteps):
            U = self.step(U, t0 + n * dt, dt)
        return U


def staggered_symbol(k, h, order):
    alpha = staggered_weights(order)
    return (2.0 / h) * sum(al * np.sin((2 * l - 1) * k * h / 2.0)
                           for l, al in enumerate(alpha, start=1))


def plane_wave(grid, c, modes, t):
    """Periodic plane wave with integer wave numbers `modes` (one per axis)."""
    kvec = [2.0 * np.pi * modes[a] / (grid.n[a] * grid.h) for a in range(grid.ndim)]
    K = np.array([staggered_symbol(kvec[a], grid.h, grid.order) for a in range(grid.ndim)])
    omega = c * np.linalg.norm(K)
    axes = [np.arange(grid.n[a]) * grid.h for a in range(grid.ndim)]
    # numpy arrays indexed [z, (y,) x]
    mesh = np.meshgrid(*[axes[a] for a in reversed(range(grid.ndim))], indexing="ij")
    pos = [mesh[grid.ndim - 1 - a] for a in range(grid.ndim)]   # pos[a] = coordinate along axis a
    phase = sum(kvec[a] * pos[a] for a in range(grid.ndim)) - omega * t
    fields = [np.cos(phase)]
    for a in range(grid.ndim):
        fields.append((K[a] / omega) * np.cos(phase + kvec[a] * grid.h / 2.0))
    return join_state(fields), omega
