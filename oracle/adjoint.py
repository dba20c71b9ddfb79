"""Oracle: the adjoint of the Faber step and the c^2 gradient of a receiver
misfit, written from the definitions.

Test infrastructure only (see the package docstring).

Paper anchors: the Faber recurrence and sum of Sec. 3.2, and the motivation of
Sec. 1 and Sec. 3.3 (large steps mean few stored wavefields for adjoint-based
inversion). The paper gives no adjoint; what follows is the exact discrete
adjoint of the forward step as built here.

- H^T: with (D+)^T = -D- (zero ghosts, checked by a test),
      (H^T Y)_p   = sum_a D-_a y_{v_a} - sigma_p y_p
      (H^T Y)_v_a = D+_a (c^2 y_p) - sigma_a(half) y_{v_a}
- Faber step u' = sum_j a_j v_j with v_0 = u, v_1 = A v_0, v_2 = A v_1 - 2 c1 v_0,
  v_j = A v_{j-1} - c1 v_{j-2} (A = H/gamma - c0 I) plus source terms that do
  not depend on u or c^2. For a functional <lam, u'>, the derivatives mu_j with
  respect to v_j satisfy, from j = m down to 0,
      mu_j = a_j lam + A^T mu_{j+1} - c_{j+2} mu_{j+2}   (mu_{m+1} = mu_{m+2} = 0,
                                                        c_2 = 2 c1, c_j = c1 for j > 2)
  so d<lam, u'>/du = mu_0, and since only the pressure row of H holds c^2,
      d<lam, u'>/dc^2[i] = -(1/gamma) sum_{j=1..m} mu_{j,p}[i] (sum_a D-_a v_{j-1,a})[i].
  The ellipse and the coefficients are held fixed.
"""
from __future__ import annotations

import numpy as np

from .operator import d_minus, d_plus, damping_fields, join_state, split_state
from .spectrum import faber_coefficients
from .steppers import faber_step, faber_terms


def apply_HT(grid, c2, Y):
    """y -> H^T y (transpose of the operator of oracle.operator.apply_H)."""
    fields = split_state(grid, Y)
    yp, yv = fields[0], fields[1:]
    sig_p, sig_v = damping_fields(grid)
    out_p = -sig_p * yp
    for a in range(grid.ndim):
        out_p = out_p + d_minus(grid, yv[a], a)
    out = [out_p]
    for a in range(grid.ndim):
        out.append(d_plus(grid, c2 * yp, a) - sig_v[a] * yv[a])
    return join_state(out)


def divergence_of_velocity(grid, U):
    """sum_a D-_a v_a of a state (the factor of c^2 in the pressure row of H)."""
    fields = split_state(grid, U)
    div = np.zeros(grid.shape)
    for a in range(grid.ndim):
        div = div + d_minus(grid, fields[1 + a], a)
    return div.ravel()


def faber_adjoint_step(prob, U, lam, t, dt, m, p=8, ellipse=None):
    """(d<lam, u'>/du, d<lam, u'>/dc^2) for the Faber step u' = step(U) from t."""
    g = prob.grid
    gamma, c0, c1 = ellipse if ellipse is not None else prob.ellipse()
    a = faber_coefficients(gamma, c0, c1, dt, m)
    v = [x[: g.nstate] for x in faber_terms(prob, U, t, m, p, (gamma, c0, c1))]
    mu = [None] * (m + 3)
    zero = np.zeros(g.nstate)
    mu[m + 1] = zero
    mu[m + 2] = zero

    def cc(j):  # the coefficient of v_{j-2} in the definition of v_j
        return 0.0 if j < 2 else (2.0 * c1 if j == 2 else c1)

    for j in range(m, -1, -1):
        At_mu = apply_HT(g, prob.c2, mu[j + 1]) / gamma - c0 * mu[j + 1]
        mu[j] = a[j] * lam + At_mu - cc(j + 2) * mu[j + 2]
    grad = np.zeros(g.npts)
    for j in range(1, m + 1):
        grad -= (1.0 / gamma) * mu[j][: g.npts] * divergence_of_velocity(g, v[j - 1])
    return mu[0], grad


def misfit(prob, U0, t0, dt, nsteps, m, receivers, d_obs, p=8, ellipse=None):
    """L = 1/2 sum_n |u_{n+1}[rec] - d_obs[n]|^2 over nsteps Faber steps."""
    U = np.array(U0, dtype=np.float64)
    L = 0.0
    for n in range(nsteps):
        U = faber_step(prob, U, t0 + n * dt, dt, m, p, ellipse)
        r = U[receivers] - d_obs[n]
        L += 0.5 * float(r @ r)
    return L


def misfit_gradient(prob, U0, t0, dt, nsteps, m, receivers, d_obs, p=8, ellipse=None):
    """(L, dL/dc^2, dL/dU0) by the adjoint: all states kept (small cases)."""
    g = prob.grid
    ell = ellipse if ellipse is not None else prob.ellipse()
    states = [np.array(U0, dtype=np.float64)]
    for n in range(nsteps):
        states.append(faber_step(prob, states[-1], t0 + n * dt, dt, m, p, ell))
    L = 0.0
    lam = np.zeros(g.nstate)
    grad = np.zeros(g.npts)
    for n in range(nsteps - 1, -1, -1):
        r = states[n + 1][receivers] - d_obs[n]
        L += 0.5 * float(r @ r)
        np.add.at(lam, receivers, r)        # dL/du_{n+1} from the misfit at step n
        lam, gn = faber_adjoint_step(prob, states[n], lam, t0 + n * dt, dt, m, p, ell)
        grad += gn
    return L, grad, lam
