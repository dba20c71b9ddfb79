"""Oracle: the time steppers of the paper, one plain step at a time.

Test infrastructure only (see the package docstring).

Paper anchors (Sec. 3, time integration methods):
- Faber approximation (FA): three-term Faber recurrence on the augmented
  matrix, u^{n+1} = sum_{j<=m} a_j F_j(H~) [u^n; e_p]  (m matrix-vector products).
- Krylov subspace projection (KRY): Arnoldi with modified Gram-Schmidt on
  H~, then the small Hessenberg exponential by Pade (scipy's expm is the
  scaling-and-squaring Pade method); exp(dt H~) x ~ beta V_k exp(dt H_k) e_1.
- RK4-4 (classical), RK3-2 (as printed), HORK (Gottlieb-Shu-Tadmor linear
  SSP family) and leap-frog.

Readings (no implementation is given in the paper):
- Krylov: the listing's inner coefficient is the (k, j) entry; the square
  k x k block is exponentiated with dt absorbed; breakdown when
  h_{j+1,j} <= 1e-14 beta; beta is the Euclidean norm over all entries of the
  augmented vector.
- Leap-frog for the first-order system is the staggered-time (Yee) scheme
  with Crank-Nicolson averaged damping; the state holds p at t_n and v at
  t_n - dt/2; the source is sampled at t_n + dt/2.
- HORK coefficients: alpha_{1,0} = 1, alpha_{m,k} = alpha_{m-1,k-1}/k
  (1 <= k <= m-2), alpha_{m,m-1} = 1/m!, alpha_{m,0} = 1 - sum_{k>=1} alpha_{m,k}.
"""
from __future__ import annotations

from dataclasses import dataclass
from math import factorial

import numpy as np
from scipy.linalg import expm

from .operator import apply_H, d_minus, d_plus, damping_fields, join_state, split_state
from .source import apply_J, apply_W, e_p
from .spectrum import ellipse_from_rectangle, faber_coefficients, spectrum_rectangle


@dataclass
class Problem:
    grid: object
    c2: np.ndarray
    src: object = None          # PointSources or None

    def H(self, U):
        return apply_H(self.grid, self.c2, U)

    def forcing(self, t):
        if self.src is None:
            return np.zeros(self.grid.nstate)
        return self.src.forcing(self.grid, t)

    def ellipse(self):
        return ellipse_from_rectangle(*spectrum_rectangle(self.grid, self.c2))


def _augment(prob, U, p):
    return np.concatenate([U, e_p(p)]) if prob.src is not None else np.array(U, dtype=np.float64)


def apply_Htilde(prob, x, G):
    """H~ x for the augmented vector x = [u; tau] (plain H when no source)."""
    if prob.src is None:
        return prob.H(x)
    n = prob.grid.nstate
    u, tau = x[:n], x[n:]
    top = prob.H(u) + apply_W(prob.grid, prob.src, G, tau)
    return np.concatenate([top, apply_J(tau)])


def faber_step(prob, U, t, dt, m, p=8, ellipse=None):
    """One Faber step of degree m from t to t + dt (m products with H~)."""
    gamma, c0, c1 = ellipse if ellipse is not None else prob.ellipse()
    a = faber_coefficients(gamma, c0, c1, dt, m)
    G = prob.src.w_columns(t, p) if prob.src is not None else None
    x0 = _augment(prob, U, p)

    def F1(x):
        return apply_Htilde(prob, x, G) / gamma - c0 * x

    acc = a[0] * x0
    if m >= 1:
        v1 = F1(x0)
        acc = acc + a[1] * v1
    if m >= 2:
        v2 = F1(v1) - 2.0 * c1 * x0
        acc = acc + a[2] * v2
        older, prev = v1, v2
        for j in range(3, m + 1):
            vj = F1(prev) - c1 * older
            acc = acc + a[j] * vj
            older, prev = prev, vj
    return acc[: prob.grid.nstate].copy()


def faber_terms(prob, U, t, m, p=8, ellipse=None):
    """The terms v_j = F_j(H~) [U; e_p], j = 0..m, of a Faber step from t.

    They depend on the ellipse and on t (through the source columns) but not
    on the step size: only the weights a_j(dt) do (Sec. 3.2, Faber series).
    """
    gamma, c0, c1 = ellipse if ellipse is not None else prob.ellipse()
    G = prob.src.w_columns(t, p) if prob.src is not None else None
    terms = [_augment(prob, U, p)]
    for j in range(1, m + 1):
        v = apply_Htilde(prob, terms[j - 1], G) / gamma - c0 * terms[j - 1]
        if j == 2:
            v = v - 2.0 * c1 * terms[0]
        elif j > 2:
            v = v - c1 * terms[j - 2]
        terms.append(v)
    return terms


def faber_dense(prob, U, t, m, taus, nodes, p=8, ellipse=None):
    """Pressure at `nodes` at t + tau for each tau in taus from one set of
    Faber terms: sum_j a_j(tau) v_j, with a_j(0) = delta_j0 (exp(0) = I)."""
    gamma, c0, c1 = ellipse if ellipse is not None else prob.ellipse()
    nodes = np.asarray(nodes, dtype=np.int64)
    at_nodes = np.array([v[nodes] for v in faber_terms(prob, U, t, m, p, (gamma, c0, c1))])
    out = np.zeros((len(taus), nodes.size))
    for i, tau in enumerate(taus):
        if tau == 0.0:
            a = np.zeros(m + 1)
            a[0] = 1.0
        else:
            a = faber_coefficients(gamma, c0, c1, tau, m)
        out[i] = a @ at_nodes
    return out


def arnoldi(prob, x, G, k, breakdown=1e-14):
    """Arnoldi with modified Gram-Schmidt on H~: (beta, Q list, Hess, k_eff)."""
    beta = float(np.linalg.norm(x))
    Hm = np.zeros((k + 1, k))
    if beta == 0.0:
        return beta, [], Hm, 0
    Q = [x / beta]
    k_eff = k
    for j in range(k):
        w = apply_Htilde(prob, Q[j], G)
        for i in range(j + 1):
            Hm[i, j] = float(np.dot(w, Q[i]))
            w = w - Hm[i, j] * Q[i]
        Hm[j + 1, j] = float(np.linalg.norm(w))
        if Hm[j + 1, j] <= breakdown * beta:
            k_eff = j + 1
            break
        Q.append(w / Hm[j + 1, j])
    return beta, Q, Hm, k_eff


def krylov_step(prob, U, t, dt, k, p=8):
    """One Krylov step of dimension k (k products with H~)."""
    G = prob.src.w_columns(t, p) if prob.src is not None else None
    x = _augment(prob, U, p)
    beta, Q, Hm, k_eff = arnoldi(prob, x, G, k)
    if k_eff == 0:
        return np.zeros(prob.grid.nstate)
    y = expm(dt * Hm[:k_eff, :k_eff])[:, 0]
    out = np.zeros_like(x)
    for i in range(k_eff):
        out += y[i] * Q[i]
    return beta * out[: prob.grid.nstate]


def krylov_step_estimate(prob, U, t, dt, k, p=8):
    """(the Krylov step of dimension k, its a-posteriori error estimate).

    With u_k(s) = beta V_k exp(s H_k) e_1, the Arnoldi relation gives the
    residual of the projected flow r(s) = H~ u_k(s) - u_k'(s)
    = beta h_{k+1,k} (e_k^T exp(s H_k) e_1) q_{k+1}; the step's error is
    int_0^dt exp((dt - s) H~) r(s) ds, and the estimate is the norm of
    int_0^dt r(s) ds = dt beta h_{k+1,k} |e_k^T phi_1(dt H_k) e_1| q_{k+1},
    phi_1(z) = (e^z - 1)/z (Saad, 1992; the paper gives none). phi_1(A) e_1 is
    the upper right column of exp([[A, e_1], [0, 0]]). Zero after a breakdown
    (k_eff < k: the space is invariant)."""
    G = prob.src.w_columns(t, p) if prob.src is not None else None
    x = _augment(prob, U, p)
    beta, Q, Hm, k_eff = arnoldi(prob, x, G, k)
    if k_eff == 0:
        return np.zeros(prob.grid.nstate), 0.0
    y = expm(dt * Hm[:k_eff, :k_eff])[:, 0]
    out = np.zeros_like(x)
    for i in range(k_eff):
        out += y[i] * Q[i]
    est = 0.0
    if k_eff == k:
        Z = np.zeros((k + 1, k + 1))
        Z[:k, :k] = dt * Hm[:k, :k]
        Z[0, k] = 1.0
        phi = expm(Z)[:k, k]
        est = dt * beta * Hm[k, k - 1] * abs(phi[k - 1])
    return beta * out[: prob.grid.nstate], float(est)


def rk4_step(prob, U, t, dt):
    """Classical four-stage, fourth-order Runge-Kutta step of U' = H U + s(t)."""
    k1 = prob.H(U) + prob.forcing(t)
    k2 = prob.H(U + 0.5 * dt * k1) + prob.forcing(t + 0.5 * dt)
    k3 = prob.H(U + 0.5 * dt * k2) + prob.forcing(t + 0.5 * dt)
    k4 = prob.H(U + dt * k3) + prob.forcing(t + dt)
    return U + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def rk32_step(prob, U, t, dt):
    """Three-stage, second-order Runge-Kutta as printed in Sec. 3.1."""
    k1 = prob.H(U) + prob.forcing(t)
    k2 = prob.H(U + 0.5 * dt * k1) + prob.forcing(t + 0.5 * dt)
    k3 = prob.H(U + 0.5 * dt * k2) + prob.forcing(t + 0.5 * dt)
    return U + dt * k3


def hork_lambdas(m):
    """lambda_0..lambda_{m-1} of the order-m linear SSP Runge-Kutta method."""
    alpha = {1: np.array([1.0])}
    for q in range(2, m + 1):
        a = np.zeros(q)
        prev = alpha[q - 1]
        for kk in range(1, q - 1):
            a[kk] = prev[kk - 1] / kk
        a[q - 1] = 1.0 / factorial(q)
        a[0] = 1.0 - np.sum(a[1:])
        alpha[q] = a
    return alpha[m]


def hork_step(prob, U, t, dt, m, p=8):
    """HORK of order m on the augmented system (Sec. 3.2)."""
    lam = hork_lambdas(m)
    G = prob.src.w_columns(t, p) if prob.src is not None else None
    x = _augment(prob, U, p)

    def E(y):
        return y + dt * apply_Htilde(prob, y, G)

    ks = [x]
    for _ in range(1, m):
        ks.append(E(ks[-1]))
    out = lam[m - 1] * E(ks[m - 1])
    for i in range(m - 1):
        out = out + lam[i] * ks[i]
    return out[: prob.grid.nstate].copy()


def leapfrog_step(prob, U, t, dt):
    """Staggered-time leap-frog: U holds (p at t, v at t - dt/2)."""
    g = prob.grid
    fields = split_state(g, U)
    p, vs = fields[0], fields[1:]
    sig_p, sig_v = damping_fields(g)
    new_v = []
    for a in range(g.ndim):
        num = (1.0 - 0.5 * dt * sig_v[a]) * vs[a] - dt * d_plus(g, p, a)
        new_v.append(num / (1.0 + 0.5 * dt * sig_v[a]))
    div = np.zeros(g.shape)
    for a in range(g.ndim):
        div += d_minus(g, new_v[a], a)
    s = split_state(g, prob.forcing(t + 0.5 * dt))[0]
    num = (1.0 - 0.5 * dt * sig_p) * p - dt * prob.c2 * div + dt * s
    p_new = num / (1.0 + 0.5 * dt * sig_p)
    return join_state([p_new] + new_v)


def step(prob, method, U, t, dt, **kw):
    if method == "faber":
        return faber_step(prob, U, t, dt, kw["m"], kw.get("p", 8), kw.get("ellipse"))
    if method == "krylov":
        return krylov_step(prob, U, t, dt, kw["k"], kw.get("p", 8))
    if method == "rk4":
        return rk4_step(prob, U, t, dt)
    if method == "rk32":
        return rk32_step(prob, U, t, dt)
    if method == "hork":
        return hork_step(prob, U, t, dt, kw["m"], kw.get("p", 8))
    if method == "leapfrog":
        return leapfrog_step(prob, U, t, dt)
    raise ValueError(method)


def run(prob, method, U0, t0, dt, nsteps, receivers=None, snapshot_every=0, **kw):
    """Advance nsteps steps; record p at receiver nodes after every step.

    Returns (U_final, traces[nsteps, nrec], {step: U}) with step counted from 1.
    """
    U = np.array(U0, dtype=np.float64)
    rec = np.asarray(receivers if receivers is not None else [], dtype=np.int64)
    traces = np.zeros((nsteps, rec.size))
    snaps = {}
    if method == "faber" and kw.get("ellipse") is None:
        kw = dict(kw, ellipse=prob.ellipse())
    for n in range(nsteps):
        U = step(prob, method, U, t0 + n * dt, dt, **kw)
        if rec.size:
            traces[n] = U[rec]
        if snapshot_every and (n + 1) % snapshot_every == 0:
            snaps[n + 1] = U.copy()
    return U, traces, snaps
