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

Krylov (Sec. 3.2, Krylov subspace projection). The Krylov step is not a
fixed linear map of the state: its polynomial depends on the start vector
through the Arnoldi process. The reading taken here differentiates the
exponential the step approximates and approximates each factor the same way
the forward step does:
- the state adjoint is the Krylov approximation (dimension k, Arnoldi with
  modified Gram-Schmidt on H^T started from lam, no augmentation: the
  transposed augmented matrix leaves the state block of [lam; 0] to H^T
  alone) of exp(dt H^T) lam;
- the c^2 derivative of <lam, exp(dt H~) [U; e_p]> is
      dt int_0^1 <exp((1-s) dt H^T) lam, dH/dc^2[x] exp(s dt H~) [U; e_p]> ds,
  and dH/dc^2[x] y has the single entry -(sum_a D-_a y_{v_a})[x] in the
  pressure row x. With exp(s dt H~)[U; e_p] ~ beta V exp(s dt H_k) e_1 (the
  forward step's basis, any s) and exp(r dt H^T) lam ~ beta' W exp(r dt G_k) e_1,
      grad[x] = -dt sum_{a,b} C_ab W_{a,p}[x] (sum_a D-_a V_{b,v_a})[x],
      C = beta beta' int_0^1 exp((1-s) dt G_k) e_1 e_1^T exp(s dt H_k^T) ds,
  the integral being the upper right block of the exponential of the block
  triangular matrix [[dt G_k, e_1 e_1^T], [0, dt H_k^T]] (Van Loan, 1978).
Both converge to the derivatives of the exact exponential as k grows.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm

from .operator import d_minus, d_plus, damping_fields, join_state, split_state
from .source import e_p
from .spectrum import faber_coefficients
from .steppers import arnoldi, faber_step, faber_terms, krylov_step


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


def arnoldi_mgs(matvec, x, k, breakdown=1e-14):
    """Arnoldi with modified Gram-Schmidt for the matrix of matvec started
    from x: (beta, basis list, (k+1) x k Hessenberg matrix, k_eff), with the
    breakdown rule of the forward Krylov step."""
    beta = float(np.linalg.norm(x))
    Hm = np.zeros((k + 1, k))
    if beta == 0.0:
        return beta, [], Hm, 0
    Q = [x / beta]
    k_eff = k
    for j in range(k):
        w = matvec(Q[j])
        for i in range(j + 1):
            Hm[i, j] = float(np.dot(w, Q[i]))
            w = w - Hm[i, j] * Q[i]
        Hm[j + 1, j] = float(np.linalg.norm(w))
        if Hm[j + 1, j] <= breakdown * beta:
            k_eff = j + 1
            break
        Q.append(w / Hm[j + 1, j])
    return beta, Q, Hm, k_eff


def van_loan(A1, B, A2):
    """(exp(A1), int_0^1 exp((1-s) A1) B exp(s A2) ds): the diagonal and
    upper right blocks of the exponential of [[A1, B], [0, A2]]."""
    n1, n2 = A1.shape[0], A2.shape[0]
    Z = np.zeros((n1 + n2, n1 + n2))
    Z[:n1, :n1] = A1
    Z[:n1, n1:] = B
    Z[n1:, n1:] = A2
    E = expm(Z)
    return E[:n1, :n1], E[:n1, n1:]


def krylov_adjoint_step(prob, U, lam, t, dt, k, p=8):
    """(lam', grad) for the Krylov step of dimension k from t (the reading in
    the module docstring): lam' ~ exp(dt H^T) lam, grad[x] ~ d<lam, step(U)>/dc^2[x]."""
    g = prob.grid
    G = prob.src.w_columns(t, p) if prob.src is not None else None
    x = np.concatenate([U, e_p(p)]) if prob.src is not None else np.array(U, dtype=np.float64)
    beta, V, Hm, kv = arnoldi(prob, x, G, k)
    beta_l, W, Gm, kw = arnoldi_mgs(lambda y: apply_HT(g, prob.c2, y), np.array(lam, dtype=np.float64), k)
    lam_new = np.zeros(g.nstate)
    grad = np.zeros(g.npts)
    if kw == 0:
        return lam_new, grad
    if kv == 0:
        E1 = expm(dt * Gm[:kw, :kw])
    else:
        B = np.zeros((kw, kv))
        B[0, 0] = 1.0
        E1, F = van_loan(dt * Gm[:kw, :kw], B, dt * Hm[:kv, :kv].T)
        C = beta * beta_l * F
        divs = [divergence_of_velocity(g, V[b][: g.nstate]) for b in range(kv)]
        for a_ in range(kw):
            for b in range(kv):
                grad -= dt * C[a_, b] * W[a_][: g.npts] * divs[b]
    for a_ in range(kw):
        lam_new += beta_l * E1[a_, 0] * W[a_]
    return lam_new, grad


def krylov_misfit(prob, U0, t0, dt, nsteps, k, receivers, d_obs, p=8):
    """L = 1/2 sum_n |u_{n+1}[rec] - d_obs[n]|^2 over nsteps Krylov steps."""
    U = np.array(U0, dtype=np.float64)
    L = 0.0
    for n in range(nsteps):
        U = krylov_step(prob, U, t0 + n * dt, dt, k, p)
        r = U[receivers] - d_obs[n]
        L += 0.5 * float(r @ r)
    return L


def krylov_misfit_gradient(prob, U0, t0, dt, nsteps, k, receivers, d_obs, p=8):
    """(L, dL/dc^2, dL/dU0) of the Krylov misfit, each step reversed by
    krylov_adjoint_step (all states kept: small cases)."""
    g = prob.grid
    states = [np.array(U0, dtype=np.float64)]
    for n in range(nsteps):
        states.append(krylov_step(prob, states[-1], t0 + n * dt, dt, k, p))
    L = 0.0
    lam = np.zeros(g.nstate)
    grad = np.zeros(g.npts)
    for n in range(nsteps - 1, -1, -1):
        r = states[n + 1][receivers] - d_obs[n]
        L += 0.5 * float(r @ r)
        np.add.at(lam, receivers, r)
        lam, gn = krylov_adjoint_step(prob, states[n], lam, t0 + n * dt, dt, k, p)
        grad += gn
    return L, grad, lam
