"""Pins of the oracle adjoint: an independently assembled transpose, the
dot-product test, and finite differences of the misfit."""
import numpy as np
import pytest

from oracle.adjoint import apply_HT, faber_adjoint_step, misfit, misfit_gradient
from oracle.operator import Grid, apply_H, assemble_H
from oracle.source import PointSources
from oracle.steppers import Problem, faber_step
from synthetic import layered_velocity, smooth_state


def _problem(n=(11, 9), source=True, abc=3):
    g = Grid(n, 10.0, 4, abc_cells=abc, sigma_max=300.0 if abc else 0.0)
    c2 = layered_velocity(n, 10.0, seed=5) ** 2
    src = PointSources((g.npts // 2 + 2,), (1.0,), 15.0, 0.05) if source else None
    return Problem(g, c2, src)


@pytest.mark.parametrize("n", [(11, 9), (6, 5, 4)])
def test_HT_is_the_assembled_transpose(n):
    prob = _problem(n, source=False)
    Y = smooth_state(n, seed=3, width_cells=2.0)
    Hs = assemble_H(prob.grid, prob.c2)
    assert np.allclose(apply_HT(prob.grid, prob.c2, Y), Hs.T @ Y, rtol=0, atol=1e-9 * np.abs(Hs.T @ Y).max())


def test_HT_dot_product():
    prob = _problem(source=False)
    x = smooth_state(prob.grid.n, seed=1, width_cells=2.0)
    y = smooth_state(prob.grid.n, seed=2, width_cells=2.0)
    lhs = apply_H(prob.grid, prob.c2, x) @ y
    rhs = x @ apply_HT(prob.grid, prob.c2, y)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("m", [1, 2, 3, 12])
def test_adjoint_step_dot_product(m):
    """Without a source the step is linear: <P(H) u, lam> = <u, P(H)^T lam>."""
    prob = _problem(source=False)
    u = smooth_state(prob.grid.n, seed=4, width_cells=2.0)
    lam = smooth_state(prob.grid.n, seed=5, width_cells=2.0)
    ell = prob.ellipse()
    lhs = faber_step(prob, u, 0.0, 2e-3, m, ellipse=ell) @ lam
    mu0, _ = faber_adjoint_step(prob, u, lam, 0.0, 2e-3, m, ellipse=ell)
    assert abs(lhs - u @ mu0) <= 1e-12 * np.linalg.norm(lam) * np.linalg.norm(u) * 10


def test_gradient_matches_finite_differences():
    """dL/dc^2 of the receiver misfit (with source, 4 steps) against central
    differences along random directions, with the ellipse held fixed."""
    prob = _problem()
    g = prob.grid
    ell = prob.ellipse()
    rng = np.random.default_rng(9)
    rec = np.array([3, 17, 40, 77, 90])
    U0 = 1e-3 * smooth_state(g.n, seed=6, width_cells=2.0)
    nst, dt, m, t0 = 4, 2e-3, 10, 0.04
    d_obs = rng.normal(size=(nst, rec.size)) * 1e-4
    L, grad, _ = misfit_gradient(prob, U0, t0, dt, nst, m, rec, d_obs, ellipse=ell)
    assert L == pytest.approx(misfit(prob, U0, t0, dt, nst, m, rec, d_obs, ellipse=ell), rel=1e-13)
    for k in range(3):
        d = rng.normal(size=g.npts) * prob.c2.ravel() * 1e-3
        eps = 1e-3
        pp = Problem(g, prob.c2 + eps * d.reshape(g.shape), prob.src)
        pm = Problem(g, prob.c2 - eps * d.reshape(g.shape), prob.src)
        fd = (misfit(pp, U0, t0, dt, nst, m, rec, d_obs, ellipse=ell)
              - misfit(pm, U0, t0, dt, nst, m, rec, d_obs, ellipse=ell)) / (2 * eps)
        assert grad @ d == pytest.approx(fd, rel=1e-6)


def test_gradient_with_respect_to_initial_state():
    """dL/dU0 from the same reverse sweep, against finite differences."""
    prob = _problem()
    g = prob.grid
    ell = prob.ellipse()
    rng = np.random.default_rng(10)
    rec = np.array([5, 33, 61])
    U0 = 1e-3 * smooth_state(g.n, seed=7, width_cells=2.0)
    nst, dt, m = 3, 2e-3, 8
    d_obs = rng.normal(size=(nst, rec.size)) * 1e-4
    _, _, gU = misfit_gradient(prob, U0, 0.0, dt, nst, m, rec, d_obs, ellipse=ell)
    d = rng.normal(size=g.nstate) * 1e-3
    eps = 1e-4
    fd = (misfit(prob, U0 + eps * d, 0.0, dt, nst, m, rec, d_obs, ellipse=ell)
          - misfit(prob, U0 - eps * d, 0.0, dt, nst, m, rec, d_obs, ellipse=ell)) / (2 * eps)
    assert gU @ d == pytest.approx(fd, rel=1e-7)


# --- Krylov adjoint (reading: the derivatives of the exponential, each factor
# approximated in a Krylov space of dimension k) ---

from scipy.integrate import quad_vec  # noqa: E402
from scipy.linalg import expm, expm_frechet  # noqa: E402

from oracle.adjoint import (krylov_adjoint_step, krylov_misfit, krylov_misfit_gradient,  # noqa: E402
                            van_loan)
from oracle.steppers import apply_Htilde, krylov_step  # noqa: E402


def test_van_loan_is_the_integral():
    rng = np.random.default_rng(11)
    A1, B, A2 = rng.normal(size=(3, 3)), rng.normal(size=(3, 4)), rng.normal(size=(4, 4))
    E1, F = van_loan(A1, B, A2)
    ref, _ = quad_vec(lambda s: expm((1 - s) * A1) @ B @ expm(s * A2), 0.0, 1.0, epsabs=1e-13, epsrel=1e-13)
    assert np.allclose(E1, expm(A1), rtol=1e-13, atol=1e-13)
    assert np.allclose(F, ref, rtol=1e-11, atol=1e-12)


def _dense(prob, G, n):
    return np.stack([apply_Htilde(prob, e, G) for e in np.eye(n)], axis=1)


def test_krylov_adjoint_state_is_the_transposed_exponential():
    """k past convergence: lam' = exp(dt H^T) lam (dense, assembled)."""
    prob = _problem((6, 5), source=False, abc=2)
    g = prob.grid
    lam = smooth_state(g.n, seed=12, width_cells=1.5)
    U = smooth_state(g.n, seed=13, width_cells=1.5)
    dt = 2e-3
    Hd = assemble_H(g, prob.c2).toarray()
    lam1, _ = krylov_adjoint_step(prob, U, lam, 0.0, dt, 40)
    ref = expm(dt * Hd.T) @ lam
    assert np.linalg.norm(lam1 - ref) <= 1e-12 * np.linalg.norm(ref)


def test_krylov_adjoint_gradient_is_the_frechet_derivative():
    """k past convergence, with a source (augmented matrix): grad[x] =
    <[lam; 0], L(dt H~, dt dH~/dc^2[x]) [U; e_p]>, L the Frechet derivative of
    the dense exponential."""
    prob = _problem((6, 5), source=True, abc=2)
    g = prob.grid
    p, t, dt = 4, 0.03, 2e-3
    G = prob.src.w_columns(t, p)
    n_aug = g.nstate + p
    lam = smooth_state(g.n, seed=14, width_cells=1.5)
    U = 1e-3 * smooth_state(g.n, seed=15, width_cells=1.5)
    x = np.concatenate([U, np.eye(p)[-1]])
    _, grad = krylov_adjoint_step(prob, U, lam, t, dt, 50, p=p)
    Hd = _dense(prob, G, n_aug)
    lam_aug = np.concatenate([lam, np.zeros(p)])
    ref = np.zeros(g.npts)
    for i in range(g.npts):
        c2i = prob.c2.copy().ravel()
        c2i[i] += 1.0
        Ei = _dense(Problem(g, c2i.reshape(g.shape), prob.src), G, n_aug) - Hd
        ref[i] = lam_aug @ (expm_frechet(dt * Hd, dt * Ei, compute_expm=False) @ x)
    assert np.linalg.norm(grad - ref) <= 1e-9 * np.linalg.norm(ref)


def test_krylov_adjoint_gradient_is_the_integral_of_the_krylov_outputs():
    """Small k (far from converged): grad = -dt int_0^1 lam(1-s)_p div u(s) ds
    with u(s) the forward Krylov output at step s dt (the basis does not
    depend on the step size) and lam(r) the adjoint output at r dt, by
    Gauss-Legendre quadrature (a path that does not use the block exponential)."""
    from oracle.adjoint import divergence_of_velocity
    prob = _problem((11, 9), source=True, abc=3)
    g = prob.grid
    p, t, dt, k = 4, 0.03, 4e-3, 6
    lam = smooth_state(g.n, seed=16, width_cells=2.0)
    U = 1e-3 * smooth_state(g.n, seed=17, width_cells=2.0)
    _, grad = krylov_adjoint_step(prob, U, lam, t, dt, k, p=p)
    xs, ws = np.polynomial.legendre.leggauss(24)
    s_nodes, s_w = 0.5 * (xs + 1.0), 0.5 * ws
    ref = np.zeros(g.npts)
    for s, wq in zip(s_nodes, s_w):
        u = krylov_step(prob, U, t, s * dt, k, p=p)
        lr, _ = krylov_adjoint_step(prob, U, lam, t, (1.0 - s) * dt, k, p=p)
        ref -= dt * wq * lr[: g.npts] * divergence_of_velocity(g, u)
    assert np.linalg.norm(grad - ref) <= 1e-11 * np.linalg.norm(ref)


def test_krylov_misfit_gradient_matches_finite_differences():
    """k past convergence (the Krylov step is then the exponential): the
    misfit gradient of three steps with a source against central differences."""
    prob = _problem((8, 7), source=True, abc=2)
    g = prob.grid
    rng = np.random.default_rng(18)
    rec = np.array([3, 17, 40])
    U0 = 1e-3 * smooth_state(g.n, seed=19, width_cells=1.5)
    nst, dt, k, t0, p = 3, 2e-3, 40, 0.04, 4
    d_obs = rng.normal(size=(nst, rec.size)) * 1e-4
    L, grad, gU = krylov_misfit_gradient(prob, U0, t0, dt, nst, k, rec, d_obs, p=p)
    assert L == pytest.approx(krylov_misfit(prob, U0, t0, dt, nst, k, rec, d_obs, p=p), rel=1e-13)
    d = rng.normal(size=g.npts) * prob.c2.ravel() * 1e-3
    eps = 1e-3
    pp = Problem(g, prob.c2 + eps * d.reshape(g.shape), prob.src)
    pm = Problem(g, prob.c2 - eps * d.reshape(g.shape), prob.src)
    fd = (krylov_misfit(pp, U0, t0, dt, nst, k, rec, d_obs, p=p)
          - krylov_misfit(pm, U0, t0, dt, nst, k, rec, d_obs, p=p)) / (2 * eps)
    assert grad @ d == pytest.approx(fd, rel=1e-6)
    dU = rng.normal(size=g.nstate) * 1e-3
    eps = 1e-4
    fdU = (krylov_misfit(prob, U0 + eps * dU, t0, dt, nst, k, rec, d_obs, p=p)
           - krylov_misfit(prob, U0 - eps * dU, t0, dt, nst, k, rec, d_obs, p=p)) / (2 * eps)
    assert gU @ dU == pytest.approx(fdU, rel=1e-6)
