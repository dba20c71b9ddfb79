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
