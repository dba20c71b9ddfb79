"""Pins of the oracle's Krylov, Runge-Kutta and leap-frog steppers (CPU only)."""
from math import factorial

import numpy as np
import pytest
from scipy.linalg import expm

from oracle.exact import ExactPropagator, plane_wave, staggered_symbol
from oracle.operator import Grid, assemble_H, split_state
from oracle.source import PointSources, apply_J, e_p
from oracle.steppers import (Problem, apply_Htilde, arnoldi, hork_lambdas, hork_step,
                             krylov_step, leapfrog_step, rk32_step, rk4_step, run)
from synthetic import layered_velocity, smooth_state


def _problem(n=(10, 9), with_source=True, abc=3):
    g = Grid(n, 10.0, 4, abc_cells=abc, sigma_max=300.0 if abc else 0.0)
    c2 = layered_velocity(n, 10.0, seed=21) ** 2
    src = PointSources((g.npts // 2 + 2,), (1.0,), 15.0, 0.05) if with_source else None
    return Problem(g, c2, src)


# ---------------------------------------------------------------- Krylov

def test_krylov_step_matches_variation_of_constants():
    prob = _problem()
    U0 = smooth_state(prob.grid.n, seed=5, width_cells=2.0)
    ex = ExactPropagator(prob, nquad=30)
    Ue = ex.step(U0, 0.04, 1e-3)
    Uk = krylov_step(prob, U0, 0.04, 1e-3, 20, p=10)
    assert np.linalg.norm(Uk - Ue) <= 1e-11 * np.linalg.norm(Ue)


def test_arnoldi_relation_and_orthonormality():
    prob = _problem()
    U0 = smooth_state(prob.grid.n, seed=6, width_cells=2.0)
    G = prob.src.w_columns(0.04, 8)
    x = np.concatenate([U0, e_p(8)])
    beta, Q, Hm, k_eff = arnoldi(prob, x, G, 12)
    assert k_eff == 12
    Qm = np.array(Q).T                       # (n, k+1)
    HQ = np.array([apply_Htilde(prob, Q[j], G) for j in range(12)]).T
    assert np.linalg.norm(HQ - Qm @ Hm) <= 1e-12 * np.linalg.norm(HQ)
    assert np.max(np.abs(Qm.T @ Qm - np.eye(13))) < 1e-10
    assert np.allclose(np.triu(Hm, -1), Hm)          # upper Hessenberg
    assert np.isclose(beta, np.linalg.norm(x))


def test_krylov_exact_when_space_is_invariant():
    """With k = dim of the whole space the projection is exact (happy breakdown)."""
    g = Grid((3, 3), 10.0, 4, abc_cells=1, sigma_max=300.0)
    c2 = layered_velocity(g.n, 10.0, seed=2) ** 2
    prob = Problem(g, c2, None)
    U0 = smooth_state(g.n, seed=7, width_cells=1.0)
    Uk = krylov_step(prob, U0, 0.0, 5e-3, g.nstate)
    Ue = expm(5e-3 * assemble_H(g, c2).toarray()) @ U0
    assert np.linalg.norm(Uk - Ue) <= 1e-12 * np.linalg.norm(Ue)


def test_krylov_global_order():
    prob = _problem(with_source=False)
    U0 = smooth_state(prob.grid.n, seed=8, width_cells=2.0)
    T = 2e-3
    Ue = ExactPropagator(prob).step(U0, 0.0, T)
    errs = []
    for ns in (8, 16):
        U, _, _ = run(prob, "krylov", U0, 0.0, T / ns, ns, k=5)
        errs.append(np.linalg.norm(U - Ue))
    assert np.log2(errs[0] / errs[1]) > 3.5          # order k-1 = 4 asymptotically


def test_krylov_zero_state_without_source_stays_zero():
    prob = _problem(with_source=False)
    assert np.all(krylov_step(prob, np.zeros(prob.grid.nstate), 0.0, 1e-3, 5) == 0.0)


# ---------------------------------------------------------------- Runge-Kutta

def _taylor(Z, m):
    out = np.eye(Z.shape[0])
    term = np.eye(Z.shape[0])
    for j in range(1, m + 1):
        term = term @ Z / j
        out = out + term
    return out


def test_rk4_and_rk32_are_their_stability_polynomials():
    prob = _problem(n=(6, 5), with_source=False)
    Hd = assemble_H(prob.grid, prob.c2).toarray()
    U = smooth_state(prob.grid.n, seed=9, width_cells=1.5)
    dt = 7e-4
    Z = dt * Hd
    assert np.allclose(rk4_step(prob, U, 0.0, dt), _taylor(Z, 4) @ U, rtol=0, atol=1e-13)
    P32 = np.eye(len(U)) + Z + Z @ Z / 2 + Z @ Z @ Z / 4
    assert np.allclose(rk32_step(prob, U, 0.0, dt), P32 @ U, rtol=0, atol=1e-13)


@pytest.mark.parametrize("m", [2, 4, 7, 10])
def test_hork_is_taylor_of_order_m(m):
    lam = hork_lambdas(m)
    assert np.all(lam >= 0) and np.isclose(lam.sum(), 1.0)
    prob = _problem(n=(6, 5), with_source=False)
    Hd = assemble_H(prob.grid, prob.c2).toarray()
    U = smooth_state(prob.grid.n, seed=10, width_cells=1.5)
    dt = 5e-4
    assert np.allclose(hork_step(prob, U, 0.0, dt, m), _taylor(dt * Hd, m) @ U, rtol=0, atol=1e-12)


def test_rk4_global_order_four_with_source():
    prob = _problem()
    U0 = smooth_state(prob.grid.n, seed=11, width_cells=2.0)
    T = 4e-3
    Ue = ExactPropagator(prob, nquad=30).step(U0, 0.03, T)
    errs = []
    for ns in (16, 32):
        U, _, _ = run(prob, "rk4", U0, 0.03, T / ns, ns)
        errs.append(np.linalg.norm(U - Ue))
    assert abs(np.log2(errs[0] / errs[1]) - 4.0) < 0.3


# ---------------------------------------------------------------- leap-frog

def test_leapfrog_plane_wave_discrete_dispersion():
    """Periodic, homogeneous, undamped: exact discrete plane wave with
    sin(w dt / 2) = (dt / 2) c |K| (and v amplitudes K_a / (c |K|))."""
    g = Grid((20, 16), 10.0, 4, bc="periodic")
    c = 2000.0
    prob = Problem(g, np.full(g.shape, c * c), None)
    modes = (3, 2)
    kvec = [2 * np.pi * modes[a] / (g.n[a] * g.h) for a in range(2)]
    K = np.array([staggered_symbol(kvec[a], g.h, g.order) for a in range(2)])
    dt = 1.5e-3
    wt = 2.0 / dt * np.arcsin(0.5 * dt * c * np.linalg.norm(K))
    # the semi-discrete closed form, with omega replaced by the discrete frequency
    # (p at t_n, v at t_n - dt/2): evaluate both and splice
    def lf_state(n):
        Up, omega = plane_wave(g, c, modes, n * dt * wt / (c * np.linalg.norm(K)))
        Uv, _ = plane_wave(g, c, modes, (n - 0.5) * dt * wt / (c * np.linalg.norm(K)))
        f = split_state(g, Up)[:1] + split_state(g, Uv)[1:]
        return np.concatenate([x.ravel() for x in f])
    U = lf_state(0)
    for _ in range(25):
        U = leapfrog_step(prob, U, 0.0, dt)
    assert np.max(np.abs(U - lf_state(25))) < 1e-12


def test_leapfrog_stability_limit():
    """Undamped periodic grid: stable iff dt < 2 / omega_max."""
    g = Grid((16, 16), 10.0, 4, bc="periodic")
    c = 2000.0
    prob = Problem(g, np.full(g.shape, c * c), None)
    omega_max = c * np.sqrt(2) * (2 / g.h) * (9 / 8 + 1 / 24)   # reached at k h = pi on both axes
    U0 = smooth_state(g.n, seed=12, width_cells=1.0)
    U0 = U0 + 1e-3 * np.random.default_rng(0).standard_normal(g.nstate)
    for factor, stable in ((0.97, True), (1.03, False)):
        dt = factor * 2.0 / omega_max
        U, _, _ = run(prob, "leapfrog", U0, 0.0, dt, 600)
        nrm = np.linalg.norm(U)
        grew = (not np.isfinite(nrm)) or nrm > 1e3 * np.linalg.norm(U0)
        assert grew != stable


def test_leapfrog_second_order_with_damping_and_source():
    prob = _problem()
    U0 = np.zeros(prob.grid.nstate)
    T = 0.04
    Ue = ExactPropagator(prob, nquad=30).run(U0, 0.0, T / 4, 4)
    errs = []
    for ns in (80, 160):
        U, _, _ = run(prob, "leapfrog", U0, 0.0, T / ns, ns)
        errs.append(np.linalg.norm(split_state(prob.grid, U)[0] - split_state(prob.grid, Ue)[0]))
    assert abs(np.log2(errs[0] / errs[1]) - 2.0) < 0.3


# ------------------------------------------------- Krylov error estimate

def test_krylov_estimate_is_the_integrated_residual_of_the_projected_flow():
    """The estimate equals |int_0^dt (H~ u_k(s) - u_k'(s)) ds| for
    u_k(s) = beta V_k exp(s H_k) e_1, the integral by Gauss-Legendre
    quadrature of residuals formed with the operator itself (augmented
    vector, with a source)."""
    from oracle.steppers import krylov_step_estimate
    prob = _problem()
    p, t, dt, k = 8, 0.04, 2e-3, 6
    U0 = smooth_state(prob.grid.n, seed=8, width_cells=2.0)
    G = prob.src.w_columns(t, p)
    x = np.concatenate([U0, e_p(p)])
    beta, Q, Hm, k_eff = arnoldi(prob, x, G, k)
    assert k_eff == k
    Vk = np.array(Q[:k]).T
    xs, ws = np.polynomial.legendre.leggauss(20)
    integral = np.zeros_like(x)
    for xq, wq in zip(xs, ws):
        s_ = 0.5 * dt * (xq + 1.0)
        E = expm(s_ * Hm[:k, :k])[:, 0]
        u = beta * Vk @ E
        du = beta * Vk @ (Hm[:k, :k] @ E)
        integral += 0.5 * dt * wq * (apply_Htilde(prob, u, G) - du)
    U1, est = krylov_step_estimate(prob, U0, t, dt, k, p=p)
    assert est == pytest.approx(np.linalg.norm(integral), rel=1e-8)
    assert np.array_equal(U1, krylov_step(prob, U0, t, dt, k, p=p))


def test_krylov_estimate_tracks_the_error_and_vanishes_on_breakdown():
    """Against the dense exponential: the estimate falls with k and stays
    within a factor 2 of the true error while that is above rounding; it is
    at rounding level once the Krylov space is the whole space."""
    from oracle.steppers import krylov_step_estimate
    prob = _problem(with_source=False)
    U0 = smooth_state(prob.grid.n, seed=9, width_cells=2.0)
    for dt in (1e-3, 3e-3):
        Ue = expm(dt * assemble_H(prob.grid, prob.c2).toarray()) @ U0
        prev = np.inf
        for k in (2, 4, 6, 8, 10, 12):
            Uk, est = krylov_step_estimate(prob, U0, 0.0, dt, k)
            err = np.linalg.norm(Uk - Ue)
            assert est < prev
            prev = est
            if err > 1e-11 * np.linalg.norm(Ue):
                assert err / 2 <= est <= err * 2, (dt, k, est, err)
    g = Grid((3, 3), 10.0, 4, abc_cells=1, sigma_max=300.0)
    small = Problem(g, layered_velocity(g.n, 10.0, seed=2) ** 2, None)
    U0 = smooth_state(g.n, seed=7, width_cells=1.0)
    _, est = krylov_step_estimate(small, U0, 0.0, 5e-3, g.nstate + 2)
    assert est <= 1e-13 * np.linalg.norm(U0)
