"""Pins of the oracle's Faber coefficients and Faber step (CPU only)."""
import numpy as np
import pytest

from oracle.exact import ExactPropagator, plane_wave
from oracle.operator import Grid
from oracle.source import PointSources
from oracle.spectrum import (ellipse_from_rectangle, faber_coefficients,
                             faber_coefficients_contour, faber_polynomials_scalar,
                             faber_series_scalar, psi, spectrum_rectangle)
from oracle.steppers import Problem, faber_step, run
from synthetic import layered_velocity, smooth_state


ELLIPSES = [(678.8, -0.442, -0.375), (1262.1, -0.2377, -0.6639), (50.0, 0.3, 0.4), (10.0, -0.1, 0.0)]


@pytest.mark.parametrize("ell", ELLIPSES)
@pytest.mark.parametrize("dt", [1e-3, 4e-3, 1e-2])
def test_bessel_coefficients_equal_contour_integral(ell, dt):
    """Closed-form (Bessel) coefficients = trapezoidal Laurent coefficients."""
    a = faber_coefficients(*ell, dt, 40)
    b = faber_coefficients_contour(*ell, dt, 40, M=2048)
    scale = np.max(np.abs(np.exp(dt * psi(np.exp(1j * np.linspace(0, 2 * np.pi, 64)), *ell))))
    assert np.max(np.abs(a - b)) <= 1e-14 * max(1.0, scale)


@pytest.mark.parametrize("ell", ELLIPSES)
def test_faber_polynomials_on_ellipse_are_laurent_monomials(ell):
    gamma, c0, c1 = ell
    rng = np.random.default_rng(0)
    w = np.exp(1j * rng.uniform(0, 2 * np.pi, 7)) * rng.uniform(0.8, 1.5, 7)
    F = faber_polynomials_scalar(psi(w, *ell), gamma, c0, c1, 12)
    assert np.allclose(F[0], 1.0)
    for j in range(1, 13):
        assert np.allclose(F[j], w ** j + (c1 / w) ** j, rtol=1e-10, atol=1e-10)


def test_faber_with_c1_zero_is_taylor_about_centre():
    """c1 = 0: the ellipse is a disc and the series is Taylor about gamma c0."""
    gamma, c0, dt = 40.0, -0.5, 0.01
    z = gamma * c0 + 3.0 + 2.0j
    approx = faber_series_scalar(z, gamma, c0, 0.0, dt, 30)
    assert abs(approx - np.exp(dt * z)) < 1e-14


def test_faber_with_symmetric_segment_is_jacobi_anger():
    """c0 = 0, c1 = -1: psi(e^{i t}) = 2 i gamma sin t and the coefficients are J_j(2 gamma dt)."""
    from scipy.special import jv
    gamma, dt = 100.0, 0.02
    a = faber_coefficients(gamma, 0.0, -1.0, dt, 30)
    assert np.allclose(a, jv(np.arange(31), 2 * gamma * dt), atol=1e-16)
    y = 0.7 * 2 * gamma
    assert abs(faber_series_scalar(1j * y, gamma, 0.0, -1.0, dt, 30) - np.exp(1j * y * dt)) < 1e-12


@pytest.mark.parametrize("ell", ELLIPSES[:3])
def test_faber_series_converges_to_exponential_inside_ellipse(ell):
    gamma, c0, c1 = ell
    dt = 2.0 / gamma
    th = np.linspace(0, 2 * np.pi, 17)
    z = psi(0.999 * np.exp(1j * th), *ell)          # on (just inside) the ellipse
    prev = None
    for m in (10, 20, 30):
        err = np.max(np.abs(faber_series_scalar(z, gamma, c0, c1, dt, m) - np.exp(dt * z)))
        if prev is not None:
            assert err < prev or err < 1e-13
        prev = err
    assert prev < 1e-10


def _small_problem(with_source=True, n=(12, 10)):
    g = Grid(n, 10.0, 4, abc_cells=3, sigma_max=300.0)
    c2 = layered_velocity(n, 10.0, seed=11) ** 2
    src = PointSources((g.npts // 2 + 3,), (1.0,), 15.0, 0.05) if with_source else None
    return Problem(g, c2, src)


def test_faber_step_matches_variation_of_constants():
    """One Faber step (augmented source) equals expm + Duhamel quadrature."""
    prob = _small_problem()
    U0 = smooth_state(prob.grid.n, seed=1, width_cells=2.0)
    ex = ExactPropagator(prob, nquad=30)
    for t in (0.03, 0.05):
        Ue = ex.step(U0, t, 1e-3)
        Uf = faber_step(prob, U0, t, 1e-3, 24, p=12)
        assert np.linalg.norm(Uf - Ue) <= 1e-12 * np.linalg.norm(Ue)


def test_faber_truncation_error_falls_with_degree():
    prob = _small_problem(with_source=False)
    U0 = smooth_state(prob.grid.n, seed=2, width_cells=2.0)
    Ue = ExactPropagator(prob).step(U0, 0.0, 4e-3)
    errs = [np.linalg.norm(faber_step(prob, U0, 0.0, 4e-3, m) - Ue) for m in (8, 16, 24, 32)]
    assert all(errs[i + 1] < errs[i] for i in range(3))
    assert errs[-1] < 1e-12 * np.linalg.norm(Ue)


def test_faber_run_on_homogeneous_101_matches_exact_one_step():
    """The 101x101 homogeneous case: one 4 ms step of degree 16 from a smooth state."""
    g = Grid((101, 101), 10.0, 4, abc_cells=20, sigma_max=300.0)
    c2 = np.full(g.shape, 2000.0 ** 2)
    prob = Problem(g, c2, None)
    gamma, c0, c1 = prob.ellipse()
    assert np.isclose(gamma, 678.8, atol=0.05) and np.isclose(c1, -0.375, atol=1e-3)
    U0 = smooth_state(g.n, seed=3)
    Ue = ExactPropagator(prob).step(U0, 0.0, 4e-3)
    Uf = faber_step(prob, U0, 0.0, 4e-3, 16)
    # degree 16 truncation at gamma*dt = 2.7: well below the 1e-5 accuracy target
    assert np.linalg.norm(Uf - Ue) <= 1e-7 * np.linalg.norm(Ue)
    Uf30 = faber_step(prob, U0, 0.0, 4e-3, 30)
    assert np.linalg.norm(Uf30 - Ue) <= 1e-12 * np.linalg.norm(Ue)


@pytest.mark.parametrize("m", [3, 4, 6])
def test_faber_global_order_in_dt(m):
    """Fixed degree m: the global error falls like dt^m as dt -> 0."""
    prob = _small_problem(with_source=False, n=(10, 9))
    U0 = smooth_state(prob.grid.n, seed=4, width_cells=2.0)
    T = 2e-3
    ex = ExactPropagator(prob)
    Ue = ex.step(U0, 0.0, T)
    errs = []
    for ns in (8, 16):
        dt = T / ns
        U, _, _ = run(prob, "faber", U0, 0.0, dt, ns, m=m)
        errs.append(np.linalg.norm(U - Ue))
    rate = np.log2(errs[0] / errs[1])
    assert rate > m - 0.6


def test_faber_amplification_of_periodic_plane_wave():
    """A periodic plane wave is multiplied by sum_j a_j F_j(+-i omega) each step."""
    g = Grid((20, 16), 10.0, 4, bc="periodic")
    c = 2000.0
    c2 = np.full(g.shape, c * c)
    prob = Problem(g, c2, None)
    gamma, c0, c1 = ellipse_from_rectangle(*spectrum_rectangle(g, c2))
    U0, omega = plane_wave(g, c, (2, 3), 0.0)
    dt, m = 3e-3, 16
    U1 = faber_step(prob, U0, 0.0, dt, m, ellipse=(gamma, c0, c1))
    G = faber_series_scalar(1j * omega, gamma, c0, c1, dt, m)
    # cos(theta - omega t) is the real part of the eigenmode of eigenvalue -i omega, so one
    # step maps it to Re(conj(G) e^{i theta}) = |G| cos(theta - arg G): the closed form at
    # t = arg(G)/omega scaled by |G| (G has real coefficients, G(-i w) = conj G(i w))
    Ushift, _ = plane_wave(g, c, (2, 3), np.angle(G) / omega)
    assert np.max(np.abs(U1 - abs(G) * Ushift)) < 1e-12
    assert abs(G - np.exp(1j * omega * dt)) < 1e-9


def test_augmented_source_run_matches_duhamel_over_many_steps():
    prob = _small_problem()
    U0 = np.zeros(prob.grid.nstate)
    dt, ns = 2e-3, 30
    Uf, _, _ = run(prob, "faber", U0, 0.0, dt, ns, m=24, p=12)
    Ue = ExactPropagator(prob, nquad=30).run(U0, 0.0, dt, ns)
    assert np.linalg.norm(Uf - Ue) <= 1e-10 * np.linalg.norm(Ue)


def test_dense_output_at_zero_and_full_step():
    """Dense output from one set of terms: tau = 0 gives the state itself,
    tau = dt gives the Faber step (computed separately by faber_step)."""
    from oracle.steppers import faber_dense
    prob = _small_problem()
    U0 = smooth_state(prob.grid.n, seed=3, width_cells=2.0)
    nodes = np.arange(0, prob.grid.npts, 7)
    dt, m = 2e-3, 20
    d = faber_dense(prob, U0, 0.04, m, [0.0, dt], nodes, p=12)
    assert np.array_equal(d[0], U0[nodes])
    Uf = faber_step(prob, U0, 0.04, dt, m, p=12)
    assert np.linalg.norm(d[1] - Uf[nodes]) <= 1e-13 * np.linalg.norm(Uf[nodes])


def test_dense_output_between_steps_matches_variation_of_constants():
    """At intermediate tau the same terms reproduce exp(tau H) with the source
    (expm + Duhamel quadrature), i.e. the solution between two steps."""
    from oracle.steppers import faber_dense
    prob = _small_problem()
    U0 = smooth_state(prob.grid.n, seed=4, width_cells=2.0)
    nodes = np.arange(3, prob.grid.npts, 5)
    ex = ExactPropagator(prob, nquad=30)
    taus = [2.5e-4, 1e-3, 1.7e-3]
    d = faber_dense(prob, U0, 0.05, 28, taus, nodes, p=12)
    for i, tau in enumerate(taus):
        Ue = ex.step(U0, 0.05, tau)[nodes]
        assert np.linalg.norm(d[i] - Ue) <= 1e-11 * np.linalg.norm(Ue)
