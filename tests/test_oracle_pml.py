"""Pins of the PML oracle (the paper's own spatial operator, Sec. 2-2.2 and the
appendix on the free surface) against closed forms and independent routes."""
from fractions import Fraction as Fr

import numpy as np
import pytest
from scipy.linalg import expm

from oracle import pml
from oracle.operator import staggered_weights
from oracle.spectrum import ellipse_from_rectangle
from oracle.steppers import faber_step


def test_fornberg_textbook_weights():
    # central differences on three equispaced nodes: (-1/2, 0, 1/2) and (1, -2, 1)
    c = pml.fornberg_weights(Fr(0), [Fr(-1), Fr(0), Fr(1)], 2)
    assert c[1] == [Fr(-1, 2), Fr(0), Fr(1, 2)]
    assert c[2] == [Fr(1), Fr(-2), Fr(1)]
    # one-sided first derivative on 0, 1, 2: (-3/2, 2, -1/2)
    c = pml.fornberg_weights(Fr(0), [Fr(0), Fr(1), Fr(2)], 1)
    assert c[1] == [Fr(-3, 2), Fr(2), Fr(-1, 2)]


def test_fornberg_reproduces_the_papers_staggered_weights():
    # Sec. 2.1: on the half points -7/2..7/2 Fornberg's recursion gives the
    # printed 1225/1024 (1, -1/15, 1/125, -1/1715), antisymmetric
    nodes = [Fr(2 * k - 1, 2) for k in range(-3, 5)]
    c = pml.fornberg_weights(Fr(0), nodes, 1)[1]
    expect = [Fr(1225, 1024) * w for w in (Fr(1), Fr(-1, 15), Fr(1, 125), Fr(-1, 1715))]
    assert c[4:] == expect
    assert c[:4] == [-w for w in reversed(expect)]
    assert np.allclose([float(w) for w in expect], staggered_weights(8), rtol=0, atol=1e-16)


def _d2(f):
    return pml.D2_CENTER * f[4] + sum(pml.D2_WEIGHTS[l - 1] * (f[4 + l] + f[4 - l]) for l in range(1, 5))


def test_second_derivative_read_with_sums_is_exact_to_degree_9():
    x = np.arange(-4, 5, dtype=float) + 0.3
    for k in range(10):
        exact = k * (k - 1) * 0.3 ** (k - 2) if k >= 2 else 0.0
        assert abs(_d2(x ** k) - exact) <= 1e-9 * max(1.0, abs(exact))
    assert abs(_d2(x ** 10) - 90 * 0.3 ** 8) > 1.0
    # the printed form (differences) is not consistent: it does not even
    # annihilate constants
    ones = np.ones(9)
    printed = pml.D2_CENTER + sum(pml.D2_WEIGHTS[l - 1] * (ones[4 + l] - ones[4 - l]) for l in range(1, 5))
    assert abs(printed) > 1.0


@pytest.mark.parametrize("k", range(11))
def test_surface_stencils_exact_on_polynomials_with_zero_slope(k):
    # appendix: u_i = u(-i h); d_yy rows exact to degree 9, d_y rows to degree
    # 8, for every monomial except the linear one (they build in u_y(0) = 0)
    for j, row in enumerate(pml.SURFACE_D2):
        val = sum(cf * Fr(-i) ** k for i, cf in enumerate(row))
        exact = k * (k - 1) * Fr(-j) ** (k - 2) if k >= 2 else 0
        assert (val == exact) == (k != 1 and k <= 9)
    for j, row in enumerate(pml.SURFACE_D1):
        val = sum(cf * Fr(-i) ** k for i, cf in enumerate(row))
        exact = k * Fr(-(2 * j + 1), 2) ** (k - 1) if k >= 1 else 0
        assert (val == exact) == (k != 1 and k <= 8)


@pytest.mark.parametrize("k", range(1, 11))
def test_surface_dw_weights_exact_for_functions_vanishing_at_the_surface(k):
    for j, row in enumerate(pml.surface_dw_weights()):
        val = sum(cf * Fr(-(2 * i + 1), 2) ** k for i, cf in enumerate(row))
        assert (val == k * Fr(-j) ** (k - 1)) == (k <= 8)


def _grid_fields(g):
    ny, nx = g.shape
    x = (np.arange(nx) - nx / 2) * g.h
    xh = (np.arange(nx) + 0.5 - nx / 2) * g.h
    y = -np.arange(ny) * g.h
    yh = -(np.arange(ny) + 0.5) * g.h
    return x, xh, y, yh


def _poly(cs, t):
    return sum(c * t ** i for i, c in enumerate(cs))


def _dpoly(cs, t, d=1):
    p = np.polynomial.polynomial.polyder(np.array(cs, dtype=float), d)
    return _poly(p, t)


def test_operator_exact_on_polynomial_fields_including_the_surface_rows():
    """H on u = P(x) Q(y) with Q'(0) = 0, and on w_x, w_y fields with w_y(0) = 0,
    equals the continuous operator at every node whose stencils stay inside the
    domain along x and above the bottom (the surface rows included)."""
    g = pml.PMLGrid(24, 20, 1.0, abc_cells=6, beta0=0.7)
    ny, nx = g.shape
    x, xh, y, yh = _grid_fields(g)
    P = [0.3, -0.2, 0.05, 0.01, -0.002, 1e-4]               # degree 5 in x
    Q = [1.0, 0.0, -0.04, 0.003, 2e-4, -1e-5, 3e-7]         # Q'(0) = 0, degree 6
    R = [0.5, 0.1, -0.03, 0.002]                            # w_x(x)
    G = [0.0, 0.2, -0.01, 1e-3, -2e-5, 1e-6]                # w_y, G(0) = 0
    c2 = np.full(g.shape, 2.25)
    u = np.outer(_poly(Q, y), _poly(P, x))
    v = np.outer(np.cos(y), np.sin(x))
    wx = np.outer(_poly(Q, y), _poly(R, xh))
    wy = np.outer(_poly(G, yh), _poly(P, x))
    HU = pml.split(g, pml.apply_H_pml(g, c2, np.concatenate([f.ravel() for f in (u, v, wx, wy)])))
    bx, bxh, by, byh = pml.betas(g)
    BX, BXH, BY, BYH = bx[None, :], bxh[None, :], by[:, None], byh[:, None]
    lap = np.outer(_poly(Q, y), _dpoly(P, x, 2)) + np.outer(_dpoly(Q, y, 2), _poly(P, x))
    dwx = np.outer(_poly(Q, y), _dpoly(R, x))
    dwy = np.outer(_dpoly(G, y), _poly(P, x))
    hv = -BX * BY * u + c2 * lap - (BX + BY) * v + c2 * (dwx + dwy)
    hwx = (BY - BXH) * np.outer(_poly(Q, y), _dpoly(P, xh)) - BXH * wx
    hwy = (BX - BYH) * np.outer(_dpoly(Q, yh), _poly(P, x)) - BYH * wy
    ins = (slice(0, ny - 5), slice(5, nx - 5))
    assert np.array_equal(HU[0], v)
    for got, want in ((HU[1], hv), (HU[2], hwx), (HU[3], hwy)):
        assert np.max(np.abs(got[ins] - want[ins])) <= 1e-11 * np.max(np.abs(want[ins]))


def test_operator_has_no_layer_at_the_top_and_zero_values_elsewhere():
    g = pml.PMLGrid(20, 16, 10.0, abc_cells=5, beta0=200.0)
    bx, bxh, by, byh = pml.betas(g)
    assert by[0] == 0.0 and by[-1] == 200.0 and byh[-1] == 200.0
    assert bx[0] == bx[-1] == 200.0 and np.all(bx[5:15] == 0.0)
    # a single nonzero u at a corner node reaches only nodes within 4 cells
    U = np.zeros(g.nstate)
    U[0] = 1.0
    hv = pml.split(g, pml.apply_H_pml(g, np.ones(g.shape), U))[1]
    nz = np.argwhere(hv != 0.0)
    assert nz[:, 0].max() <= 8 and nz[:, 1].max() <= 4


def _ellipse_contains(gamma, c0, c1, lam, tol=1e-9):
    a = gamma * abs(1 + c1)
    b = gamma * abs(1 - c1)
    re = lam.real - gamma * c0
    if a == 0.0:
        return np.all(np.abs(lam.real) <= tol * b) and np.all(np.abs(lam.imag) <= b * (1 + tol))
    return np.all((re / a) ** 2 + (lam.imag / b) ** 2 <= 1 + tol)


@pytest.mark.parametrize("cells,beta0,medium", [(0, 0.0, "const"), (4, 150.0, "const"),
                                                (4, 150.0, "layered"), (4, 300.0, "surface_fast")])
def test_spectrum_rectangle_reading_encloses_dense_eigenvalues(cells, beta0, medium):
    """The reading of the spectrum bound: every eigenvalue of the dense operator
    lies inside the Faber ellipse built from it (small grids)."""
    g = pml.PMLGrid(16, 12, 10.0, abc_cells=cells, beta0=beta0)
    ny, nx = g.shape
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    c = {"const": np.full(g.shape, 2500.0), "layered": 1500.0 + 150.0 * y,
         "surface_fast": 3500.0 - 150.0 * y}[medium]
    lam = np.linalg.eigvals(pml.assemble_H_pml(g, c ** 2))
    x_lo, B = pml.spectrum_rectangle_pml(g, c ** 2)
    assert _ellipse_contains(*ellipse_from_rectangle(x_lo, B), lam)
    if medium != "layered":
        # with the fastest medium at the surface the margin is needed: the
        # interior symbol bound alone is exceeded
        assert np.max(np.abs(lam.imag)) > B / pml.SURFACE_MARGIN


def _small_problem(src):
    g = pml.PMLGrid(14, 11, 10.0, abc_cells=3, beta0=120.0)
    ny, nx = g.shape
    c = 1800.0 + 60.0 * np.arange(ny)[:, None] * np.ones((1, nx))
    rng = np.random.default_rng(11)
    U = rng.standard_normal(g.nstate) * 1e-3
    s = pml.PMLSources((5 * nx + 7,), (2.0,), 25.0, 0.04) if src else None
    return pml.PMLProblem(g, c ** 2, s), U


def test_faber_on_the_pml_operator_matches_the_dense_exponential():
    prob, U = _small_problem(src=False)
    H = pml.assemble_H_pml(prob.grid, prob.c2)
    dt = 2e-3
    got = faber_step(prob, U, 0.0, dt, 40)
    want = expm(dt * H) @ U
    assert np.linalg.norm(got - want) <= 1e-10 * np.linalg.norm(want)


def test_faber_with_source_matches_the_dense_augmented_exponential():
    """Sec. 3.2, augmented matrix: the source enters the v equation; the
    exponential of [[H, W], [0, J]] applied to [U; e_p] is the reference."""
    from oracle.source import e_p
    prob, U = _small_problem(src=True)
    p, t0, dt = 6, 0.03, 2e-3
    n = prob.grid.nstate
    H = pml.assemble_H_pml(prob.grid, prob.c2)
    G = prob.src.w_columns(t0, p)
    W = np.zeros((n, p))
    for node, st in zip(prob.src.nodes, prob.src.strengths(prob.grid)):
        assert node >= prob.grid.npts  # a v-field entry
        W[node] += st * G
    J = np.eye(p, k=1)
    Ht = np.block([[H, W], [np.zeros((p, n)), J]])
    want = (expm(dt * Ht) @ np.concatenate([U, e_p(p)]))[:n]
    got = faber_step(prob, U, t0, dt, 40, p)
    assert np.linalg.norm(got - want) <= 1e-10 * np.linalg.norm(want)
