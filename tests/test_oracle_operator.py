"""Pins of the oracle's operator H (CPU only).

Each test checks the oracle against something other than itself: the paper's
printed weights, polynomial exactness, exact adjointness, an independently
assembled sparse matrix, energy conservation of the exact flow, the spectrum
bound, and the periodic plane-wave closed form.
"""
from fractions import Fraction
import os

import numpy as np
import pytest
from scipy.linalg import expm
from scipy.sparse.linalg import expm_multiply

from oracle.operator import (Grid, apply_H, assemble_H, d_minus, d_plus, damping_fields, damping_profile,
                             energy, split_state, staggered_weights)
from oracle.exact import plane_wave, staggered_symbol
from oracle.spectrum import ellipse_from_rectangle, spectrum_rectangle
from synthetic import layered_velocity


def test_order8_weights_match_paper(golden_dir):
    lines = [ln.strip() for ln in open(os.path.join(golden_dir, "staggered_weights_order8.txt"))
             if ln.strip() and not ln.startswith("#")]
    printed = np.array([float(Fraction(s)) for s in lines])
    assert np.allclose(staggered_weights(8), printed, rtol=0, atol=1e-16)


@pytest.mark.parametrize("order", [4, 8])
def test_staggered_derivative_polynomial_exactness(order):
    """D+ and D- are exact on polynomials of degree <= order (interior points).

    The stencils are centred on the output point, so the even-derivative error
    terms cancel and the first non-zero term involves the (order+1)-th derivative.
    """
    n, h = 20, 1.0
    K = order // 2
    x = (np.arange(n) - n / 2) * h
    xh = x + h / 2
    g = Grid((n, 1), h, order)
    interior = slice(K + 1, n - K - 1)

    def errs(deg):
        dfx = deg * x ** (deg - 1) if deg > 0 else np.zeros(n)
        dfh = deg * xh ** (deg - 1) if deg > 0 else np.zeros(n)
        dp = d_plus(g, (x ** deg)[None, :], 0)[0]
        dm = d_minus(g, (xh ** deg)[None, :], 0)[0]
        scale = max(1.0, np.max(np.abs(dfh)))
        return (np.max(np.abs(dp - dfh)[interior]) / scale,
                np.max(np.abs(dm - dfx)[interior]) / scale)

    for deg in range(order + 1):
        ep, em = errs(deg)
        assert ep < 1e-13 and em < 1e-13, deg
    ep, em = errs(order + 1)
    assert ep > 1e-9 and em > 1e-9


@pytest.mark.parametrize("order", [4, 8])
def test_staggered_derivative_convergence_rate(order):
    """Error of D+ on sin(x) falls by 2^order per halving of h."""
    errs = []
    for n in ((32, 64) if order == 4 else (12, 24)):
        h = 2 * np.pi / n
        g = Grid((n, 1), h, order, bc="periodic")
        x = np.arange(n) * h
        dp = d_plus(g, np.sin(x)[None, :], 0)[0]
        errs.append(np.max(np.abs(dp - np.cos(x + h / 2))))
    rate = np.log2(errs[0] / errs[1])
    assert abs(rate - order) < 0.2


@pytest.mark.parametrize("bc", ["zero", "periodic"])
@pytest.mark.parametrize("order", [4, 8])
def test_d_minus_is_minus_adjoint_of_d_plus(bc, order):
    rng = np.random.default_rng(1)
    g = Grid((13, 11), 7.0, order, bc=bc)
    for a in range(2):
        f = rng.standard_normal(g.shape)
        v = rng.standard_normal(g.shape)
        lhs = np.sum(d_plus(g, f, a) * v)
        rhs = -np.sum(f * d_minus(g, v, a))
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)


@pytest.mark.parametrize("n", [(9, 7), (6, 5, 7)])
@pytest.mark.parametrize("order", [4, 8])
@pytest.mark.parametrize("bc", ["zero", "periodic"])
def test_slicing_operator_equals_assembled_matrix(n, order, bc):
    rng = np.random.default_rng(2)
    g = Grid(n, 10.0, order, bc=bc, abc_cells=3 if bc == "zero" else 0,
             sigma_max=300.0 if bc == "zero" else 0.0)
    c2 = layered_velocity(n, 10.0, seed=7) ** 2
    U = rng.standard_normal(g.nstate)
    y1 = apply_H(g, c2, U)
    y2 = assemble_H(g, c2) @ U
    assert np.max(np.abs(y1 - y2)) <= 1e-13 * np.max(np.abs(y1))


def test_damping_profile_reading():
    n, h, L, smax = 30, 10.0, 5, 300.0
    s_int = damping_profile(n, h, L, smax, half=False)
    s_half = damping_profile(n, h, L, smax, half=True)
    assert s_int[0] == smax and s_int[-1] == smax
    assert np.all(s_int[L:n - L] == 0.0)
    # quadratic: at distance delta/2 from the edge -> sigma_max / 4
    g2 = damping_profile(n, h, 4, smax, half=False)
    assert np.isclose(g2[2], smax / 4)
    # half point i + 1/2: distance (i + 1/2) h from node 0
    assert np.isclose(s_half[0], smax * (1 - 0.5 / L) ** 2)
    # the last half point lies beyond the last node: distance clamped to 0
    assert s_half[-1] == smax
    assert np.isclose(s_half[-2], smax * (1 - 0.5 / L) ** 2)
    # symmetric about the centre for integer points
    assert np.allclose(s_int, s_int[::-1])


def test_weighted_skew_adjointness_without_damping():
    """For sigma = 0, W H + H^T W = 0 with W = diag(1/c^2, 1, ..., 1)."""
    g = Grid((8, 7), 10.0, 4)
    c2 = layered_velocity(g.n, 10.0, seed=3) ** 2
    Hd = assemble_H(g, c2).toarray()
    w = np.concatenate([1.0 / c2.ravel()] + [np.ones(g.npts)] * g.ndim)
    M = w[:, None] * Hd + (w[:, None] * Hd).T
    assert np.max(np.abs(M)) <= 1e-14 * np.max(np.abs(w[:, None] * Hd))


def test_energy_conserved_by_exact_flow_without_damping_and_decays_with_it():
    rng = np.random.default_rng(4)
    g0 = Grid((16, 14), 10.0, 4)
    c2 = layered_velocity(g0.n, 10.0, seed=5) ** 2
    U = rng.standard_normal(g0.nstate)
    E0 = energy(g0, c2, U)
    A = assemble_H(g0, c2)
    Ut = expm_multiply(0.02 * A, U)
    assert abs(energy(g0, c2, Ut) / E0 - 1.0) < 1e-12
    g1 = Grid((16, 14), 10.0, 4, abc_cells=4, sigma_max=300.0)
    A1 = assemble_H(g1, c2)
    Es = [energy(g1, c2, expm_multiply(t * A1, U)) for t in (0.0, 0.005, 0.01, 0.02)]
    assert all(Es[i + 1] < Es[i] for i in range(3))


@pytest.mark.parametrize("ndim", [2, 3])
def test_spectrum_inside_rectangle_and_ellipse(ndim):
    n = (11, 9) if ndim == 2 else (6, 5, 7)
    g = Grid(n, 10.0, 4, abc_cells=2, sigma_max=300.0)
    c2 = layered_velocity(n, 10.0, seed=6) ** 2
    lam = np.linalg.eigvals(assemble_H(g, c2).toarray())
    x_lo, B = spectrum_rectangle(g, c2)
    assert np.all(lam.real <= 1e-9) and np.all(lam.real >= x_lo - 1e-9)
    assert np.all(np.abs(lam.imag) <= B * (1 + 1e-12))
    gamma, c0, c1 = ellipse_from_rectangle(x_lo, B)
    xc, ar, bi = gamma * c0, gamma * (1 + c1), gamma * (1 - c1)
    assert np.all(((lam.real - xc) / ar) ** 2 + (lam.imag / bi) ** 2 <= 1 + 1e-9)


def test_ellipse_passes_through_rectangle_corners():
    x_lo, B = -600.0, 660.0
    gamma, c0, c1 = ellipse_from_rectangle(x_lo, B)
    xc, ar, bi = gamma * c0, gamma * (1 + c1), gamma * (1 - c1)
    for cx in (x_lo, 0.0):
        for cy in (-B, B):
            assert np.isclose(((cx - xc) / ar) ** 2 + (cy / bi) ** 2, 1.0)
    # minimum area among ellipses through the corners: perturbing the axis ratio grows the area
    area = ar * bi
    for s in (0.9, 1.1):
        a2 = ar * s
        b2 = B / np.sqrt(1 - (0.5 * x_lo / a2) ** 2)
        assert a2 * b2 > area


@pytest.mark.parametrize("order", [4, 8])
def test_plane_wave_closed_form_periodic(order):
    g = Grid((24, 20), 10.0, order, bc="periodic")
    c = 1800.0
    c2 = np.full(g.shape, c * c)
    U0, omega = plane_wave(g, c, (3, 2), 0.0)
    # H U equals the time derivative of the closed form
    dt = 1e-7
    Up, _ = plane_wave(g, c, (3, 2), dt)
    Um, _ = plane_wave(g, c, (3, 2), -dt)
    assert np.max(np.abs(apply_H(g, c2, U0) - (Up - Um) / (2 * dt))) < 1e-5 * omega
    # the exact flow reproduces the closed form at a later time
    T = 0.013
    UT, _ = plane_wave(g, c, (3, 2), T)
    Ue = expm_multiply(T * assemble_H(g, c2), U0)
    assert np.max(np.abs(Ue - UT)) < 1e-12
    # the symbol is the eigenvalue of D+ on e^{ikx}
    k = 2 * np.pi * 3 / (24 * 10.0)
    K = staggered_symbol(k, 10.0, order)
    assert np.isclose(K, k, rtol=0.05)


def test_dense_and_sparse_exponentials_agree_on_tiny_grid():
    g = Grid((6, 5), 10.0, 4, abc_cells=2, sigma_max=300.0)
    c2 = layered_velocity(g.n, 10.0, seed=8) ** 2
    A = assemble_H(g, c2)
    U = np.random.default_rng(9).standard_normal(g.nstate)
    assert np.allclose(expm(0.003 * A.toarray()) @ U, expm_multiply(0.003 * A, U), atol=1e-12)


def test_split_state_layout_is_field_major_x_fastest():
    g = Grid((5, 3), 1.0)
    U = np.arange(g.nstate, dtype=float)
    p, vx, vz = split_state(g, U)
    assert p[1, 2] == 1 * 5 + 2 and vx[0, 0] == 15 and vz[2, 4] == 30 + 2 * 5 + 4


def test_interior_mask_and_relative_error_metric():
    from oracle.operator import interior_mask, rel_l2_pressure
    g = Grid((30, 20), 10.0, abc_cells=5)
    m = interior_mask(g)
    assert m.sum() == (30 - 10) * (20 - 10)
    assert not m[4, 10] and m[5, 5] and m[14, 24] and not m[15, 24]
    rng = np.random.default_rng(0)
    U = rng.standard_normal(g.nstate)
    V = U.copy()
    V[: g.npts] *= 1.0 + 1e-6
    assert np.isclose(rel_l2_pressure(g, V, U, interior=False), 1e-6)


def _custom_profiles(n, seed):
    """Non-quadratic, non-symmetric damping profiles: a random non-negative
    ramp on one side of each axis plus a bump, different at the half points."""
    rng = np.random.default_rng(seed)
    out = []
    for na in n:
        for half in (0.0, 0.5):
            x = (np.arange(na) + half) / max(na - 1, 1)
            prof = 200.0 * rng.uniform(0.5, 1.0) * np.clip(1.0 - 3.0 * x, 0.0, None) ** 3
            prof += 50.0 * rng.uniform() * np.exp(-((x - rng.uniform()) / 0.1) ** 2)
            out.append(prof)
    return tuple(out)


@pytest.mark.parametrize("n", [(9, 7), (6, 5, 7)])
def test_custom_profiles_slicing_equals_assembled_matrix(n):
    """Caller-given profiles enter the slicing H and the independently
    assembled sparse H the same way; with the quadratic profile passed
    explicitly H is unchanged."""
    rng = np.random.default_rng(12)
    c2 = layered_velocity(n, 10.0, seed=13) ** 2
    g = Grid(n, 10.0, 4, profiles=_custom_profiles(n, 14))
    U = rng.standard_normal(g.nstate)
    y1 = apply_H(g, c2, U)
    assert np.max(np.abs(y1 - assemble_H(g, c2) @ U)) <= 1e-13 * np.max(np.abs(y1))
    gq = Grid(n, 10.0, 4, abc_cells=3, sigma_max=300.0)
    quad = tuple(damping_profile(n[a], 10.0, 3, 300.0, half) for a in range(len(n))
                 for half in (False, True))
    ge = Grid(n, 10.0, 4, profiles=quad)
    assert np.array_equal(apply_H(gq, c2, U), apply_H(ge, c2, U))
    # the profile values sit where the reading puts them: sigma_p sums the
    # axes' integer-point values, v_a takes axis a's half-point values
    sig_p, sig_v = damping_fields(g)
    prof = g.profiles
    node = tuple(rng.integers(0, v) for v in n)          # (i_x, i_y/z, ...)
    npi = tuple(reversed(node))
    assert np.isclose(sig_p[npi], sum(prof[2 * a][node[a]] for a in range(len(n))))
    for a in range(len(n)):
        assert sig_v[a][npi] == prof[2 * a + 1][node[a]]


def test_custom_profiles_energy_decays_and_spectrum_inside_ellipse():
    n = (12, 10)
    c2 = layered_velocity(n, 10.0, seed=15) ** 2
    g = Grid(n, 10.0, 4, profiles=_custom_profiles(n, 16))
    A = assemble_H(g, c2)
    U = np.random.default_rng(17).standard_normal(g.nstate)
    Es = [energy(g, c2, expm_multiply(t * A, U)) for t in (0.0, 0.005, 0.01, 0.02)]
    assert all(Es[i + 1] < Es[i] for i in range(3))
    lam = np.linalg.eigvals(A.toarray())
    x_lo, B = spectrum_rectangle(g, c2)
    assert x_lo < 0.0
    assert np.all(lam.real <= 1e-9) and np.all(lam.real >= x_lo - 1e-9)
    gamma, c0, c1 = ellipse_from_rectangle(x_lo, B)
    xc, ar, bi = gamma * c0, gamma * (1 + c1), gamma * (1 - c1)
    assert np.all(((lam.real - xc) / ar) ** 2 + (lam.imag / bi) ** 2 <= 1 + 1e-9)
