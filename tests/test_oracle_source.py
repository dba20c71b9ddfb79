"""Pins of the oracle's source handling (CPU only)."""
import numpy as np
import pytest
import sympy
from math import factorial
from scipy.linalg import expm

from oracle.source import apply_J, e_p, hermite_phys, ricker, ricker_derivatives


def test_ricker_shape():
    f, t0 = 15.0, 0.18
    assert ricker(t0, f, t0) == 1.0
    tz = 1.0 / (np.pi * f * np.sqrt(2.0))          # zeros of the Ricker wavelet
    assert abs(ricker(t0 + tz, f, t0)) < 1e-15 and abs(ricker(t0 - tz, f, t0)) < 1e-15
    t = np.linspace(0, 0.36, 11)
    assert np.allclose(ricker(t, f, t0), ricker(2 * t0 - t, f, t0))
    assert abs(ricker(0.0, f, t0)) < 1e-25          # the delay makes the onset negligible


def test_hermite_matches_numpy_hermite_module():
    x = np.linspace(-3, 3, 13)
    H = hermite_phys(12, x)
    for n in range(13):
        c = np.zeros(n + 1)
        c[n] = 1.0
        assert np.allclose(H[n], np.polynomial.hermite.hermval(x, c), rtol=1e-13, atol=1e-10)


@pytest.mark.parametrize("t", [0.1, 0.17, 0.18, 0.23, 0.31])
def test_ricker_derivatives_match_symbolic_differentiation(t):
    f0, t0 = 15.0, 0.18
    ts = sympy.symbols("t")
    a = (sympy.pi * f0) ** 2
    g = (1 - 2 * a * (ts - t0) ** 2) * sympy.exp(-a * (ts - t0) ** 2)
    p = 12
    ours = ricker_derivatives(t, f0, t0, p)
    for k in range(p):
        ref = float(sympy.diff(g, ts, k).subs(ts, t).evalf(30))
        assert abs(ours[k] - ref) <= 1e-13 * abs(ref) + 1e-300, k


def test_augmented_tail_holds_taylor_monomials():
    """exp(t J) e_p has t^(p-c) / (p-c)! in entry c (1-based): W's column order."""
    p, t = 7, 0.37
    J = np.diag(np.ones(p - 1), 1)
    tau = expm(t * J) @ e_p(p)
    for c in range(1, p + 1):
        assert np.isclose(tau[c - 1], t ** (p - c) / factorial(p - c))
    x = np.arange(1.0, p + 1)
    assert np.allclose(apply_J(x), J @ x)
