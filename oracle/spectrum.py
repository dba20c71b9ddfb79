"""Oracle: spectrum rectangle, Faber ellipse and Faber coefficients.

Test infrastructure only (see the package docstring).

Paper anchor: Sec. 3.2, Faber approximation (FA). The Faber polynomials of
the ellipse map psi(w) = gamma (w + c0 + c1 / w) satisfy
    F_0 = I,  F_1 = H/gamma - c0 I,  F_2 = F_1^2 - 2 c1 I,
    F_j = F_1 F_{j-1} - c1 F_{j-2}   (j >= 3),
and a step is u^{n+1} = sum_{j=0..m} a_j F_j(H) u^n. The paper says gamma,
c0, c1 and a_j depend on the eigenvalue distribution but gives no formula;
the reading used here:

* the spectrum lies in the rectangle [x_lo, 0] x i[-B, B], with
  x_lo = -max diagonal damping and B = c_max sqrt(d) (2/h) sum |alpha_l|
  (for sigma = 0 the operator is skew-adjoint in the energy inner product, and
  the diagonal damping only moves the field of values left);
* the ellipse is the minimum-area ellipse through the rectangle's corners
  (semi-axes sqrt(2) times the half-widths), centred at x_lo/2;
* a_j are the Laurent coefficients of exp(dt psi(w)) on the unit circle,
  which in closed form are scaled Bessel functions.
"""
from __future__ import annotations

import numpy as np
from scipy.special import iv, jv, gammaln

from .operator import damping_fields, staggered_weights


def spectrum_rectangle(grid, c2):
    """(x_lo, B): real and imaginary extent of the field of values of H."""
    alpha = staggered_weights(grid.order)
    B = np.sqrt(np.max(c2)) * np.sqrt(grid.ndim) * (2.0 / grid.h) * np.sum(np.abs(alpha))
    sig_p, sig_v = damping_fields(grid)
    smax = max([np.max(sig_p)] + [np.max(s) for s in sig_v])
    return -float(smax), float(B)


def ellipse_from_rectangle(x_lo, B):
    """(gamma, c0, c1) of the minimum-area ellipse around [x_lo, 0] x i[-B, B].

    psi maps the unit circle onto the ellipse with real semi-axis
    gamma (1 + c1), imaginary semi-axis gamma (1 - c1) and centre gamma c0.
    A degenerate rectangle (x_lo = 0) gives the segment i[-B, B].
    """
    x_c = 0.5 * x_lo
    if x_lo < 0.0:
        a_r = np.sqrt(2.0) * 0.5 * abs(x_lo)
        b_i = np.sqrt(2.0) * B
    else:
        a_r = 0.0
        b_i = B
    gamma = 0.5 * (a_r + b_i)
    c1 = (a_r - b_i) / (a_r + b_i)
    c0 = x_c / gamma
    return float(gamma), float(c0), float(c1)


def faber_coefficients(gamma, c0, c1, dt, m):
    """a_0..a_m for exp(dt z) on the ellipse (closed form via Bessel functions).

    With z = gamma dt: exp(z (w + c0 + c1/w)) = e^{z c0} sum_j a'_j (w^j + (c1/w)^j)
    where, by the Bessel generating functions,
      c1 < 0: a_j = e^{z c0} |c1|^{-j/2} J_j(2 z sqrt|c1|)
      c1 > 0: a_j = e^{z c0} c1^{-j/2} I_j(2 z sqrt(c1))
      c1 = 0: a_j = e^{z c0} z^j / j!
    """
    z = gamma * dt
    j = np.arange(m + 1)
    pre = np.exp(z * c0)
    if c1 < 0.0:
        r = np.sqrt(-c1)
        return pre * jv(j, 2.0 * z * r) / r ** j
    if c1 > 0.0:
        r = np.sqrt(c1)
        return pre * iv(j, 2.0 * z * r) / r ** j
    return pre * np.exp(j * np.log(z) - gammaln(j + 1.0)) if z > 0 else np.eye(1, m + 1)[0] * pre


def faber_coefficients_contour(gamma, c0, c1, dt, m, M=1024):
    """a_j by the trapezoidal rule on |w| = 1 (Laurent coefficients via FFT)."""
    theta = 2.0 * np.pi * np.arange(M) / M
    w = np.exp(1j * theta)
    f = np.exp(dt * gamma * (w + c0 + c1 / w))
    coef = np.fft.fft(f) / M          # coefficient of w^{+j} is sum f e^{-i j theta} / M
    return coef[: m + 1].real.copy()


def faber_polynomials_scalar(z, gamma, c0, c1, m):
    """F_0(z) .. F_m(z) for scalar (array) z by the three-term recurrence."""
    z = np.asarray(z, dtype=np.complex128)
    F = [np.ones_like(z), z / gamma - c0]
    if m >= 2:
        F.append(F[1] * F[1] - 2.0 * c1)
    for _ in range(3, m + 1):
        F.append(F[1] * F[-1] - c1 * F[-2])
    return F[: m + 1]


def faber_series_scalar(z, gamma, c0, c1, dt, m):
    """sum_j a_j F_j(z): the Faber approximation of exp(dt z) for scalar z."""
    a = faber_coefficients(gamma, c0, c1, dt, m)
    F = faber_polynomials_scalar(z, gamma, c0, c1, m)
    return sum(a[j] * F[j] for j in range(m + 1))


def psi(w, gamma, c0, c1):
    """The exterior conformal map of the ellipse."""
    return gamma * (w + c0 + c1 / w)
