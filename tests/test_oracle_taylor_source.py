"""Pins of the oracle's tabulated source (Sec. 3.2: over a step the source is
its Taylor polynomial) against the pinned Ricker source."""
import numpy as np

from oracle.operator import Grid
from oracle.source import PointSources, TaylorTableSource, ricker, ricker_derivatives
from oracle.steppers import Problem, faber_step, krylov_step


def _setup():
    g = Grid((23, 17), 10.0, 4, abc_cells=3, sigma_max=200.0)
    rng = np.random.default_rng(3)
    c2 = (1800.0 + 300.0 * rng.random(g.shape)) ** 2
    U = rng.standard_normal(g.nstate) * 1e-3
    return g, c2, U


def test_a_ricker_table_reproduces_the_ricker_source_in_faber_and_krylov():
    g, c2, U = _setup()
    p, t0, dt = 8, 0.04, 2e-3
    ps = PointSources((100,), (1.3,), 15.0, 0.05)
    tab = TaylorTableSource((100,), (1.3,), [ricker_derivatives(t0, 15.0, 0.05, p)])
    tab.bind(0, t0)
    for step, kw in ((faber_step, dict(m=14)), (krylov_step, dict(k=12))):
        a = step(Problem(g, c2, ps), U, t0, dt, p=p, **kw)
        b = step(Problem(g, c2, tab), U, t0, dt, p=p, **kw)
        assert np.array_equal(a, b)


def test_table_forcing_is_the_taylor_polynomial_of_the_row():
    p, t0 = 8, 0.04
    tab = TaylorTableSource((0,), (1.0,), [ricker_derivatives(t0, 15.0, 0.05, p)])
    tab.bind(0, t0)
    for tau in (0.0, 5e-4, 1e-3, 2e-3):
        # the Taylor remainder of degree p of the Ricker wavelet over tau
        err = abs(tab.value(t0 + tau) - ricker(t0 + tau, 15.0, 0.05))
        bound = np.max(np.abs(ricker_derivatives(t0 + tau, 15.0, 0.05, p + 2))) * tau ** p / 40320.0 * 4
        assert err <= bound + 1e-15
    # a polynomial table is exact at every tau: g(t) = 1 + 2 (t - t0) + 3 (t - t0)^2
    tab = TaylorTableSource((0,), (1.0,), [[1.0, 2.0, 6.0, 0.0]])
    tab.bind(0, t0)
    assert abs(tab.value(t0 + 0.1) - (1.0 + 0.2 + 0.03)) <= 1e-15


def test_bound_row_selects_the_step():
    tab = TaylorTableSource((5,), (2.0,), [[1.0, 0.0], [3.0, 0.0]])
    tab.bind(1, 0.5)
    assert tab.value(0.7) == 3.0
    assert list(tab.w_columns(0.5, 2)) == [0.0, 3.0]
