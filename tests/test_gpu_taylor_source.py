"""GPU parity of a tabulated source time function (expw_set_source_taylor)."""
import numpy as np
import pytest

from gpu_cases import TOL, make_case, rel_l2, to_dev
from oracle.source import TaylorTableSource, ricker_derivatives
from oracle.steppers import Problem, step

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("method", ["faber", "krylov", "rk4", "leapfrog"])
def test_tabulated_source_matches_oracle(dtype, method):
    case = make_case((41, 29), dtype, src=False, seed=21, max_k=12)
    g = case.prob.grid
    rng = np.random.default_rng(22)
    nst, p, t0, dt = 3, 6, 0.02, 1e-3
    table = rng.standard_normal((nst, p)) * np.array([1.0, 50.0, 2e3, 1e5, 4e6, 1e8])[:p]
    nodes, amps = [int(g.npts // 2 + 7)], [1.4]
    case.op.set_source_taylor(nodes, amps, table)
    src = TaylorTableSource(nodes, amps, table)
    prob = Problem(g, case.prob.c2, src)
    kw = {"faber": dict(m=12, p=p, ellipse=prob.ellipse()), "krylov": dict(k=12, p=p),
          "rk4": {}, "leapfrog": {}}[method]
    U = to_dev(case, case.U0)
    if method == "faber":
        case.op.step_faber(U, t0, dt, 12, nst)
    elif method == "krylov":
        case.op.step_krylov(U, t0, dt, 12, nst)
    elif method == "rk4":
        case.op.step_rk4(U, t0, dt, nst)
    else:
        case.op.step_leapfrog(U, t0, dt, nst)
    ref = np.array(case.U0, dtype=np.float64)
    for n in range(nst):
        src.bind(n, t0 + n * dt)
        ref = step(prob, method, ref, t0 + n * dt, dt, **kw)
    assert rel_l2(U.cpu().numpy(), ref) <= TOL[dtype]


def test_ricker_table_equals_the_ricker_source_bit_for_bit():
    case = make_case((41, 29), "float64", src=False, seed=23)
    nst, p, t0, dt = 4, 8, 0.03, 2e-3
    nodes, amps = [300], [1.1]
    outs = []
    for tabulated in (False, True):
        if tabulated:
            case.op.set_source_taylor(nodes, amps,
                                      np.array([ricker_derivatives(t0 + n * dt, 15.0, 0.05, p) for n in range(nst)]))
        else:
            case.op.set_source_ricker(nodes, amps, 15.0, 0.05, p)
        U = to_dev(case, case.U0)
        case.op.step_faber(U, t0, dt, 16, nst)
        outs.append(U.cpu().numpy())
    assert rel_l2(outs[1], outs[0]) <= 1e-15


def test_a_call_longer_than_the_table_is_rejected():
    from paper_2401_16322_amd import expwave as ew
    case = make_case((20, 12), "float64", src=False, seed=24)
    case.op.set_source_taylor([10], [1.0], np.ones((2, 4)))
    U = to_dev(case, case.U0)
    with pytest.raises(ew.ExpwError) as e:
        case.op.step_faber(U, 0.0, 1e-3, 6, 3)
    assert e.value.status == ew.EXPW_EINVAL
    case.op.step_faber(U, 0.0, 1e-3, 6, 2)
    case.op.sync()


@pytest.mark.parametrize("method", ["faber", "krylov", "rk4", "leapfrog"])
def test_non_finite_guard_reports_at_the_next_sync(method):
    """One NaN entry in the state: with the guard on, the next sync reports
    EXPW_ENONFINITE once; with it off, steps run and sync reports nothing."""
    import math
    from paper_2401_16322_amd import expwave as ew
    case = make_case((24, 18), "float64", src=True, seed=25, max_k=8)
    run = {"faber": lambda U: case.op.step_faber(U, 0.0, 1e-3, 6, 2),
           "krylov": lambda U: case.op.step_krylov(U, 0.0, 1e-3, 6, 2),
           "rk4": lambda U: case.op.step_rk4(U, 0.0, 1e-3, 2),
           "leapfrog": lambda U: case.op.step_leapfrog(U, 0.0, 1e-3, 2)}[method]
    U0 = np.array(case.U0)
    U0[37] = math.nan
    case.op.set_guard(True)
    U = to_dev(case, U0)
    run(U)
    with pytest.raises(ew.ExpwError) as e:
        case.op.sync()
    assert e.value.status == ew.EXPW_ENONFINITE
    case.op.sync()  # reported once
    # a finite state passes the guard
    U = to_dev(case, case.U0)
    run(U)
    case.op.sync()
    # guard off: the NaN goes through unreported
    case.op.set_guard(False)
    U = to_dev(case, U0)
    run(U)
    case.op.sync()
