"""GPU parity of the HIP library against the FP64 oracle (element by element).

Tolerances: FP64 1e-11 and FP32 1e-5 relative L2 per state for the steppers;
the operator itself is compared in the max norm relative to max |H x|.
"""
import numpy as np
import pytest

from oracle.operator import apply_H, split_state
from oracle.steppers import run
from gpu_cases import TOL, make_case, rel_l2, to_dev

pytestmark = pytest.mark.gpu

DTYPES = ["float64", "float32"]
APPLY_TOL = {"float64": 1e-13, "float32": 2e-6}


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,order,bc", [
    ((37, 29), 4, "zero"), ((130, 67), 4, "zero"), ((64, 48), 8, "zero"),
    ((24, 20), 4, "periodic"), ((24, 20), 8, "periodic"),
    ((21, 17, 13), 4, "zero"), ((16, 12, 10), 8, "periodic"), ((1, 9), 4, "zero"), ((7, 1), 4, "zero"),
])
def test_apply_matches_oracle(dtype, n, order, bc):
    case = make_case(n, dtype, order, bc, abc=3, src=False, seed=1)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(case.prob.grid.nstate)
    y = case.op.apply(to_dev(case, x)).cpu().numpy()
    ref = apply_H(case.prob.grid, case.prob.c2, x)
    assert np.max(np.abs(y - ref)) <= APPLY_TOL[dtype] * np.max(np.abs(ref))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,fuse", [(1, 1), (2, 1), (3, 1), (7, 1), (16, 1), (2, 2), (5, 2), (16, 4),
                                    (7, 3), (16, 8), (12, 6), (10, 4)])
def test_faber_steps_match_oracle(dtype, m, fuse):
    if dtype == "float64" and fuse > 4:
        fuse = 4
    case = make_case((150, 70), dtype, seed=2)     # several 64x16 tiles and ragged edges
    case.op.set_tuning(fuse)
    dt, nst = 1.5e-3, 3
    U = to_dev(case, case.U0)
    case.op.step_faber(U, 0.02, dt, m, nst)
    ref, _, _ = run(case.prob, "faber", case.U0, 0.02, dt, nst, m=m, p=case.p)
    assert rel_l2(U.cpu().numpy(), ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,m,fuse", [((600, 300), 16, 4), ((600, 300), 13, 6), ((600, 300), 7, 3),
                                      ((257, 129), 16, 2), ((150, 70), 10, 5), ((5, 3), 8, 4),
                                      ((1, 40), 8, 4), ((70, 1), 9, 3)])
def test_streamed_passes_match_oracle_and_tiled(dtype, n, m, fuse):
    """The row-streaming fused passes (forced on grids of any size): several
    column bands with a ragged last one, row segments of 64 rows with their
    warm-up, three sources, passes of 2..6 terms and a shorter last pass,
    and degenerate grids. Against the oracle on its own ellipse, and against
    the tiled passes (the same polynomial up to rounding)."""
    from paper_2401_16322_amd.expwave import EXPW_PASS_STREAMED, EXPW_PASS_TILED
    if dtype == "float64":
        fuse = min(fuse, 4)
    case = make_case(n, dtype, seed=21, n_src=3 if min(n) > 2 else 1, abc=min(6, max(1, min(n) // 3)))
    case.op.set_tuning(fuse)
    dt, nst = 2e-3, 3
    outs = {}
    for kind in (EXPW_PASS_STREAMED, EXPW_PASS_TILED):
        case.op.set_pass_kernel(kind)
        U = to_dev(case, case.U0)
        case.op.step_faber(U, 0.03, dt, m, nst)
        outs[kind] = U.cpu().numpy()
    ref, _, _ = run(case.prob, "faber", case.U0, 0.03, dt, nst, m=m, p=case.p, ellipse=case.prob.ellipse())
    assert rel_l2(outs[EXPW_PASS_STREAMED], ref) <= TOL[dtype]
    assert rel_l2(outs[EXPW_PASS_STREAMED], outs[EXPW_PASS_TILED]) <= (1e-13 if dtype == "float64" else 2e-6)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,m,fuse", [((900, 300), 16, 4), ((900, 300), 7, 3), ((257, 129), 9, 2),
                                      ((150, 70), 10, 4), ((9, 5), 8, 4), ((1, 40), 8, 4), ((70, 1), 9, 3)])
def test_streamed_passes_order8_match_oracle_and_tiled(dtype, n, m, fuse):
    """The row-streaming passes at the paper's 8th order (every term four rows
    behind the previous one, four halo columns per term; FP64 at most three
    terms per pass): two bands with a ragged last one, row segments with
    their warm-up, sources, passes of 2..4 terms and a shorter last pass, and
    degenerate grids. Against the oracle on its own ellipse and against the
    tiled passes."""
    from paper_2401_16322_amd.expwave import EXPW_PASS_STREAMED, EXPW_PASS_TILED
    case = make_case(n, dtype, order=8, seed=23, n_src=3 if min(n) > 2 else 1,
                     abc=min(6, max(1, min(n) // 3)))
    case.op.set_tuning(fuse)
    dt, nst = 2e-3, 2
    outs = {}
    for kind in (EXPW_PASS_STREAMED, EXPW_PASS_TILED):
        case.op.set_pass_kernel(kind)
        U = to_dev(case, case.U0)
        case.op.step_faber(U, 0.03, dt, m, nst)
        outs[kind] = U.cpu().numpy()
    ref, _, _ = run(case.prob, "faber", case.U0, 0.03, dt, nst, m=m, p=case.p, ellipse=case.prob.ellipse())
    assert rel_l2(outs[EXPW_PASS_STREAMED], ref) <= TOL[dtype]
    assert rel_l2(outs[EXPW_PASS_STREAMED], outs[EXPW_PASS_TILED]) <= (1e-13 if dtype == "float64" else 2e-6)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("fuse", [2, 4, 8])
def test_fused_and_unfused_faber_agree_to_rounding(dtype, fuse):
    """Tiling/fusion invariance: results depend on the fusion depth only through rounding."""
    case = make_case((200, 90), dtype, seed=3, n_src=3)
    outs = []
    for f in (1, fuse):
        case.op.set_tuning(f)
        U = to_dev(case, case.U0)
        case.op.step_faber(U, 0.03, 2e-3, 16, 2)
        outs.append(U.cpu().numpy())
    assert rel_l2(outs[1], outs[0]) <= (1e-14 if dtype == "float64" else 2e-6)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,m", [((21, 17, 13), 5), ((70, 9, 6), 12), ((1, 9, 11), 4), ((37, 29), 7)])
def test_faber_order8_one_term_kernel_matches_oracle(dtype, n, m):
    """The paper's 8th-order stencil one term per sweep with zero ghosts (the
    zero-ghost term kernel at K = 4: every 3D order-8 step, and 2D with fuse
    = 1), ragged in every direction, with sources, against the oracle."""
    case = make_case(n, dtype, order=8, seed=27, n_src=2 if min(n) > 2 else 1, abc=2)
    case.op.set_tuning(1)
    dt, nst = 1.5e-3, 2
    U = to_dev(case, case.U0)
    case.op.step_faber(U, 0.02, dt, m, nst)
    ref, _, _ = run(case.prob, "faber", case.U0, 0.02, dt, nst, m=m, p=case.p, ellipse=case.prob.ellipse())
    assert rel_l2(U.cpu().numpy(), ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [(5, 3), (1, 40), (70, 1), (13, 11, 9)])
def test_faber_tiny_and_degenerate_grids(dtype, n):
    case = make_case(n, dtype, abc=1, seed=4)
    U = to_dev(case, case.U0)
    case.op.step_faber(U, 0.04, 1e-3, 8, 2)
    ref, _, _ = run(case.prob, "faber", case.U0, 0.04, 1e-3, 2, m=8, p=case.p)
    assert rel_l2(U.cpu().numpy(), ref) <= TOL[dtype]


@pytest.mark.parametrize("path", ["persistent", "launches"])
@pytest.mark.parametrize("mode", ["device", "host"])
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("k,src", [(1, True), (5, True), (16, True), (17, True), (20, True),
                                   (12, False), (32, True), (40, True)])
def test_krylov_steps_match_oracle(dtype, k, src, mode, path):
    case = make_case((45, 33), dtype, src=src, seed=5, max_k=40)
    case.op.set_krylov_expm(mode)
    case.op.set_krylov_persistent(path == "persistent")
    dt, nst = 1e-3, 2
    U = to_dev(case, case.U0)
    case.op.step_krylov(U, 0.03, dt, k, nst)
    ref, _, _ = run(case.prob, "krylov", case.U0, 0.03, dt, nst, k=k, p=case.p)
    assert rel_l2(U.cpu().numpy(), ref) <= TOL[dtype]


def test_krylov_happy_breakdown_on_plane_wave():
    """A periodic plane wave spans a 2-dimensional invariant subspace of H, so the
    Arnoldi process breaks down after two vectors (k_eff = 2) and the step is
    exact: the closed form shifted by dt."""
    from oracle.exact import plane_wave
    case = make_case((24, 20), "float64", bc="periodic", src=False, homogeneous=1.0, max_k=10)
    U0, omega = plane_wave(case.prob.grid, 1.0, (3, 2), 0.0)
    U = to_dev(case, U0)
    case.op.step_krylov(U, 0.0, 2.0, 10, 1)
    ref, _, _ = run(case.prob, "krylov", U0, 0.0, 2.0, 1, k=10)
    exact, _ = plane_wave(case.prob.grid, 1.0, (3, 2), 2.0)
    keff, beta = case.op.krylov_info()
    assert keff == 2 and np.isclose(beta, np.linalg.norm(U0))
    assert rel_l2(U.cpu().numpy(), ref) <= 1e-11
    assert rel_l2(U.cpu().numpy(), exact) <= 1e-11


@pytest.mark.parametrize("path", ["persistent", "launches"])
def test_krylov_zero_state_without_source_stays_zero(path):
    case = make_case((20, 10), "float64", src=False, seed=7, max_k=8, smooth=False)
    case.op.set_krylov_persistent(path == "persistent")
    U = to_dev(case, case.U0)
    case.op.step_krylov(U, 0.0, 1e-3, 6, 2)
    case.op.sync()
    assert float(U.abs().max()) == 0.0


@pytest.mark.parametrize("dtype", DTYPES)
def test_krylov_persistent_at_full_1001x501_size(dtype):
    """The persistent Arnoldi kernel at the 1001x501 bench size, against the
    launch-per-step path (rounding-level agreement) and the oracle."""
    import torch
    from oracle.operator import Grid
    from oracle.source import PointSources
    from oracle.steppers import Problem
    from paper_2401_16322_amd.expwave import Operator
    from synthetic import get_workload, smooth_state
    w = get_workload("layered2d_1001x501")
    g = Grid(w.n, w.h, 4, abc_cells=w.abc_cells, sigma_max=w.sigma_max)
    c2 = w.c2()
    prob = Problem(g, c2, PointSources((w.source_node(),), (1.0,), w.f_peak, w.t_delay))
    U0 = smooth_state(w.n, seed=2002, width_cells=12.0)
    tdt = torch.float64 if dtype == "float64" else torch.float32
    op = Operator(w.n, w.h, torch.tensor(c2, dtype=tdt, device="cuda"), abc_cells=w.abc_cells,
                  sigma_max=w.sigma_max, max_krylov_k=16, max_taylor_p=w.taylor_p)
    op.set_source_ricker([w.source_node()], [1.0], w.f_peak, w.t_delay, w.taylor_p)
    outs = []
    for persistent in (True, False):
        op.set_krylov_persistent(persistent)
        U = torch.tensor(U0, dtype=tdt, device="cuda")
        op.step_krylov(U, 0.2, 2e-3, 16, 2)
        op.sync()
        outs.append(U.cpu().numpy())
    ref, _, _ = run(prob, "krylov", U0, 0.2, 2e-3, 2, k=16, p=w.taylor_p)
    assert rel_l2(outs[0], outs[1]) <= (1e-13 if dtype == "float64" else 1e-6)
    assert rel_l2(outs[0], ref) <= TOL[dtype]


@pytest.mark.parametrize("path", ["persistent", "launches"])
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,order,bc", [((17, 13, 11), 4, "zero"), ((40, 31), 8, "zero"),
                                        ((14, 12, 10), 4, "periodic"), ((36, 28), 8, "periodic"),
                                        ((9, 8, 7), 8, "zero")])
def test_krylov_3d_order8_periodic_match_oracle(n, order, bc, dtype, path):
    """Both Krylov paths in 3D (four fields per grid point in the persistent
    kernel), at order 8 and with periodic ghosts."""
    case = make_case(n, dtype, order=order, bc=bc, src=(bc == "zero"), seed=21, max_k=12)
    case.op.set_krylov_persistent(path == "persistent")
    U = to_dev(case, case.U0)
    case.op.step_krylov(U, 0.02, 1e-3, 12, 2)
    ref, _, _ = run(case.prob, "krylov", case.U0, 0.02, 1e-3, 2, k=12, p=case.p)
    assert rel_l2(U.cpu().numpy(), ref) <= TOL[dtype]


@pytest.mark.parametrize("n,src", [((509, 515), True), ((512, 512), True), ((512, 512), False),
                                   ((511, 513), True)])
def test_krylov_persistent_slot_boundaries(n, src):
    """Grids at the edges of the persistent kernel's layout (with 256 workgroups
    of 1024 threads: 262,144 threads): 509 x 515 + 8 tail elements fill one
    point per thread up to the last threads; 512 x 512 needs a second point
    per thread and puts the tail in the second slot of the first threads;
    511 x 513 + 8 just overflows one point per thread. Against the
    launch-per-step path."""
    import torch
    case = make_case(n, "float64", seed=41, max_k=8, src=src)
    outs = []
    for persistent in (True, False):
        case.op.set_krylov_persistent(persistent)
        U = to_dev(case, case.U0)
        case.op.step_krylov(U, 0.02, 2e-3, 8, 2)
        case.op.sync()
        outs.append(U.cpu().numpy())
    assert rel_l2(outs[0], outs[1]) <= 1e-13


@pytest.mark.parametrize("dtype", DTYPES)
def test_krylov_persistent_consecutive_launches(dtype):
    """One operator, many persistent launches: the reduction area is carried
    from launch to launch (barrier numbering continued) and filled again only
    when the Krylov dimension changes its layout. Against the launch-per-step
    path over the same sequence of calls."""
    outs = []
    for persistent in (True, False):
        case = make_case((70, 52), dtype, seed=51, max_k=12, n_src=2)
        case.op.set_krylov_persistent(persistent)
        U = to_dev(case, case.U0)
        t = 0.01
        for k, nst in ((12, 4), (5, 3), (12, 2), (12, 1), (7, 5)):
            case.op.step_krylov(U, t, 1e-3, k, nst)
            t += nst * 1e-3
        case.op.sync()
        outs.append(U.cpu().numpy())
    assert rel_l2(outs[0], outs[1]) <= (1e-13 if dtype == "float64" else 2e-6)


@pytest.mark.parametrize("dtype", DTYPES)
def test_krylov_persistent_three_points_per_thread(dtype):
    """1001 x 650 points: more than two grid points per thread of the
    persistent kernel (three in 2D), against the launch-per-step path and the
    oracle."""
    import torch
    case = make_case((1001, 650), dtype, seed=31, max_k=16)
    outs = []
    for persistent in (True, False):
        case.op.set_krylov_persistent(persistent)
        U = to_dev(case, case.U0)
        case.op.step_krylov(U, 0.02, 2e-3, 16, 2)
        case.op.sync()
        outs.append(U.cpu().numpy())
    assert rel_l2(outs[0], outs[1]) <= (1e-13 if dtype == "float64" else 1e-6)
    ref, _, _ = run(case.prob, "krylov", case.U0, 0.02, 2e-3, 2, k=16, p=case.p)
    assert rel_l2(outs[0], ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [(60, 41), (17, 13, 11)])
def test_rk4_matches_oracle(dtype, n):
    case = make_case(n, dtype, seed=8)
    dt, nst = 5e-4, 6
    U = to_dev(case, case.U0)
    case.op.step_rk4(U, 0.03, dt, nst)
    ref, _, _ = run(case.prob, "rk4", case.U0, 0.03, dt, nst)
    assert rel_l2(U.cpu().numpy(), ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [(60, 41), (17, 13, 11)])
def test_leapfrog_matches_oracle(dtype, n):
    case = make_case(n, dtype, seed=9)
    dt, nst = 5e-4, 10
    U = to_dev(case, case.U0)
    case.op.step_leapfrog(U, 0.03, dt, nst)
    ref, _, _ = run(case.prob, "leapfrog", case.U0, 0.03, dt, nst)
    assert rel_l2(U.cpu().numpy(), ref) <= TOL[dtype]


@pytest.mark.parametrize("layout", ["scattered", "run", "surface_row"])
@pytest.mark.parametrize("method", ["faber", "faber13", "krylov", "rk4", "leapfrog"])
def test_receiver_traces_match_oracle(method, layout):
    """Scattered receivers are gathered after each step; consecutive ones (a run
    that crosses a row end, or the whole surface row) are written by the step's
    last kernel. faber13: passes of 4, 4, 4 terms and an unfused last term."""
    import torch
    case = make_case((80, 50), "float64", seed=10, max_k=10, n_src=2)
    g = case.prob.grid
    rec = {"scattered": np.array([0, g.npts - 1, 5 * 80 + 7, 25 * 80 + 40, 49 * 80 + 79]),
           "run": np.arange(5 * 80 + 70, 5 * 80 + 95),
           "surface_row": np.arange(80)}[layout].astype(np.int64)
    case.op.set_receivers(rec)
    nst = 5
    m = 13 if method == "faber13" else 12
    method = "faber" if method == "faber13" else method
    kw = {"faber": dict(m=m, p=case.p), "krylov": dict(k=10, p=case.p)}.get(method, {})
    dt = 1e-3 if method in ("faber", "krylov") else 3e-4
    U = to_dev(case, case.U0)
    tr = torch.zeros(nst * rec.size, dtype=torch.float64, device="cuda")
    getattr(case.op, "step_" + method)(U, 0.02, dt, *([kw["m"]] if method == "faber" else
                                                     [kw["k"]] if method == "krylov" else []),
                                       nsteps=nst, traces=tr)
    _, traces, _ = run(case.prob, method, case.U0, 0.02, dt, nst, receivers=rec, **kw)
    assert rel_l2(tr.cpu().numpy().reshape(nst, rec.size), traces) <= 1e-11


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("method", ["faber", "krylov", "krylov_host", "rk4", "leapfrog"])
def test_receivers_on_a_run_equal_the_gathered_state(method, dtype):
    """Receivers written by the step's last kernel hold exactly the values a
    gather of the state gives: the same nodes as a run and in reverse order
    (not a run, so gathered) give the same traces bit for bit, and the last
    row equals the final state at the nodes."""
    import torch
    rec = np.arange(3 * 61 + 50, 3 * 61 + 90, dtype=np.int64)   # crosses a row end
    outs = []
    for order in (rec, rec[::-1].copy()):
        case = make_case((61, 47), dtype, seed=12, max_k=12, n_src=1)
        if method == "krylov_host":
            case.op.set_krylov_expm("host")
        case.op.set_receivers(order)
        U = to_dev(case, case.U0)
        nst = 4
        tr = torch.zeros(nst * order.size, dtype=U.dtype, device="cuda")
        name = "krylov" if method == "krylov_host" else method
        args = [14] if name == "faber" else [12] if name == "krylov" else []
        dt = 1e-3 if name in ("faber", "krylov") else 3e-4
        getattr(case.op, "step_" + name)(U, 0.01, dt, *args, nsteps=nst, traces=tr)
        case.op.sync()
        t = tr.cpu().numpy().reshape(nst, order.size)
        assert np.array_equal(t[-1], U.cpu().numpy()[order])
        outs.append(t)
    assert np.array_equal(outs[0], outs[1][:, ::-1])


@pytest.mark.parametrize("dtype", DTYPES)
def test_homogeneous_101_full_run(dtype):
    """The 101x101 homogeneous case in full: Faber degree 16, dt = 4 ms, 100 steps
    (T = 0.4 s), 15 Hz Ricker at the centre with 0.18 s delay, zero initial state;
    every 10th snapshot compared (pressure, physical interior)."""
    import torch
    from oracle.operator import Grid, rel_l2_pressure
    from oracle.source import PointSources
    from oracle.steppers import Problem
    from paper_2401_16322_amd.expwave import Operator
    from synthetic import get_workload
    w = get_workload("homog2d_101")
    g = Grid(w.n, w.h, 4, abc_cells=w.abc_cells, sigma_max=w.sigma_max)
    c2 = w.c2()
    prob = Problem(g, c2, PointSources((w.source_node(),), (1.0,), w.f_peak, w.t_delay))
    tdt = torch.float64 if dtype == "float64" else torch.float32
    op = Operator(w.n, w.h, torch.tensor(c2, dtype=tdt, device="cuda"), abc_cells=w.abc_cells,
                  sigma_max=w.sigma_max, max_taylor_p=w.taylor_p)
    op.set_source_ricker([w.source_node()], [1.0], w.f_peak, w.t_delay, w.taylor_p)
    U = torch.zeros(g.nstate, dtype=tdt, device="cuda")
    nsteps = int(round(w.T / w.dt))
    _, _, snaps = run(prob, "faber", np.zeros(g.nstate), 0.0, w.dt, nsteps, snapshot_every=10,
                      m=w.faber_m, p=w.taylor_p)
    pmax = max(np.linalg.norm(split_state(g, s)[0]) for s in snaps.values())
    for s in range(10, nsteps + 1, 10):
        op.step_faber(U, (s - 10) * w.dt, w.dt, w.faber_m, 10)
        ref = snaps[s]
        err = rel_l2_pressure(g, U.cpu().numpy(), ref)
        if np.linalg.norm(split_state(g, ref)[0]) >= 1e-3 * pmax:
            assert err <= TOL[dtype], (s, err)


def test_layered_1001x501_steps_at_full_size():
    """The 1001x501 layered medium at full size in the bench's launch
    configuration (FP32, Faber degree 16, fused passes of 6, 6 and 4 terms), three
    steps of 2 ms from a seeded smooth state, with the surface receiver line."""
    import torch
    from oracle.operator import Grid
    from oracle.source import PointSources
    from oracle.steppers import Problem
    from paper_2401_16322_amd.expwave import Operator
    from synthetic import get_workload, smooth_state
    w = get_workload("layered2d_1001x501")
    g = Grid(w.n, w.h, 4, abc_cells=w.abc_cells, sigma_max=w.sigma_max)
    c2 = w.c2()
    prob = Problem(g, c2, PointSources((w.source_node(),), (1.0,), w.f_peak, w.t_delay))
    U0 = smooth_state(w.n, seed=2001, width_cells=12.0)
    rec = w.receiver_nodes()
    _, traces, _ = run(prob, "faber", U0, 0.15, w.dt, 3, receivers=rec, m=w.faber_m, p=w.taylor_p)
    for dtype, tdt in (("float32", torch.float32), ("float64", torch.float64)):
        op = Operator(w.n, w.h, torch.tensor(c2, dtype=tdt, device="cuda"), abc_cells=w.abc_cells,
                      sigma_max=w.sigma_max, max_taylor_p=w.taylor_p)
        op.set_source_ricker([w.source_node()], [1.0], w.f_peak, w.t_delay, w.taylor_p)
        op.set_receivers(rec)
        U = torch.tensor(U0, dtype=tdt, device="cuda")
        tr = torch.zeros(3 * rec.size, dtype=tdt, device="cuda")
        op.step_faber(U, 0.15, w.dt, w.faber_m, 3, traces=tr)
        ref, _, _ = run(prob, "faber", U0, 0.15, w.dt, 3, m=w.faber_m, p=w.taylor_p)
        assert rel_l2(U.cpu().numpy(), ref) <= TOL[dtype]
        assert rel_l2(tr.cpu().numpy().reshape(3, -1), traces) <= TOL[dtype]


def test_source_at_grid_corners_and_many_sources():
    case = make_case((66, 40), "float64", seed=11, n_src=0, src=False)
    import numpy as _np
    from oracle.source import PointSources
    g = case.prob.grid
    nodes = _np.array([0, g.npts - 1, 65, 39 * 66, 1000, 1001, 1066], dtype=_np.int64)
    amps = _np.linspace(0.5, 2.0, nodes.size)
    case.op.set_source_ricker(nodes, amps, 15.0, 0.05, 8)
    case.prob.src = PointSources(tuple(nodes), tuple(amps), 15.0, 0.05)
    for fuse in (1, 4):
        case.op.set_tuning(fuse)
        U = to_dev(case, case.U0)
        case.op.step_faber(U, 0.04, 1e-3, 9, 2)
        ref, _, _ = run(case.prob, "faber", case.U0, 0.04, 1e-3, 2, m=9, p=8)
        assert rel_l2(U.cpu().numpy(), ref) <= 1e-11


def test_zero_steps_leave_state_unchanged():
    case = make_case((30, 20), "float64", seed=12)
    U = to_dev(case, case.U0)
    case.op.step_faber(U, 0.0, 1e-3, 8, 0)
    case.op.sync()
    assert np.array_equal(U.cpu().numpy(), case.U0)


def test_invalid_arguments_raise():
    import torch
    from paper_2401_16322_amd.expwave import ExpwError, Operator
    case = make_case((30, 20), "float64", seed=13, max_k=4)
    U = to_dev(case, case.U0)
    with pytest.raises(ExpwError):
        case.op.step_krylov(U, 0.0, 1e-3, 5, 1)        # k above max_krylov_k
    with pytest.raises(ExpwError):
        case.op.step_faber(U, 0.0, -1e-3, 8, 1)        # dt <= 0
    with pytest.raises(ExpwError):
        case.op.set_source_ricker([600], [1.0], 15.0, 0.1, 8)   # index out of range
    with pytest.raises(ExpwError):
        case.op.set_receivers([-1])
    bad = torch.full((30, 20), float("nan"), dtype=torch.float64, device="cuda")
    with pytest.raises(ExpwError) as e:
        Operator((20, 30), 10.0, bad)
    assert e.value.status == -4


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", DTYPES)
def test_faber_dense_output_matches_oracle(dtype):
    """Faber steps that record every term at the receivers: the state equals
    the oracle's (and the default fused path's), the recorded terms equal the
    oracle's terms at the receivers, and the dense output at tau in
    {0, dt/3, dt/2, dt} equals the oracle's sum of a_j(tau) v_j."""
    import torch
    from oracle.steppers import faber_dense, faber_step, faber_terms
    case = make_case((70, 45), dtype, seed=21, n_src=2)
    g = case.prob.grid
    rec = np.array(sorted({0, g.npts - 1, 7 * 70 + 3, 22 * 70 + 35, 44 * 70 + 69, case.nodes[0]}),
                   dtype=np.int64)
    case.op.set_receivers(rec)
    m, dt, nst, t0 = 12, 2e-3, 3, 0.03
    tdt = case.torch_dtype
    U = to_dev(case, case.U0)
    terms = torch.zeros(nst * (m + 1) * rec.size, dtype=tdt, device="cuda")
    tr = torch.zeros(nst * rec.size, dtype=tdt, device="cuda")
    case.op.step_faber_dense(U, t0, dt, m, nst, terms, traces=tr)
    U2 = to_dev(case, case.U0)
    case.op.step_faber(U2, t0, dt, m, nst)
    ell = case.prob.ellipse()
    Us = [case.U0]
    for s in range(nst):
        Us.append(faber_step(case.prob, Us[-1], t0 + s * dt, dt, m, p=case.p, ellipse=ell))
    tol = TOL[dtype]
    tight = 1e-13 if dtype == "float64" else 2e-6
    assert rel_l2(U.cpu().numpy(), Us[-1]) <= tol
    assert rel_l2(U.cpu().numpy(), U2.cpu().numpy()) <= tight
    gt = terms.cpu().numpy().reshape(nst, m + 1, rec.size)
    for s in range(nst):
        ot = np.array([v[rec] for v in faber_terms(case.prob, Us[s], t0 + s * dt, m, case.p, ell)])
        assert rel_l2(gt[s], ot) <= tol
    taus = [0.0, dt / 3, dt / 2, dt]
    coef = case.op.dense_coefficients(m, taus)
    steps = torch.tensor(np.repeat(np.arange(nst), len(taus)))
    coefs = torch.tensor(np.tile(coef, (nst, 1)))
    out = case.op.dense_output(m, terms, nst, steps, coefs).cpu().numpy()
    for s in range(nst):
        od = faber_dense(case.prob, Us[s], t0 + s * dt, m, taus, rec, case.p, ell)
        assert rel_l2(out[s * 4:(s + 1) * 4], od) <= tol
    # tau = dt reproduces the receiver trace of the same step
    assert rel_l2(out[3::4], tr.view(nst, -1).cpu().numpy()) <= tight


@pytest.mark.gpu
def test_faber_dense_output_edge_cases():
    """An out-of-range step index gives NaN; dense steps need receivers."""
    import torch
    from paper_2401_16322_amd import expwave as xw
    case = make_case((20, 12), "float64", seed=22)
    U = to_dev(case, case.U0)
    with pytest.raises(xw.ExpwError):
        xw.expw_step_faber_dense(case.op.op, U.data_ptr(), 0.0, 1e-3, 4, 1, None,
                                 torch.zeros(100, dtype=torch.float64, device="cuda").data_ptr())
    rec = np.array([5, 17], dtype=np.int64)
    case.op.set_receivers(rec)
    terms = torch.zeros(2 * 5 * rec.size, dtype=torch.float64, device="cuda")
    case.op.step_faber_dense(U, 0.0, 1e-3, 4, 2, terms)
    out = case.op.dense_output(4, terms, 2, torch.tensor([1, 2, -1]),
                               torch.ones(3 * 5, dtype=torch.float64)).cpu().numpy()
    assert np.all(np.isfinite(out[0])) and np.all(np.isnan(out[1])) and np.all(np.isnan(out[2]))
    t = terms.cpu().numpy().reshape(2, 5, rec.size)
    assert np.allclose(out[0], t[1].sum(axis=0), rtol=1e-14, atol=0)


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m", [2, 3, 5, 16])
def test_faber_3d_fused_matches_oracle_and_unfused(dtype, m):
    """Two terms per sweep in 3D: several x-y tiles with ragged edges, three
    z-chunks (64, 64, 22 planes), sources on tile and chunk boundaries; odd m
    ends with one unfused term. Compared with the oracle and with the one-term
    path."""
    from oracle.source import PointSources
    from oracle.steppers import Problem
    n = (70, 20, 150)
    case = make_case(n, dtype, seed=41, src=False, abc=4)
    g = case.prob.grid
    nodes = [g.npts // 2 + 7, 55 + 70 * (7 + 20 * 63), 56 + 70 * (8 + 20 * 64), 3 + 70 * (19 + 20 * 127)]
    amps = [1.0, -0.7, 0.5, 1.3]
    case.op.set_source_ricker(np.array(nodes), np.array(amps), 15.0, 0.05, case.p)
    prob = Problem(g, case.prob.c2, PointSources(tuple(nodes), tuple(amps), 15.0, 0.05))
    dt, nst = 2e-3, 2
    U = to_dev(case, case.U0)
    case.op.set_tuning(2)
    case.op.step_faber(U, 0.04, dt, m, nst)
    U1 = to_dev(case, case.U0)
    case.op.set_tuning(1)
    case.op.step_faber(U1, 0.04, dt, m, nst)
    Uref, _, _ = run(prob, "faber", case.U0, 0.04, dt, nst, m=m, p=case.p, ellipse=prob.ellipse())
    assert rel_l2(U.cpu().numpy(), Uref) <= TOL[dtype]
    assert rel_l2(U.cpu().numpy(), U1.cpu().numpy()) <= (1e-13 if dtype == "float64" else 2e-6)


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,fuse", [(2, 2), (3, 3), (7, 3), (8, 4), (16, 0), (13, 4)])
def test_faber_order8_fused_matches_oracle_and_unfused(dtype, m, fuse):
    """The paper's 8th-order stencil in fused passes (tiles of 64 - 8(S - 1)
    columns) over several tiles with ragged edges and sources, against the
    oracle and the one-term path."""
    case = make_case((150, 90), dtype, order=8, seed=81, n_src=2)
    dt, nst = 2e-3, 2
    U = to_dev(case, case.U0)
    case.op.set_tuning(fuse)
    case.op.step_faber(U, 0.04, dt, m, nst)
    U1 = to_dev(case, case.U0)
    case.op.set_tuning(1)
    case.op.step_faber(U1, 0.04, dt, m, nst)
    ref, _, _ = run(case.prob, "faber", case.U0, 0.04, dt, nst, m=m, p=case.p,
                    ellipse=case.prob.ellipse())
    assert rel_l2(U.cpu().numpy(), ref) <= TOL[dtype]
    assert rel_l2(U.cpu().numpy(), U1.cpu().numpy()) <= (1e-13 if dtype == "float64" else 2e-6)


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [(57, 41), (19, 14, 23)])
def test_caller_damping_profiles_match_oracle(dtype, n):
    """Caller-given, non-quadratic damping profiles (Sec. 2) through
    expw_op_create_profiles: H x, Faber steps (default fusion) and Krylov steps
    with a source against the oracle on the same profiles and its own ellipse."""
    import torch
    from oracle.operator import Grid, apply_H
    from oracle.source import PointSources
    from oracle.steppers import Problem
    from paper_2401_16322_amd.expwave import Operator
    from synthetic import layered_velocity, smooth_state
    rng = np.random.default_rng(91)
    profs = []
    for na in n:
        for half in (0.0, 0.5):
            x = (np.arange(na) + half) / (na - 1)
            profs.append(250.0 * rng.uniform(0.5, 1.0) * np.clip(1.0 - 3.0 * x, 0.0, None) ** 3
                         + 60.0 * np.exp(-((x - rng.uniform()) / 0.1) ** 2))
    c2 = layered_velocity(n, 10.0, seed=92) ** 2
    if dtype == "float32":
        c2 = c2.astype(np.float32).astype(np.float64)
    g = Grid(n, 10.0, 4, profiles=tuple(profs))
    node = int(rng.integers(0, g.npts))
    prob = Problem(g, c2, PointSources((node,), (1.0,), 15.0, 0.05))
    tdt = torch.float64 if dtype == "float64" else torch.float32
    op = Operator(n, 10.0, torch.tensor(c2, dtype=tdt, device="cuda"), max_krylov_k=12,
                  max_taylor_p=8, sigma_profiles=profs)
    assert np.allclose(op.ellipse, prob.ellipse(), rtol=1e-12, atol=0.0)
    U0 = smooth_state(n, seed=93, width_cells=max(1.0, min(n) / 8))
    y = op.apply(torch.tensor(U0, dtype=tdt, device="cuda")).cpu().numpy()
    ref = apply_H(g, c2, U0)
    assert np.max(np.abs(y - ref)) <= (1e-13 if dtype == "float64" else 2e-6) * np.max(np.abs(ref))
    op.set_source_ricker([node], [1.0], 15.0, 0.05, 8)
    for method, kw in (("faber", dict(m=12, p=8, ellipse=prob.ellipse())), ("krylov", dict(k=12, p=8))):
        U = torch.tensor(U0, dtype=tdt, device="cuda")
        if method == "faber":
            op.step_faber(U, 0.04, 2e-3, 12, 3)
        else:
            op.step_krylov(U, 0.04, 2e-3, 12, 3)
        Uref, _, _ = run(prob, method, U0, 0.04, 2e-3, 3, **kw)
        assert rel_l2(U.cpu().numpy(), Uref) <= TOL[dtype], method
    op.close()


@pytest.mark.parametrize("path", ["persistent", "launches"])
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("k", [4, 8, 16])
def test_krylov_error_estimate_matches_oracle(dtype, k, path):
    """The a-posteriori estimate of one Krylov step (with a source) against
    the oracle's: FP64 to 1e-8 relative; FP32 to 1e-2 where the estimate is
    above the FP32 rounding of the basis (1e-5 of the state), else below
    that level. The step itself still matches the oracle."""
    from paper_2401_16322_amd.expwave import ExpwError
    from oracle.steppers import krylov_step_estimate
    case = make_case((70, 45), dtype, seed=81, n_src=1, max_k=k)
    case.op.set_krylov_persistent(path == "persistent")
    U = to_dev(case, case.U0)
    case.op.step_krylov(U, 0.05, 2e-3, k, 1)
    with pytest.raises(ExpwError):
        case.op.krylov_estimate()
    case.op.set_krylov_estimate(True)
    U = to_dev(case, case.U0)
    case.op.step_krylov(U, 0.05, 2e-3, k, 1)
    est = case.op.krylov_estimate()
    Uref, eref = krylov_step_estimate(case.prob, case.U0, 0.05, 2e-3, k, p=case.p)
    assert rel_l2(U.cpu().numpy(), Uref) <= TOL[dtype]
    print(f"krylov estimate {dtype} k={k} {path}: {est:.6e} oracle {eref:.6e}")
    if dtype == "float64":
        assert est == pytest.approx(eref, rel=1e-8)
    elif eref >= 1e-5 * np.linalg.norm(Uref):
        assert est == pytest.approx(eref, rel=1e-2)
    else:
        assert est <= 1e-4 * np.linalg.norm(Uref)


def test_krylov_error_estimate_is_the_largest_over_the_steps():
    """Three steps in one call: the reported estimate is the largest of the
    oracle's three per-step estimates (FP64)."""
    from oracle.steppers import krylov_step_estimate
    case = make_case((60, 40), "float64", seed=82, n_src=1, max_k=8)
    case.op.set_krylov_estimate(True)
    U = to_dev(case, case.U0)
    case.op.step_krylov(U, 0.04, 3e-3, 8, 3)
    est = case.op.krylov_estimate()
    Ur, ests = case.U0, []
    for n in range(3):
        Ur, e = krylov_step_estimate(case.prob, Ur, 0.04 + n * 3e-3, 3e-3, 8, p=case.p)
        ests.append(e)
    assert rel_l2(U.cpu().numpy(), Ur) <= 1e-11
    assert est == pytest.approx(max(ests), rel=1e-8)
