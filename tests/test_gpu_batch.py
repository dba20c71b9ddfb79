"""Batched Faber steps of several shots against one-shot steps and the oracle."""
import numpy as np
import pytest

from gpu_cases import TOL, make_case, rel_l2, to_dev
from oracle.steppers import run

pytestmark = pytest.mark.gpu
DTYPES = ["float64", "float32"]


def _shots(dtype, dims):
    cases = []
    for i, n in enumerate(dims):
        c = make_case(n, dtype, seed=50 + i, n_src=1 + i % 2, abc=3)
        g = c.prob.grid
        rec = np.unique(np.linspace(0, g.npts - 1, 7).astype(np.int64))
        c.op.set_receivers(rec)
        cases.append((c, rec))
    return cases


@pytest.mark.parametrize("dtype", DTYPES)
def test_batch_matches_single_shots_and_oracle(dtype):
    import torch
    from paper_2401_16322_amd.expwave import Batch
    dims = [(90, 40), (33, 71), (128, 65), (20, 18), (257, 30)]
    ms = [2, 3, 16, 7, 12]
    dts = [1e-3, 2e-3, 2e-3, 1.5e-3, 3e-3]
    cases = _shots(dtype, dims)
    nst, t0 = 3, 0.02
    states = [to_dev(c, c.U0) for c, _ in cases]
    traces = [torch.zeros(nst * r.size, dtype=c.torch_dtype, device="cuda") for c, r in cases]
    b = Batch([c.op for c, _ in cases], ms, dts, states, traces)
    b.step(t0, nst)
    torch.cuda.synchronize()
    tight = 1e-13 if dtype == "float64" else 2e-6
    for (c, rec), S, tr, m, dt in zip(cases, states, traces, ms, dts):
        U = to_dev(c, c.U0)
        tr1 = torch.zeros(nst * rec.size, dtype=c.torch_dtype, device="cuda")
        c.op.set_tuning(1)
        c.op.step_faber(U, t0, dt, m, nst, traces=tr1)
        assert rel_l2(S.cpu().numpy(), U.cpu().numpy()) <= tight
        assert rel_l2(tr.cpu().numpy(), tr1.cpu().numpy()) <= tight
    c, rec = cases[2]
    Uref, trref, _ = run(c.prob, "faber", c.U0, t0, dts[2], nst, receivers=rec, m=ms[2], p=c.p,
                         ellipse=c.prob.ellipse())
    assert rel_l2(states[2].cpu().numpy(), Uref) <= TOL[dtype]
    assert rel_l2(traces[2].cpu().numpy().reshape(nst, -1), trref) <= TOL[dtype]
    b.close()


def test_batch_3d_and_trace_offset():
    import torch
    from paper_2401_16322_amd.expwave import Batch
    cases = _shots("float64", [(17, 13, 11), (9, 20, 14)])
    states = [to_dev(c, c.U0) for c, _ in cases]
    traces = [torch.zeros(4 * r.size, dtype=torch.float64, device="cuda") for c, r in cases]
    b = Batch([c.op for c, _ in cases], [5, 8], [2e-3, 1e-3], states, [traces[0], None])
    b.step(0.03, 2, step0=2)          # steps 2 and 3: from 0.03 + 2 dt
    torch.cuda.synchronize()
    for (c, rec), S, m, dt in zip(cases, states, [5, 8], [2e-3, 1e-3]):
        Uref, _, _ = run(c.prob, "faber", c.U0, 0.03 + 2 * dt, dt, 2, m=m, p=c.p,
                         ellipse=c.prob.ellipse())
        assert rel_l2(S.cpu().numpy(), Uref) <= 1e-11
    t = traces[0].cpu().numpy().reshape(4, -1)
    assert not np.any(t[:2]) and np.all(np.isfinite(t[2:])) and np.any(t[2:])
    assert not np.any(traces[1].cpu().numpy())
    b.close()


def test_batch_validation():
    import torch
    from paper_2401_16322_amd.expwave import Batch, ExpwError
    a = make_case((20, 10), "float64", seed=60)
    b = make_case((20, 10), "float32", seed=61)
    sa, sb = to_dev(a, a.U0), to_dev(b, b.U0)
    with pytest.raises(ExpwError):
        Batch([a.op, b.op], [4, 4], [1e-3, 1e-3], [sa, sb])       # mixed dtype
    with pytest.raises(ExpwError):
        Batch([a.op], [1], [1e-3], [sa])                        # degree < 2
    c = make_case((20, 10), "float64", seed=62)
    with pytest.raises(ExpwError):
        Batch([a.op, c.op], [4, 4], [1e-3, 1e-3], [sa, sa])     # shared state


def test_autotune_picks_and_caches_a_choice_with_the_same_results(tmp_path):
    """The library's autotuner times the depths and pass kernels, keeps the
    fastest, appends it to the cache file, and a second operator of the same
    layout takes it from the cache without timing; any choice gives the same
    step (rounding order aside)."""
    cache = tmp_path / "tune.txt"
    case = make_case((300, 140), "float32", seed=70)
    fz, pk, ms = case.op.autotune(16, 2e-3, cache_path=str(cache))
    assert 1 <= fz <= 6 and pk in (0, 1, 2) and ms > 0
    assert case.op.fuse == fz
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and lines[0].split()[-3:-1] == [str(fz), str(pk)]
    other = make_case((300, 140), "float32", seed=71)
    assert other.op.autotune(16, 2e-3, cache_path=str(cache)) == (fz, pk, pytest.approx(ms, rel=1e-5))
    assert len(cache.read_text().splitlines()) == 1
    U = to_dev(case, case.U0)
    case.op.step_faber(U, 0.0, 2e-3, 16, 2)
    case.op.set_tuning(1)
    V = to_dev(case, case.U0)
    case.op.step_faber(V, 0.0, 2e-3, 16, 2)
    assert rel_l2(U.cpu().numpy(), V.cpu().numpy()) <= 2e-6


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("depth", [2, 4, 6])
def test_batch_depths_and_persistent_launch(dtype, depth):
    """Batches run passes of the depth set on shot 0's operator (6 becomes 4
    in FP64); one cooperative launch per step gives the per-pass launches'
    states and traces bit for bit; both match single shots and the oracle.
    Degrees 2 and 3 make one-pass shots (copied into the state) for depth
    >= 4."""
    import torch
    from paper_2401_16322_amd.expwave import Batch
    dims = [(90, 40), (33, 71), (128, 65), (20, 18), (257, 30)]
    ms = [2, 3, 16, 7, 12]
    dts = [1e-3, 2e-3, 2e-3, 1.5e-3, 3e-3]
    nst, t0 = 3, 0.02
    runs = []
    for persistent in (False, True):
        cases = _shots(dtype, dims)
        cases[0][0].op.set_tuning(depth)
        states = [to_dev(c, c.U0) for c, _ in cases]
        traces = [torch.zeros(nst * r.size, dtype=c.torch_dtype, device="cuda") for c, r in cases]
        b = Batch([c.op for c, _ in cases], ms, dts, states, traces)
        if persistent:
            b.set_persistent(True)
        b.step(t0, 1)
        b.step(t0, nst - 1, step0=1)
        torch.cuda.synchronize()
        runs.append(([S.cpu().numpy() for S in states], [t.cpu().numpy() for t in traces]))
        b.close()
    for a, c_ in zip(runs[0][0] + runs[0][1], runs[1][0] + runs[1][1]):
        assert np.array_equal(a, c_)
    tight = 1e-13 if dtype == "float64" else 2e-6
    cases = _shots(dtype, dims)
    for (c, rec), S, tr, m, dt in zip(cases, runs[1][0], runs[1][1], ms, dts):
        U = to_dev(c, c.U0)
        tr1 = torch.zeros(nst * rec.size, dtype=c.torch_dtype, device="cuda")
        c.op.set_tuning(1)
        c.op.step_faber(U, t0, dt, m, nst, traces=tr1)
        assert rel_l2(S, U.cpu().numpy()) <= tight
        assert rel_l2(tr, tr1.cpu().numpy()) <= tight
    c, rec = cases[2]
    Uref, trref, _ = run(c.prob, "faber", c.U0, t0, dts[2], nst, receivers=rec, m=ms[2], p=c.p,
                         ellipse=c.prob.ellipse())
    assert rel_l2(runs[1][0][2], Uref) <= TOL[dtype]
    assert rel_l2(runs[1][1][2].reshape(nst, -1), trref) <= TOL[dtype]


def test_persistent_batch_rejects_unsupported_shots():
    from paper_2401_16322_amd.expwave import Batch, ExpwError
    cases = _shots("float64", [(17, 13, 11), (9, 20, 14)])
    states = [to_dev(c, c.U0) for c, _ in cases]
    b = Batch([c.op for c, _ in cases], [5, 8], [2e-3, 1e-3], states)
    with pytest.raises(ExpwError):
        b.set_persistent(True)
    b.close()


@pytest.mark.parametrize("dtype", DTYPES)
def test_batch_graph_replays_match_eager(dtype):
    """A captured 2-step graph replayed three times (eager work and
    synchronisations between the replays) gives the same states and traces
    as the same steps launched eagerly, bit for bit, after every replay; a
    remainder step after the replays runs eagerly."""
    import torch
    from paper_2401_16322_amd.expwave import Batch
    dims = [(90, 40), (64, 33), (120, 50)]
    ms, dts = [3, 9, 16], [1e-3, 2e-3, 2e-3]
    A = _shots(dtype, dims)
    B = _shots(dtype, dims)
    sa = [to_dev(c, c.U0) for c, _ in A]
    sb = [to_dev(c, c.U0) for c, _ in B]
    ta = [torch.zeros(7 * r.size, dtype=c.torch_dtype, device="cuda") for c, r in A]
    tb = [torch.zeros(7 * r.size, dtype=c.torch_dtype, device="cuda") for c, r in B]
    ga = Batch([c.op for c, _ in A], ms, dts, sa, ta)
    eb = Batch([c.op for c, _ in B], ms, dts, sb, tb)
    ga.capture(2)
    for rep in range(3):
        ga.step(0.02, 2, step0=2 * rep)          # one graph replay
        eb.step(0.02, 1, step0=2 * rep)          # the same two steps, eagerly
        eb.step(0.02, 1, step0=2 * rep + 1)
        torch.cuda.synchronize()
        x = torch.randn(4096, device="cuda")     # eager work between replays
        float((x * x).sum())
        torch.cuda.synchronize()
        for u, v in zip(sa + ta, sb + tb):
            assert torch.equal(u, v)
    ga.step(0.02, 1, step0=6)                    # shorter than the graph: eager
    eb.step(0.02, 1, step0=6)
    torch.cuda.synchronize()
    for u, v in zip(sa + ta, sb + tb):
        assert torch.equal(u, v)
    # and the eager batch itself matches one-shot stepping after 7 steps
    tight = 1e-13 if dtype == "float64" else 2e-6
    for (c, rec), S, m, dt in zip(B, sb, ms, dts):
        U = to_dev(c, c.U0)
        c.op.set_tuning(1)
        c.op.step_faber(U, 0.02, dt, m, 7)
        assert rel_l2(S.cpu().numpy(), U.cpu().numpy()) <= tight
    ga.close()
    eb.close()
