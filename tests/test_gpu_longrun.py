"""Whole runs against stored oracle runs.

The stored runs (tests/golden/oracle_*.npz) are written by
tests/golden/make_oracle_runs.py, which calls only the FP64 oracle: each one
advances a workload from rest with its Ricker source by one method (Faber of
degree m or Krylov of dimension k, Sec. 3.2) and keeps the pressure over the
physical domain (or, for the 256^3 grid, three central planes) at fixed
snapshot times. The GPU advances the same workload with the same method,
degree and step in one process, FP32 and FP64, and every snapshot must match
the stored one within 1e-5 (FP32) or 1e-11 (FP64) relative L2. Snapshots
whose reference norm is below 1e-3 of the run's largest are reported but not
gated (the field there has left through the absorbing layer)."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = {"float32": 1e-5, "float64": 1e-11}


def _load(name):
    path = os.path.join(GOLDEN, f"oracle_{name}.npz")
    if not os.path.exists(path):
        # the 256^3 run takes the oracle hours per snapshot; the others are committed
        pytest.skip(f"stored oracle run {path} not generated yet (tests/golden/make_oracle_runs.py {name})")
    with np.load(path, allow_pickle=False) as z:
        meta = json.loads(str(z["meta"]))
        snaps = {k: z[k] for k in z.files if k != "meta"}
    return meta, snaps


def _interior(w, p):
    L = w.abc_cells
    sl = tuple(slice(L, n - L) for n in reversed(w.n))
    return p.reshape(tuple(reversed(w.n)))[sl]


def _planes(w, p):
    f = p.reshape(tuple(reversed(w.n)))
    nz, ny, nx = f.shape
    return [f[nz // 2], f[:, ny // 2, :], f[:, :, nx // 2]]


def _gpu_run(meta, dtype, pass_kernel=0):
    """The GPU's snapshots of the stored run's configuration (numpy float64),
    keyed like the stored ones; pass_kernel picks the fused-pass kernel of
    2D Faber steps (0 automatic, 1 tiled, 2 streamed)."""
    import torch
    from paper_2401_16322_amd.expwave import Operator
    from synthetic import get_workload
    w = get_workload(meta["workload"])
    tdt = torch.float64 if dtype == "float64" else torch.float32
    op = Operator(w.n, w.h, torch.tensor(w.c2(), dtype=tdt, device="cuda"), abc_cells=w.abc_cells,
                  sigma_max=w.sigma_max, max_krylov_k=meta["order"] if meta["method"] == "krylov" else 0,
                  max_taylor_p=meta["taylor_p"])
    op.set_source_ricker([w.source_node()], [1.0], w.f_peak, w.t_delay, meta["taylor_p"])
    op.set_pass_kernel(pass_kernel)
    U = torch.zeros((w.ndim + 1) * w.npts, dtype=tdt, device="cuda")
    dt, every = meta["dt"], meta["snapshot_every"]
    per = int(round(every / dt))
    out = {}
    for k in range(1, meta["snapshots_done"] + 1):
        if meta["method"] == "faber":
            op.step_faber(U, (k - 1) * per * dt, dt, meta["order"], per)
        else:
            op.step_krylov(U, (k - 1) * per * dt, dt, meta["order"], per)
        p = U[: w.npts].double().cpu().numpy()
        if meta["stored"] == "interior":
            out[f"p{k}"] = _interior(w, p)
        else:
            for i, pl in enumerate(_planes(w, p)):
                out[f"p{k}_plane{i}"] = pl
    op.sync()
    op.close()
    return out


def _check(name, dtype, pass_kernel=0):
    meta, ref = _load(name)
    got = _gpu_run(meta, dtype, pass_kernel)
    keys = sorted(ref, key=lambda s: (int(s[1:].split("_")[0]), s))
    norms = {k: float(np.linalg.norm(ref[k])) for k in keys}
    big = max(norms.values())
    errs = {}
    for k in keys:
        errs[k] = float(np.linalg.norm(got[k] - ref[k]) / norms[k]) if norms[k] > 0 else 0.0
    print(f"{name} {dtype} pass kernel {pass_kernel}: " + " ".join(f"{k}={e:.2e}" for k, e in errs.items()),
          flush=True)
    gated = [k for k in keys if norms[k] >= 1e-3 * big]
    assert gated, "no snapshot to gate"
    worst = max(errs[k] for k in gated)
    assert worst <= TOL[dtype], (name, dtype, errs)
    return errs


@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("name,pass_kernel", [
    ("box241_faber16_dt1", 1), ("box241_faber16_dt1", 2), ("box241_faber16_dt2", 1),
    ("box241_faber16_dt2", 2), ("box241_faber24_dt4", 1), ("box241_faber24_dt4", 2),
    ("box241_krylov10_dt2.5", 0)])
def test_small_box_long_runs_match_stored_oracle(name, pass_kernel, dtype):
    """241 x 161 layered box without a layer (its energy stays in the grid),
    T = 2 s: 2000 steps of Faber m = 16 at dt = 1 ms, 1000 at 2 ms, 500 of
    m = 24 at 4 ms (fused passes on the tiled and on the streamed kernel) and
    800 Krylov steps of k = 10 at 2.5 ms, snapshots every 0.25 s (0.2 s at
    4 ms)."""
    _check(name, dtype, pass_kernel)


@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("pass_kernel", [1, 2])
def test_layered_1001x501_whole_run_matches_stored_oracle(dtype, pass_kernel):
    """The 1001 x 501 workload (40-cell layer, source and the bench's Faber
    configuration m = 16, dt = 2 ms) over T = 2 s: 1000 steps, snapshots of
    the physical domain every 0.5 s, on both fused-pass kernels."""
    _check("layered1001_faber16_dt2", dtype, pass_kernel)


@pytest.mark.parametrize("dtype", ["float32", "float64"])
def test_time_to_solution_reference_configuration_matches_stored_oracle(dtype):
    """The configuration of the time-to-solution reference (Faber m = 40,
    dt = 1 ms, 2000 steps over T = 2 s on the 1001 x 501 workload)."""
    _check("layered1001_ref_faber40_dt1", dtype)


@pytest.mark.parametrize("dtype", ["float32", "float64"])
def test_layered3d_256_whole_run_planes_match_stored_oracle(dtype):
    """The 256^3 workload (Faber m = 24, dt = 2.5 ms, source at the centre):
    the three central planes of the pressure every 0.25 s, as far as the
    stored oracle run goes (an oracle step at this size takes about three
    minutes on one core, so the stored run holds the first snapshot,
    t = 0.25 s after 100 steps)."""
    _check("layered3d256_faber24_dt2.5", dtype)


@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("path", [0, 3, 4])
def test_pml_whole_run_matches_stored_oracle(dtype, path):
    """The paper's operator (PML system with a free surface, 8th-order
    stencils) on the 241 x 161 box with a 20-cell PML (beta0 = 200): 500
    Faber steps of m = 16 at dt = 2 ms, the first field over the whole grid
    every 0.25 s, on the automatic path, the two-term pairs and the
    row-streamed passes."""
    import torch
    from paper_2401_16322_amd.expwave import PMLOperator
    from synthetic import get_workload
    meta, ref = _load("pml241_faber16_dt2")
    w = get_workload(meta["workload"])
    nx, ny = w.n
    tdt = torch.float64 if dtype == "float64" else torch.float32
    op = PMLOperator(nx, ny, w.h, torch.tensor(w.c2(), dtype=tdt, device="cuda"), abc_cells=meta["pml_cells"],
                     beta0=meta["beta0"], max_taylor_p=meta["taylor_p"])
    op.set_source_ricker([w.source_node()], [1.0], w.f_peak, w.t_delay, meta["taylor_p"])
    op.set_path(path)
    U = torch.zeros(4 * nx * ny, dtype=tdt, device="cuda")
    dt, per = meta["dt"], int(round(meta["snapshot_every"] / meta["dt"]))
    errs = {}
    for k in range(1, meta["snapshots_done"] + 1):
        op.step_faber(U, (k - 1) * per * dt, dt, meta["order"], per)
        got = U[: nx * ny].double().cpu().numpy().reshape(ny, nx)
        r = ref[f"p{k}"]
        errs[k] = float(np.linalg.norm(got - r) / np.linalg.norm(r))
    op.sync()
    del op
    print(f"pml whole run {dtype} path {path}: " + " ".join(f"p{k}={e:.2e}" for k, e in errs.items()), flush=True)
    assert max(errs.values()) <= TOL[dtype], errs
