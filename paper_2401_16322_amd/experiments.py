"""Single-signal dispersion and dissipation experiment on one GPU
(Sec. 4.2, single signal experiment; metric of Sec. 4.1).

Homogeneous 6 km x 5 km medium (c = 3 km/s, h = 10 m, no absorbing layer), a
15 Hz Ricker source 10 m above the bottom edge and one receiver at mid-depth;
the receiver is sampled every 0.417 ms over [0.6, 1.3] s.
- Faber steps of any size record their terms at the receiver and the samples
  come from the dense output (no change of step size needed).
- Krylov and RK4 follow the sampling protocol of the paper: steps of dt up to
  0.6 s, then steps of 0.417 ms.
The reference is the FP64 Faber path at degree 40 and dt = 0.5 ms (checked
against dt = 1 ms) on the same grid, so the errors here are those of the time
integration only (the paper's reference also changes the grid).

    python -m paper_2401_16322_amd.experiments [dispersion] [--dtype f64|f32]
    python -m paper_2401_16322_amd.experiments gradient [--dtype f32|f64] [--shots N]
    python -m paper_2401_16322_amd.experiments shots [--dtype f32|f64] [--shots N]
print one JSON object each (the second times the inversion gradient, the
third compares batched and shot-by-shot stepping of uneven shots).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

SAMPLE_DT = 0.417e-3
T_SAMPLE0 = 0.6


def _operator(w, dtype, kmax):
    import torch
    from paper_2401_16322_amd.expwave import Operator
    tdt = torch.float64 if dtype == "f64" else torch.float32
    c2 = torch.tensor(w.c2(), dtype=tdt, device="cuda")
    op = Operator(w.n, w.h, c2, abc_cells=w.abc_cells, sigma_max=w.sigma_max,
                  max_krylov_k=kmax, max_taylor_p=w.taylor_p)
    op.set_source_ricker([w.source_node()], [1.0], w.f_peak, w.t_delay, w.taylor_p)
    op.set_receivers(w.receiver_nodes())
    return op, tdt


def sample_times(w):
    n = int(math.floor((w.T - T_SAMPLE0) / SAMPLE_DT + 1e-9)) + 1
    return T_SAMPLE0 + SAMPLE_DT * np.arange(n)


def faber_signal(op, tdt, w, m, dt, ts):
    """Receiver samples at times ts from Faber steps of size dt (dense output)."""
    import torch
    nsteps = int(math.ceil(ts[-1] / dt - 1e-9))
    nrec = w.receiver_nodes().size
    U = torch.zeros((w.ndim + 1) * w.npts, dtype=tdt, device="cuda")
    terms = torch.zeros(nsteps * (m + 1) * nrec, dtype=tdt, device="cuda")
    op.step_faber_dense(U, 0.0, dt, m, nsteps, terms)
    steps = np.minimum(np.floor(ts / dt + 1e-9).astype(np.int64), nsteps - 1)
    taus = np.maximum(ts - steps * dt, 0.0)
    coef = op.dense_coefficients(m, taus)
    out = op.dense_output(m, terms, nsteps, torch.tensor(steps), torch.tensor(coef))
    op.sync()
    return out[:, 0].double().cpu().numpy()


def switched_signal(op, tdt, w, method, order, dt, ts):
    """Steps of dt up to the first sample time, then steps of SAMPLE_DT."""
    import torch
    U = torch.zeros((w.ndim + 1) * w.npts, dtype=tdt, device="cuda")
    nrec = w.receiver_nodes().size

    def advance(t, h, n, traces=None):
        if n <= 0:
            return t
        if method == "krylov":
            op.step_krylov(U, t, h, order, n, traces=traces)
        else:
            op.step_rk4(U, t, h, n, traces=traces)
        return t + n * h

    n1 = int(math.floor(T_SAMPLE0 / dt + 1e-9))
    t = advance(0.0, dt, n1)
    rest = T_SAMPLE0 - n1 * dt
    if rest > 1e-12:
        t = advance(t, rest, 1)
    first = U[w.receiver_nodes()[0]].clone()
    tr = torch.zeros((ts.size - 1) * nrec, dtype=tdt, device="cuda")
    advance(T_SAMPLE0, SAMPLE_DT, ts.size - 1, traces=tr)
    op.sync()
    return np.concatenate([[first.double().item()], tr.view(-1, nrec)[:, 0].double().cpu().numpy()])


def run(dtype="f64", faber_orders=(8, 16, 24, 32, 40), krylov_orders=(10, 20, 30),
        faber_dts_ms=(1, 2, 4, 6, 8, 10), krylov_dts_ms=(1, 2, 4, 6, 8, 10),
        rk4_dts_ms=(0.5, 1.0, 1.5)):
    from paper_2401_16322_amd.analysis import dispersion_dissipation
    from synthetic import get_workload
    w = get_workload("homog2d_single_signal")
    ts = sample_times(w)
    op64, t64 = _operator(w, "f64", 0)
    ref = faber_signal(op64, t64, w, 40, 0.5e-3, ts)
    ref2 = faber_signal(op64, t64, w, 40, 1.0e-3, ts)
    op64.close()
    chk = dispersion_dissipation(ref, ref2, SAMPLE_DT)
    op, tdt = _operator(w, dtype, max(krylov_orders) if krylov_orders else 0)
    rows = []

    def record(method, order, dt_ms, sig, wall):
        if not np.all(np.isfinite(sig)):
            rows.append({"method": method, "order": order, "dt_ms": dt_ms, "diverged": True})
            return
        e = dispersion_dissipation(ref, sig, SAMPLE_DT)
        rows.append({"method": method, "order": order, "dt_ms": dt_ms,
                     "dispersion": e["dispersion"], "dissipation": e["dissipation"],
                     "wall_s": wall})

    for m in faber_orders:
        for d in faber_dts_ms:
            t0 = time.perf_counter()
            sig = faber_signal(op, tdt, w, m, d * 1e-3, ts)
            record("faber", m, d, sig, time.perf_counter() - t0)
    for k in krylov_orders:
        for d in krylov_dts_ms:
            t0 = time.perf_counter()
            sig = switched_signal(op, tdt, w, "krylov", k, d * 1e-3, ts)
            record("krylov", k, d, sig, time.perf_counter() - t0)
    for d in rk4_dts_ms:
        t0 = time.perf_counter()
        sig = switched_signal(op, tdt, w, "rk4", 4, d * 1e-3, ts)
        record("rk4", 4, d, sig, time.perf_counter() - t0)
    op.close()
    return {"experiment": "single signal", "workload": w.name, "dtype": dtype,
            "samples": int(ts.size), "sample_dt_ms": SAMPLE_DT * 1e3,
            "reference": {"method": "faber", "order": 40, "dt_ms": 0.5,
                          "vs_dt_1ms": {"dispersion": chk["dispersion"],
                                        "dissipation": chk["dissipation"]}},
            "runs": rows}


def gradient(dtype="f32", shots=None):
    """Inversion gradient on the 601 x 301 case: observed traces from the true
    model, then the misfit gradient with respect to c^2 at the smoothed start
    model, shot by shot (forward with checkpoints + reverse sweep). Returns the
    timings and the misfit."""
    import torch
    from paper_2401_16322_amd.expwave import Operator
    from paper_2401_16322_amd.fwi import _forward, misfit_gradient
    from synthetic import get_workload, smoothed
    w = get_workload("fwi2d_601x301")
    tdt = torch.float64 if dtype == "f64" else torch.float32
    c_true = w.velocity()
    c_start = smoothed(c_true, w.extra["smooth_cells"])
    nshots = int(shots or w.extra["shots"])
    xs = np.linspace(w.abc_cells + 10, w.n[0] - w.abc_cells - 11, nshots).round().astype(int)
    rec = w.receiver_nodes()
    nsteps = int(round(w.T / w.dt))

    def make(c):
        op = Operator(w.n, w.h, torch.tensor(c ** 2, dtype=tdt, device="cuda"),
                      abc_cells=w.abc_cells, sigma_max=w.sigma_max, max_taylor_p=w.taylor_p)
        op.set_receivers(rec)
        return op

    op_true, op = make(c_true), make(c_start)
    op.ellipse = op_true.ellipse   # one ellipse for both models
    U0 = torch.zeros((w.ndim + 1) * w.npts, dtype=tdt, device="cuda")
    grad = torch.zeros(w.npts, dtype=torch.float64, device="cuda")
    total_L, t_fwd, t_grad = 0.0, 0.0, 0.0
    for x in xs:
        node = w.flat_index((int(x), w.src[1]))
        for o in (op_true, op):
            o.set_source_ricker([node], [1.0], w.f_peak, w.t_delay, w.taylor_p)
        d_obs, _, _ = _forward(op_true, U0, 0.0, w.dt, nsteps, w.faber_m, 1, False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _forward(op, U0, 0.0, w.dt, nsteps, w.faber_m, 1, False)
        torch.cuda.synchronize()
        t_fwd += time.perf_counter() - t0
        t0 = time.perf_counter()
        L, g, _, _ = misfit_gradient(op, U0, 0.0, w.dt, nsteps, w.faber_m, d_obs,
                                     checkpoint_every=w.extra["checkpoint_every"])
        torch.cuda.synchronize()
        t_grad += time.perf_counter() - t0
        grad += g.double()
        total_L += L
    op.sync()
    return {"experiment": "inversion gradient", "workload": w.name, "dtype": dtype,
            "shots": nshots, "steps_per_shot": nsteps, "faber_m": w.faber_m, "dt_ms": w.dt * 1e3,
            "checkpoint_every": w.extra["checkpoint_every"], "misfit": total_L,
            "grad_norm": float(torch.linalg.vector_norm(grad)),
            "forward_s_per_shot": t_fwd / nshots, "gradient_s_per_shot": t_grad / nshots,
            "gradient_over_forward": t_grad / t_fwd if t_fwd > 0 else None}


def shots(dtype="f32", nshots=64, steps=20, seed0=4000):
    """Many uneven 2D shots: nx ~ U[200, 1000], nz ~ U[200, 500], Faber degree
    ~ U{12..32}, a layered model per shot (seed seed0 + s), the source at the
    surface centre, receivers on row 42. The same steps run (a) shot by shot
    with each operator's default (fused) path and (b) as one batch; returns
    both rates in grid-point matrix-vector products per second."""
    import torch
    from paper_2401_16322_amd.expwave import Batch, Operator
    from synthetic import layered_velocity
    rng = np.random.default_rng(seed0)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    ops, states, ms, dts, npts = [], [], [], [], []
    for s_ in range(nshots):
        nx, nz = int(rng.integers(200, 1001)), int(rng.integers(200, 501))
        m = int(rng.integers(12, 33))
        c = layered_velocity((nx, nz), 10.0, seed0 + s_)
        op = Operator((nx, nz), 10.0, torch.tensor(c ** 2, dtype=tdt, device="cuda"),
                      abc_cells=40, sigma_max=300.0, max_taylor_p=8)
        op.set_source_ricker([nx // 2 + 42 * nx], [1.0], 15.0, 0.18, 8)
        op.set_receivers(np.arange(nx, dtype=np.int64) + 42 * nx)
        # a step a little below the degree's reach (about 0.16 ms per term)
        ops.append(op)
        ms.append(m)
        dts.append(1.6e-4 * m)
        npts.append(nx * nz)
        states.append(torch.zeros(3 * nx * nz, dtype=tdt, device="cuda"))
    work = sum(n * m for n, m in zip(npts, ms)) * steps

    def sequential():
        for st in range(steps):
            for op, S, m, dt in zip(ops, states, ms, dts):
                op.step_faber(S, st * dt, dt, m, 1)

    sequential()  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sequential()
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    b = Batch(ops, ms, dts, states)
    b.step(0.0, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(0.0, steps, step0=2)
    torch.cuda.synchronize()
    t_bat = time.perf_counter() - t0
    b.capture(steps)
    b.step(0.0, steps, step0=2 + steps)   # first replay (warm-up)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(0.0, steps, step0=2 + 2 * steps)
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - t0
    for S in states:
        if not torch.isfinite(S).all():
            raise RuntimeError("non-finite state")
    b.close()
    return {"experiment": "uneven shots", "dtype": dtype, "shots": nshots, "steps": steps,
            "points": int(sum(npts)), "degrees": [min(ms), max(ms), float(np.mean(ms))],
            "sequential_s": t_seq, "batched_s": t_bat, "batched_graph_s": t_graph,
            "batched_graph_grid_pt_matvecs_per_s": work / t_graph,
            "sequential_grid_pt_matvecs_per_s": work / t_seq,
            "batched_grid_pt_matvecs_per_s": work / t_bat,
            "launches_per_step": {"sequential": int(sum(math.ceil(m / 4) for m in ms)),
                                  "batched": int(math.ceil(max(ms) / 4))}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="?", default="dispersion",
                    choices=["dispersion", "gradient", "shots"])
    ap.add_argument("--dtype", default=None, choices=["f32", "f64"])
    ap.add_argument("--shots", type=int, default=None)
    args = ap.parse_args()
    if args.which == "dispersion":
        out = run(args.dtype or "f64")
    elif args.which == "gradient":
        out = gradient(args.dtype or "f32", args.shots)
    else:
        out = shots(args.dtype or "f32", args.shots or 64)
    print(json.dumps(out, allow_nan=False), flush=True)


if __name__ == "__main__":
    main()
