"""Throughput bench of the exponential wave-propagation hot path on one GPU.

One bench step is one pass of the whole hot path over the 1001 x 501 layered
medium (40-cell damping layer, 15 Hz Ricker source, receivers on the surface
row), each method advancing its own wavefield by one step with source
injection and receiver recording:
  - Faber, degree m (default 16, dt = 2 ms), in fused multi-term sweeps;
  - Krylov (Arnoldi + Hessenberg exponential), dimension k (default 16, dt = 2 ms);
  - RK4 (dt = 1 ms) and staggered leap-frog (dt = 1 ms) baselines.
value = grid points x matrix-vector products of H / wall second over the
timed steps. The roofline object describes the kernel class with the largest
share of kernel time, timed per launch with HIP events on the launch stream.
The CPU baseline times the FP64 oracle on a bounded number of the same steps.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
METRIC = "grid-pt matvecs/s + HBM % of peak; time-to-solution at 1e-5 rel. L2 error"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="layered2d_1001x501")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--faber-m", type=int, default=0, help="0 = the workload's degree")
    ap.add_argument("--krylov-k", type=int, default=16)
    ap.add_argument("--fuse", type=int, default=0)
    ap.add_argument("--methods", default="faber,krylov,rk4,leapfrog")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run a plain device copy of this size first (HBM counter calibration)")
    ap.add_argument("--cpu-steps", type=int, default=4,
                    help="oracle steps timed for the CPU baseline (0 = skip)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2401_16322_amd import expwave as xw
    if not os.path.exists(xw.LIB_PATH):
        from paper_2401_16322_amd.build_native import build
        build()
    from synthetic import get_workload

    w = get_workload(args.workload)
    if args.faber_m == 0:
        args.faber_m = w.faber_m
    methods = [m for m in args.methods.split(",") if m]
    tdt = torch.float32 if args.dtype == "f32" else torch.float64
    dev = torch.device("cuda:0")
    c2_np = w.velocity() ** 2
    c2 = torch.tensor(c2_np, dtype=tdt, device=dev)
    op = xw.Operator(w.n, w.h, c2, abc_cells=w.abc_cells, sigma_max=w.sigma_max,
                     max_krylov_k=max(args.krylov_k, 1), max_taylor_p=w.taylor_p)
    op.set_tuning(args.fuse)
    src = w.source_node()
    op.set_source_ricker([src], [1.0], w.f_peak, w.t_delay, w.taylor_p)
    rec = w.receiver_nodes()
    op.set_receivers(rec)
    npts = w.npts
    if args.calib_copy_mb > 0:
        nel = args.calib_copy_mb * (1 << 20) // 4
        a_ = torch.ones(nel, dtype=torch.float32, device=dev)
        b_ = torch.empty_like(a_)
        for _ in range(3):
            b_.copy_(a_)
        torch.cuda.synchronize()
        del a_, b_
    nstate = (w.ndim + 1) * npts

    dts = {"faber": w.dt, "krylov": min(w.dt, 2e-3), "rk4": 1e-3, "leapfrog": 1e-3}
    mvos = {"faber": args.faber_m, "krylov": args.krylov_k, "rk4": 4, "leapfrog": 1}
    states = {m: torch.zeros(nstate, dtype=tdt, device=dev) for m in methods}
    total_steps = args.warmup + args.steps
    traces = {m: torch.zeros(total_steps * max(rec.size, 1), dtype=tdt, device=dev) for m in methods}
    tcur = {m: 0.0 for m in methods}
    counter = {m: 0 for m in methods}

    def one(m):
        tr = traces[m][counter[m] * rec.size:] if rec.size else None
        if m == "faber":
            op.step_faber(states[m], tcur[m], dts[m], args.faber_m, 1, traces=tr)
        elif m == "krylov":
            op.step_krylov(states[m], tcur[m], dts[m], args.krylov_k, 1, traces=tr)
        elif m == "rk4":
            op.step_rk4(states[m], tcur[m], dts[m], 1, traces=tr)
        else:
            op.step_leapfrog(states[m], tcur[m], dts[m], 1, traces=tr)
        tcur[m] += dts[m]
        counter[m] += 1

    def step():
        for m in methods:
            one(m)

    # warm-up steps; the last one times every kernel class to find the dominant one
    for i in range(args.warmup):
        if i == args.warmup - 1:
            torch.cuda.synchronize()
            op.set_timing(None)
        step()
    torch.cuda.synchronize()
    kt_warm = op.timing()
    dom = max(kt_warm, key=lambda k: kt_warm[k][0])
    # timed region: HIP events only around launches of the dominant kernel class
    op.set_timing([dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt = op.timing()
    for m in methods:
        if not torch.isfinite(states[m]).all():
            raise RuntimeError(f"{m}: non-finite wavefield")

    mv_per_step = sum(mvos[m] for m in methods)
    value = npts * mv_per_step * args.steps / elapsed
    # the dominant kernel class and its achieved algorithmic bandwidth (timed region)
    ms, launches, nbytes = kt[dom]
    achieved = nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    # per-class table and per-method rates from the instrumented warm-up step
    kernels = {k: {"ms": round(v[0], 4), "launches": v[1],
                   "avg_us": round(1e3 * v[0] / v[1], 3) if v[1] else None,
                   "GB_per_s": round(v[2] / (v[0] * 1e-3) / 1e9, 1) if v[0] > 0 else None}
               for k, v in kt_warm.items() if v[1]}
    cls = {"faber": ["faber"], "krylov": ["krylov_matvec", "krylov_mgs", "krylov_aux", "krylov_arnoldi"],
           "rk4": ["rk4"], "leapfrog": ["leapfrog_v", "leapfrog_p"]}
    per_method = {}
    for m in methods:
        kms = sum(kt_warm[c][0] for c in cls[m])
        per_method[m] = {"dt_ms": dts[m] * 1e3, "mvo_per_step": mvos[m],
                         "kernel_ms_per_step": round(kms, 4),
                         "kernel_grid_pt_matvecs_per_s":
                             (npts * mvos[m] / (kms * 1e-3)) if kms > 0 else None}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "grid-pt matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": w.name, "grid": list(w.n), "h_m": w.h, "abc_cells": w.abc_cells,
                   "methods": {m: {"dt_ms": dts[m] * 1e3, "mvo": mvos[m]} for m in methods},
                   "receivers": int(rec.size), "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None, "avg_launch_us": round(1e3 * ms / launches, 3),
                     "launches": launches},
        "methods": per_method,
        "kernels": kernels,
    }
    if args.cpu_steps > 0:
        out["cpu_baseline"] = cpu_baseline(w, methods, mvos, dts, args, c2_np, rec)
    print(json.dumps(out), flush=True)


def cpu_baseline(w, methods, mvos, dts, args, c2_np, rec):
    """The FP64 oracle on the same composite step, single-threaded."""
    from threadpoolctl import threadpool_limits
    from oracle.operator import Grid
    from oracle.source import PointSources
    from oracle.steppers import Problem, step
    g = Grid(w.n, w.h, 4, abc_cells=w.abc_cells, sigma_max=w.sigma_max)
    prob = Problem(g, c2_np, PointSources((w.source_node(),), (1.0,), w.f_peak, w.t_delay))
    ell = prob.ellipse()
    states = {m: np.zeros(g.nstate) for m in methods}
    kw = {"faber": dict(m=args.faber_m, p=w.taylor_p, ellipse=ell),
          "krylov": dict(k=args.krylov_k, p=w.taylor_p)}
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for s in range(args.cpu_steps):
            for m in methods:
                states[m] = step(prob, m, states[m], s * dts[m], dts[m], **kw.get(m, {}))
                _ = states[m][rec]
        el = time.perf_counter() - t0
    total = w.npts * sum(mvos[m] for m in methods) * args.cpu_steps
    return {"value": total / el, "unit": "grid-pt matvecs/s", "cores": 1, "kind": "oracle",
            "sample": f"{args.cpu_steps} composite steps ({'+'.join(methods)}) of {w.name}, "
                      f"FP64 numpy, {el:.1f} s"}


if __name__ == "__main__":
    main()
