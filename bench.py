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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
CSRC = os.path.join(ROOT, "paper_2401_16322_amd", "csrc")


# the sources each timed kernel class is compiled from (its own header and
# the device headers it includes)
KERNEL_SOURCES = {
    "krylov_arnoldi": ("arnoldi.h", "device_common.h", "kernels.h"),
    "faber": ("fused.h", "fused3d.h", "stream2d.h", "term_zero.h", "device_common.h", "kernels.h"),
    "pml_faber_pair": ("pml.h", "device_common.h"),
    "pml_faber_stream": ("pml_stream.h", "pml.h", "device_common.h", "kernels.h"),
    "pml_faber_term": ("pml.h", "device_common.h"),
}


def kernel_sources_digest(kernel):
    """sha256 over the sources of one kernel class (names and contents)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(kernel, tuple(sorted(os.listdir(CSRC)))):
        h.update(f.encode())
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, workload, dtype):
    """HBM bytes per launch of a kernel class from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE, calibrated against a plain copy), or
    None when there is none for this case or the kernels changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    digest = kernel_sources_digest(kernel)
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            f = line.split()
            if len(f) == 5 and not line.startswith("#") and f[:3] == [kernel, workload, dtype]:
                return float(f[3]) if f[4] == digest else None
    return None
METRIC = "grid-pt matvecs/s + HBM % of peak; time-to-solution at 1e-5 rel. L2 error"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="layered3d_256")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--faber-m", type=int, default=0, help="0 = the workload's degree")
    ap.add_argument("--krylov-k", type=int, default=16)
    ap.add_argument("--fuse", type=int, default=0)
    ap.add_argument("--order", type=int, default=4, choices=[4, 8],
                    help="stencil order (4: the workloads' stencil; 8: the paper's)")
    ap.add_argument("--methods", default="",
                    help="comma list of faber,krylov,rk4,leapfrog (default: faber in 3D, all in 2D)")
    ap.add_argument("--pml-path", type=int, default=0,
                    help="PML term kernel: 0 automatic, 1 per node, 2 LDS tiles, 3 two terms per pass, "
                         "4 row-streamed passes")
    ap.add_argument("--operator", default="pv", choices=["pv", "pml"],
                    help="pv: the first-order p/v operator (the composite step); pml: "
                         "Faber steps on the paper's PML system with a free surface")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run a plain device copy of this size first (HBM counter calibration)")
    ap.add_argument("--cpu-steps", type=int, default=24,
                    help="oracle steps timed for the CPU baseline (0 = skip)")
    ap.add_argument("--tts", type=int, default=1,
                    help="1 = also measure time-to-solution at --tts-tol over the full simulated time")
    ap.add_argument("--tts-tol", type=float, default=1e-5)
    ap.add_argument("--tts-workload", default="layered2d_1001x501",
                    help="workload of the time-to-solution measurement (its oracle reference is stored)")
    ap.add_argument("--tts-dtypes", default="f32,f64")
    ap.add_argument("--tts-repeats", type=int, default=3)
    return ap.parse_args()


def bench_pml(args, w):
    """Faber steps on the paper's own operator (2D PML system, free surface at
    row 0): the workload's grid, medium, layer (delta = abc_cells h, beta_0 =
    sigma_max), source (on v) and receivers (u); state starts at rest."""
    import torch
    from paper_2401_16322_amd import expwave as xw
    if len(w.n) != 2:
        raise SystemExit("the PML operator is 2D")
    tdt = torch.float32 if args.dtype == "f32" else torch.float64
    dev = torch.device("cuda:0")
    nx, ny = w.n
    c2 = torch.tensor(w.c2(), dtype=tdt, device=dev)
    op = xw.PMLOperator(nx, ny, w.h, c2, abc_cells=w.abc_cells, beta0=w.sigma_max,
                        max_taylor_p=w.taylor_p)
    op.set_source_ricker([w.source_node()], [1.0], w.f_peak, w.t_delay, w.taylor_p)
    op.set_path(args.pml_path)
    rec = w.receiver_nodes()
    op.set_receivers(rec)
    m, dt = args.faber_m, w.dt
    if args.calib_copy_mb > 0:
        nel = args.calib_copy_mb * (1 << 20) // 4
        a_ = torch.ones(nel, dtype=torch.float32, device=dev)
        b_ = torch.empty_like(a_)
        for _ in range(3):
            b_.copy_(a_)
        torch.cuda.synchronize()
        del a_, b_
    U = torch.zeros(4 * nx * ny, dtype=tdt, device=dev)
    tr = torch.zeros(max(args.steps, args.warmup, 1) * len(rec), dtype=tdt, device=dev)
    op.step_faber(U, 0.0, dt, m, args.warmup, traces=tr)
    op.sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    op.step_faber(U, args.warmup * dt, dt, m, args.steps, traces=tr)
    e1.record()
    op.sync()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    if not bool(torch.isfinite(U).all()):
        raise RuntimeError("pml: non-finite wavefield")
    npts = nx * ny
    es = 4 if args.dtype == "f32" else 8
    # algorithmic bytes per point per step (four fields of es bytes: reads of
    # v_{j-1}, v_{j-2} and c^2, writes of the new terms; the partial sum is FP64,
    # 32 B read and 32 B written per pass), by term kernel
    path = op.path_for(m)
    if path in (3, 4) and m >= 2:
        # passes of several terms (pairs; row-streamed passes of up to 4 terms at
        # FP32 and 2 at FP64, as evenly sized as their count allows): the first
        # pass reads v_0 and c^2 and writes the last two terms and the sum
        # (13 es + 32; 9 es if it is also the last); middle passes 17 es + 64; a
        # last pass, or a last single term, 13 es + 32
        smax = 2 if path == 3 else (4 if args.dtype == "f32" else 2)
        npass = -(-m // smax)
        bpp = 9 * es if npass == 1 else 2 * (13 * es + 32) + (17 * es + 64) * (npass - 2)
    else:
        # one term per sweep: first term 9 es + 32, middle terms 17 es + 64, last
        # term 13 es + 32 (a single term 9 es)
        npass = m
        bpp = (9 * es + 32) + (17 * es + 64) * (m - 2) + (13 * es + 32) if m >= 2 else 9 * es
    gbps = bpp * npts * args.steps / (ms * 1e-3) / 1e9
    kclass = {3: "pml_faber_pair", 4: "pml_faber_stream"}.get(path, "pml_faber_term")
    out = {
        "metric": "grid-pt matvecs/s", "value": npts * m * args.steps / (ms * 1e-3),
        "unit": "grid-pt matvecs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": args.workload, "operator": "pml", "term_kernel": path,
                   "grid": [nx, ny], "faber_m": m,
                   "dt_ms": dt * 1e3, "abc_cells": w.abc_cells, "beta0": w.sigma_max},
        "roofline": {"bound": "hbm", "kernel": kclass,
                     "achieved": round(gbps, 1),
                     "peak": 8000.0, "unit": "GB/s", "frac": round(gbps / 8000.0, 4),
                     "traffic": measured_traffic(kclass, w.name, args.dtype),
                     "traffic_unit": "HBM bytes per launch, mean over the passes of a step "
                                     "(rocprofv3 counters, copy-calibrated)",
                     "avg_term_us": round(ms * 1e3 / (args.steps * m), 3),
                     "passes_per_step": npass,
                     "avg_pass_us": round(ms * 1e3 / (args.steps * npass), 3)},
    }
    if args.cpu_steps > 0:
        out["cpu_baseline"] = cpu_baseline_pml(w, args, c2.double().cpu().numpy())
    if args.tts:
        out["time_to_solution"] = pml_time_to_solution(w, args)
    print(json.dumps(out, allow_nan=False), flush=True)


def cpu_baseline_pml(w, args, c2_np):
    """The FP64 oracle's Faber steps on the PML operator (same grid, medium,
    layer, source, degree and dt), single-threaded, on a bounded number of
    steps (a quarter of --cpu-steps, at least 1)."""
    from threadpoolctl import threadpool_limits
    from oracle import pml as opml
    from oracle.steppers import faber_step
    nx, ny = w.n
    g = opml.PMLGrid(nx, ny, w.h, abc_cells=w.abc_cells, beta0=w.sigma_max)
    prob = opml.PMLProblem(g, c2_np, opml.PMLSources((w.source_node(),), (1.0,), w.f_peak, w.t_delay))
    ell = prob.ellipse()
    nsteps = max(1, args.cpu_steps // 4)
    U = np.zeros(g.nstate)
    rec = np.asarray(w.receiver_nodes())
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for s in range(nsteps):
            U = faber_step(prob, U, s * w.dt, w.dt, args.faber_m, p=w.taylor_p, ellipse=ell)
            _ = U[rec]
        el = time.perf_counter() - t0
    total = nx * ny * args.faber_m * nsteps
    return {"value": total / el, "unit": "grid-pt matvecs/s", "cores": 1, "kind": "oracle",
            "host_cpu": host_cpu(),
            "sample": f"{nsteps} Faber steps (m = {args.faber_m}) of the PML operator on {w.name}, "
                      f"FP64 numpy, {el:.1f} s"}


PML_TTS_CANDIDATES = (("faber", 8), ("faber", 16), ("faber", 24), ("faber", 32), ("faber", 40),
                      ("krylov", 10), ("krylov", 20), ("krylov", 30), ("krylov", 40), ("rk4", 4))


def pml_time_to_solution(w, args):
    """Time to solution on the PML operator (Faber, Krylov, RK4): the largest dt of the
    ladder whose displacement snapshots every 0.5 s up to the final time stay
    within tol (relative L2 of u over the physical domain: the layers on the
    sides and the bottom excluded, the free-surface rows included) of an FP64
    reference (Faber degree 40, dt = 0.5 ms, checked against dt = 1 ms), and the
    wall time of that run (receiver recording included)."""
    import torch
    from paper_2401_16322_amd import expwave as xw
    dev = torch.device("cuda:0")
    nx, ny = w.n
    L, T, snap_every = w.abc_cells, w.T, 0.5
    nsnap = int(round(T / snap_every))
    rec = w.receiver_nodes()
    c2_np = w.c2()

    kmax = max(k for m_, k in PML_TTS_CANDIDATES if m_ == "krylov")

    def make_op(tdt):
        op = xw.PMLOperator(nx, ny, w.h, torch.tensor(c2_np, dtype=tdt, device=dev),
                            abc_cells=w.abc_cells, beta0=w.sigma_max, max_taylor_p=w.taylor_p,
                            max_krylov_k=kmax)
        op.set_source_ricker([w.source_node()], [1.0], w.f_peak, w.t_delay, w.taylor_p)
        op.set_receivers(rec)
        return op

    def interior(state):
        return state[:nx * ny].view(ny, nx)[: ny - L, L: nx - L].double()

    def run(op, tdt, method, m, dt, ref=None, tol=None):
        state = torch.zeros(4 * nx * ny, dtype=tdt, device=dev)
        nper = int(round(snap_every / dt))
        traces = torch.zeros(nper * max(rec.size, 1), dtype=tdt, device=dev)
        snaps, err = [], 0.0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s_ in range(nsnap):
            tr = traces if rec.size else None
            if method == "faber":
                op.step_faber(state, s_ * snap_every, dt, m, nper, traces=tr)
            elif method == "krylov":
                op.step_krylov(state, s_ * snap_every, dt, m, nper, traces=tr)
            else:
                op.step_rk4(state, s_ * snap_every, dt, nper, traces=tr)
            if ref is None:
                snaps.append(interior(state).clone())
            else:
                torch.cuda.synchronize()
                t_pause = time.perf_counter()
                r = ref[s_]
                e = (torch.linalg.vector_norm(interior(state) - r) / torch.linalg.vector_norm(r)).item()
                err = max(err, e if np.isfinite(e) else float("inf"))
                t0 += time.perf_counter() - t_pause
                if err > tol:
                    break
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        op.sync()
        return err, wall, snaps

    op64 = make_op(torch.float64)
    _, _, ref = run(op64, torch.float64, "faber", 40, 0.5e-3)
    _, _, ref2 = run(op64, torch.float64, "faber", 40, 1.0e-3)
    ref_check = max((torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(a)).item()
                    for a, b in zip(ref, ref2))
    del op64
    out = {"tol": args.tts_tol, "T_s": T, "snapshots_s": [snap_every * (i + 1) for i in range(nsnap)],
           "error": "relative L2 of u over the physical domain (free-surface rows included), max over snapshots",
           "reference": {"method": "faber", "order": 40, "dt_ms": 0.5, "dtype": "f64", "vs_dt_1ms": ref_check},
           "dt_ladder_ms": list(TTS_DTS_MS)}
    for dname in [d for d in args.tts_dtypes.split(",") if d]:
        tdt = {"f32": torch.float32, "f64": torch.float64}[dname]
        op = make_op(tdt)
        results = []
        for method, m in PML_TTS_CANDIDATES:
            best, tried = None, []
            for dt_ms in TTS_DTS_MS:
                dt = dt_ms * 1e-3
                err, _, _ = run(op, tdt, method, m, dt, ref=ref, tol=args.tts_tol)
                tried.append([dt_ms, float(f"{err:.3g}") if np.isfinite(err) else None])
                if err <= args.tts_tol:
                    walls = [run(op, tdt, method, m, dt, ref=ref, tol=args.tts_tol)[1]
                             for _ in range(args.tts_repeats)]
                    nsteps = int(round(T / dt))
                    best = {"method": method, "order": m, "dt_ms": dt_ms, "max_rel_l2": err,
                            "wall_s": float(np.median(walls)), "n_steps": nsteps, "n_op": nsteps * m,
                            "n_mem": nsteps}
                    break
            r = best if best else {"method": method, "order": m, "dt_ms": None}
            r["tried"] = tried
            results.append(r)
        del op
        ok = [r for r in results if r.get("dt_ms")]
        out[dname] = {"runs": results, "fastest": min(ok, key=lambda r: r["wall_s"]) if ok else None}
    return out


def host_cpu():
    """CPU model name and the host's logical CPU count."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "os_cpu_count": os.cpu_count()}


def ceiling(nbytes=1 << 30, reps=10):
    """Measured HBM ceiling: the library's plain stream kernels (read, copy,
    triad) over 1 GiB arrays, plain and non-temporal, in GB/s."""
    from paper_2401_16322_amd import expwave as xw
    return {k: round(v, 1) for k, v in xw.stream_ceiling(nbytes, reps).items()}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
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
    if args.operator == "pml":
        return bench_pml(args, w)
    if not args.methods:
        # the 3D workload is stated for Faber; the 2D ones step every method
        args.methods = "faber" if w.ndim == 3 else "faber,krylov,rk4,leapfrog"
    methods = [m for m in args.methods.split(",") if m]
    tdt = torch.float32 if args.dtype == "f32" else torch.float64
    dev = torch.device("cuda:0")
    c2_np = w.c2()
    c2 = torch.tensor(c2_np, dtype=tdt, device=dev)
    kmax = max(args.krylov_k, 1) if "krylov" in methods else 0
    op = xw.Operator(w.n, w.h, c2, order=args.order, abc_cells=w.abc_cells,
                     sigma_max=w.sigma_max, max_krylov_k=kmax, max_taylor_p=w.taylor_p)
    try:
        out = bench_steps(args, w, methods, op, c2_np, tdt, dev)
    finally:
        op.close()
    ceil = ceiling()
    out["roofline"]["ceiling_GBps"] = ceil
    best = max(ceil.get("copy", 0.0), ceil.get("copy_nt", 0.0))
    out["roofline"]["frac_of_copy_ceiling"] = round(out["roofline"]["achieved"] / best, 4) if best else None
    if args.tts:
        out["time_to_solution"] = time_to_solution(get_workload(args.tts_workload), args)
    if args.cpu_steps > 0:
        out["cpu_baseline"] = cpu_baseline(w, methods, out["_mvos"], out["_dts"], args, c2_np,
                                           w.receiver_nodes())
    out.pop("_mvos")
    out.pop("_dts")
    print(json.dumps(out, allow_nan=False), flush=True)


def bench_steps(args, w, methods, op, c2_np, tdt, dev):
    """The timed steps of every method on one operator; the bench line
    without the ceiling, time-to-solution and CPU baseline."""
    import torch
    op.set_tuning(args.fuse)
    src = w.source_node()
    op.set_source_ricker([src], [1.0], w.f_peak, w.t_delay, w.taylor_p)
    rec = w.receiver_nodes()
    if rec.size:
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
    traces = {m: (torch.zeros(total_steps * rec.size, dtype=tdt, device=dev) if rec.size else None)
              for m in methods}
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
    # timed region: HIP events attached to the launches of the dominant kernel class
    op.set_timing([dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt = op.timing()
    op.sync()
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
    return {
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
                   "order": args.order,
                   "methods": {m: {"dt_ms": dts[m] * 1e3, "mvo": mvos[m]} for m in methods},
                   "receivers": int(rec.size), "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     # (the counters were taken at order 4 with the automatic tuning)
                     "traffic": (measured_traffic(dom, w.name, args.dtype)
                                 if args.order == 4 and args.fuse == 0 else None),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 counters, copy-calibrated)",
                     "algorithmic_bytes_per_launch": round(nbytes / launches) if launches else None,
                     "avg_launch_us": round(1e3 * ms / launches, 3) if launches else None,
                     "launches": launches},
        "methods": per_method,
        "kernels": kernels,
        "_mvos": mvos,
        "_dts": dts,
    }


# dt ladder (ms): every value divides the 0.5 s snapshot spacing
TTS_DTS_MS = (12.5, 10.0, 5.0, 4.0, 2.5, 2.0, 1.0, 0.5)
TTS_CANDIDATES = (("faber", 8), ("faber", 16), ("faber", 24), ("faber", 32), ("faber", 40),
                  ("krylov", 10), ("krylov", 20), ("krylov", 30), ("krylov", 40),
                  ("rk4", 4), ("leapfrog", 1))


GOLDEN = os.path.join(ROOT, "tests", "golden")


def load_oracle_run(name):
    """Snapshots and parameters of a stored oracle run (tests/golden, written
    by tests/golden/make_oracle_runs.py), or None when it is not there."""
    path = os.path.join(GOLDEN, f"oracle_{name}.npz")
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        meta = json.loads(str(z["meta"]))
        snaps = [z[f"p{k}"] for k in range(1, meta["snapshots_done"] + 1)]
    return meta, snaps


def time_to_solution(w, args):
    """Largest dt per method and order whose pressure snapshots every 0.5 s
    up to the final time stay within tol (relative L2 over the physical
    domain, damping layer excluded) of the FP64 oracle's converged solution
    (Faber degree 40, dt = 1 ms, stored; checked against the oracle at
    dt = 0.5 ms); the wall time of that whole run (receiver recording
    included) is the time to solution. The library's own FP64 run of the
    reference configuration is reported beside it as a cross-check."""
    import torch
    from paper_2401_16322_amd import expwave as xw
    ref_run = load_oracle_run("layered1001_ref_faber40_dt1")
    if ref_run is None or ref_run[0]["workload"] != w.name:
        return {"skipped": "no stored oracle reference for " + w.name}
    meta, ref_np = ref_run
    if meta["snapshots_done"] * meta["snapshot_every"] < meta["T"] - 1e-9:
        return {"skipped": "stored oracle reference incomplete"}
    dev = torch.device("cuda:0")
    L = w.abc_cells
    T = w.T
    snap_every = meta["snapshot_every"]
    nsnap = int(round(T / snap_every))
    rec = w.receiver_nodes()
    src = w.source_node()
    npts = w.npts
    c2_np = w.c2()
    ref = [torch.tensor(r, dtype=torch.float64, device=dev) for r in ref_np]
    check = load_oracle_run("layered1001_ref_faber40_dt0.5")
    ref_check = None
    if check is not None and check[0]["snapshots_done"] == meta["snapshots_done"]:
        ref_check = max(float(np.linalg.norm(a - b) / np.linalg.norm(a)) for a, b in zip(ref_np, check[1]))

    def make_op(tdt, kmax):
        op = xw.Operator(w.n, w.h, torch.tensor(c2_np, dtype=tdt, device=dev),
                         abc_cells=w.abc_cells, sigma_max=w.sigma_max,
                         max_krylov_k=kmax, max_taylor_p=w.taylor_p)
        op.set_source_ricker([src], [1.0], w.f_peak, w.t_delay, w.taylor_p)
        op.set_receivers(rec)
        return op

    def interior(state):
        p = state[:npts].view(*reversed(w.n))
        sl = tuple(slice(L, n - L) for n in reversed(w.n))
        return p[sl].double()

    def run(op, tdt, method, order, dt, tol):
        """Full run; returns (max snapshot error, wall seconds)."""
        state = torch.zeros((w.ndim + 1) * npts, dtype=tdt, device=dev)
        nper = int(round(snap_every / dt))
        traces = torch.zeros(nper * max(rec.size, 1), dtype=tdt, device=dev)
        err = 0.0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(nsnap):
            t = s * snap_every
            tr = traces if rec.size else None
            if method == "faber":
                op.step_faber(state, t, dt, order, nper, traces=tr)
            elif method == "krylov":
                op.step_krylov(state, t, dt, order, nper, traces=tr)
            elif method == "rk4":
                op.step_rk4(state, t, dt, nper, traces=tr)
            else:
                op.step_leapfrog(state, t, dt, nper, traces=tr)
            # the error check is outside the method; it stops a failing run early
            torch.cuda.synchronize()
            t_pause = time.perf_counter()
            r = ref[s]
            e = (torch.linalg.vector_norm(interior(state) - r) / torch.linalg.vector_norm(r)).item()
            if not np.isfinite(e):
                e = float("inf")
            err = max(err, e)
            t0 += time.perf_counter() - t_pause
            if err > tol:
                break
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        op.sync()
        return err, wall

    # the library's FP64 run of the reference configuration, against the oracle's
    op64 = make_op(torch.float64, 0)
    try:
        gpu_ref_err, _ = run(op64, torch.float64, "faber", meta["order"], meta["dt"], float("inf"))
    finally:
        op64.close()

    kmax = max(k for m, k in TTS_CANDIDATES if m == "krylov")
    mvo_step = {"rk4": 4, "leapfrog": 1}
    out = {"workload": w.name, "tol": args.tts_tol, "T_s": T,
           "snapshots_s": [snap_every * (i + 1) for i in range(nsnap)],
           "error": "relative L2 of pressure over the physical domain, max over snapshots",
           "reference": {"source": "FP64 oracle (tests/golden/oracle_layered1001_ref_faber40_dt1.npz)",
                         "method": "faber", "order": meta["order"], "dt_ms": meta["dt"] * 1e3,
                         "vs_oracle_dt_0.5ms": ref_check,
                         "library_f64_same_config_vs_oracle": gpu_ref_err},
           "dt_ladder_ms": list(TTS_DTS_MS)}
    for dname in [d for d in args.tts_dtypes.split(",") if d]:
        tdt = {"f32": torch.float32, "f64": torch.float64}[dname]
        op = make_op(tdt, kmax)
        results = []
        try:
            for method, order in TTS_CANDIDATES:
                best, tried = None, []
                for dt_ms in TTS_DTS_MS:
                    dt = dt_ms * 1e-3
                    err, _ = run(op, tdt, method, order, dt, args.tts_tol)
                    tried.append([dt_ms, float(f"{err:.3g}") if np.isfinite(err) else None])
                    if err <= args.tts_tol:
                        walls = [run(op, tdt, method, order, dt, args.tts_tol)[1]
                                 for _ in range(args.tts_repeats)]
                        nsteps = int(round(T / dt))
                        best = {"method": method, "order": order, "dt_ms": dt_ms, "max_rel_l2": err,
                                "wall_s": float(np.median(walls)), "n_steps": nsteps,
                                "n_op": nsteps * mvo_step.get(method, order), "n_mem": nsteps}
                        break
                r = best if best else {"method": method, "order": order, "dt_ms": None}
                r["tried"] = tried  # [dt_ms, error at the first snapshot that failed, or the max]
                results.append(r)
        finally:
            op.close()
        ok = [r for r in results if r.get("dt_ms")]
        out[dname] = {"runs": results,
                      "fastest": min(ok, key=lambda r: r["wall_s"]) if ok else None}
    return out


def cpu_baseline(w, methods, mvos, dts, args, c2_np, rec):
    """The FP64 oracle on the same step, single-threaded: --cpu-steps steps,
    stopping after the first step that ends past 20 s of CPU time."""
    from threadpoolctl import threadpool_limits
    from oracle.operator import Grid
    from oracle.source import PointSources
    from oracle.steppers import Problem, step
    g = Grid(w.n, w.h, args.order, abc_cells=w.abc_cells, sigma_max=w.sigma_max)
    prob = Problem(g, c2_np, PointSources((w.source_node(),), (1.0,), w.f_peak, w.t_delay))
    ell = prob.ellipse()
    states = {m: np.zeros(g.nstate) for m in methods}
    kw = {"faber": dict(m=args.faber_m, p=w.taylor_p, ellipse=ell),
          "krylov": dict(k=args.krylov_k, p=w.taylor_p)}
    done = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for s in range(args.cpu_steps):
            for m in methods:
                states[m] = step(prob, m, states[m], s * dts[m], dts[m], **kw.get(m, {}))
                if rec.size:
                    _ = states[m][rec]
            done += 1
            if time.perf_counter() - t0 > 20.0:
                break
        el = time.perf_counter() - t0
    total = w.npts * sum(mvos[m] for m in methods) * done
    return {"value": total / el, "unit": "grid-pt matvecs/s", "cores": 1, "kind": "oracle",
            "host_cpu": host_cpu(),
            "sample": f"{done} step(s) ({'+'.join(methods)}) of {w.name} from rest, "
                      f"FP64 numpy on one thread, {el:.1f} s"}


if __name__ == "__main__":
    main()
