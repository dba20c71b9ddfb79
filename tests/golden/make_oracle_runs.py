"""Writes the stored oracle runs under tests/golden/ (FP64, the oracle only).

Each run advances a workload from rest with its Ricker source and stores the
pressure over the physical domain (the damping layer excluded) at fixed
snapshot times, as float64, together with the run's parameters. Nothing here
calls the HIP library: the inputs come from `synthetic`, every value from
`oracle`.

    python tests/golden/make_oracle_runs.py <run>

Runs (see RUNS and PML_RUNS): whole runs for the long-run parity tests, the
converged reference of the time-to-solution measurement and its dt/2 check,
the central planes of the 256^3 workload, and a whole run of the paper's PML
operator.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.operator import Grid  # noqa: E402
from oracle.source import PointSources  # noqa: E402
from oracle.steppers import Problem, step  # noqa: E402
from synthetic import get_workload  # noqa: E402

# name: (workload, method, order (m or k), dt (s), T (s), snapshot spacing (s), what is stored)
RUNS = {
    # long runs on the small box (no layer): 2000, 1000 and 500 steps
    "box241_faber16_dt1": ("layered2d_241x161", "faber", 16, 1e-3, 2.0, 0.25, "interior"),
    "box241_faber16_dt2": ("layered2d_241x161", "faber", 16, 2e-3, 2.0, 0.25, "interior"),
    "box241_faber24_dt4": ("layered2d_241x161", "faber", 24, 4e-3, 2.0, 0.2, "interior"),
    "box241_krylov10_dt2.5": ("layered2d_241x161", "krylov", 10, 2.5e-3, 2.0, 0.25, "interior"),
    # the 1001 x 501 workload: the bench's Faber configuration over T = 2 s
    "layered1001_faber16_dt2": ("layered2d_1001x501", "faber", 16, 2e-3, 2.0, 0.5, "interior"),
    # converged reference of the time-to-solution measurement and its check at dt / 2
    "layered1001_ref_faber40_dt1": ("layered2d_1001x501", "faber", 40, 1e-3, 2.0, 0.5, "interior"),
    "layered1001_ref_faber40_dt0.5": ("layered2d_1001x501", "faber", 40, 5e-4, 2.0, 0.5, "interior"),
    # the 256^3 workload over T = 1 s: central planes every 0.25 s
    "layered3d256_faber24_dt2.5": ("layered3d_256", "faber", 24, 2.5e-3, 1.0, 0.25, "planes"),
}

# the paper's operator (the PML system with a free surface, Sec. 2) on the
# small box: name: (workload, PML cells, beta0, method, order, dt, T, snapshot
# spacing); stores the first field over the whole grid
PML_RUNS = {
    "pml241_faber16_dt2": ("layered2d_241x161", 20, 200.0, "faber", 16, 2e-3, 1.0, 0.25),
}


def interior(w, p):
    """Pressure over the physical domain (layer of abc_cells cells excluded)."""
    L = w.abc_cells
    sl = tuple(slice(L, n - L) for n in reversed(w.n))
    return np.ascontiguousarray(p.reshape(tuple(reversed(w.n)))[sl])


def planes(w, p):
    """The three central planes of a 3D pressure field: (xy at z = nz/2,
    xz at y = ny/2, yz at x = nx/2), numpy order."""
    f = p.reshape(tuple(reversed(w.n)))          # (nz, ny, nx)
    nz, ny, nx = f.shape
    return [np.ascontiguousarray(f[nz // 2]), np.ascontiguousarray(f[:, ny // 2, :]),
            np.ascontiguousarray(f[:, :, nx // 2])]


def main_pml(name):
    from oracle import pml
    wname, cells, beta0, method, order, dt, T, every = PML_RUNS[name]
    w = get_workload(wname)
    nx, ny = w.n
    g = pml.PMLGrid(nx, ny, w.h, abc_cells=cells, beta0=beta0)
    src = pml.PMLSources((w.source_node(),), (1.0,), w.f_peak, w.t_delay)
    prob = pml.PMLProblem(g, w.c2(), src)
    nsteps = int(round(T / dt))
    per = int(round(every / dt))
    assert abs(per * dt - every) < 1e-12 and per * (nsteps // per) == nsteps
    ell = prob.ellipse()
    U = np.zeros(g.nstate)
    out = {}
    t0 = time.time()
    for n in range(nsteps):
        U = step(prob, method, U, n * dt, dt, m=order, p=w.taylor_p, ellipse=ell)
        if (n + 1) % per == 0:
            k = (n + 1) // per
            out[f"p{k}"] = np.ascontiguousarray(U[: g.npts].reshape(ny, nx))
            print(f"{name}: t = {(n + 1) * dt:.3f} s after {time.time() - t0:.0f} s", flush=True)
            meta = {"workload": wname, "operator": "pml", "pml_cells": cells, "beta0": beta0,
                    "method": method, "order": order, "dt": dt, "T": T, "snapshot_every": every,
                    "stored": "pml_first_field", "snapshots_done": k, "taylor_p": w.taylor_p,
                    "c2": "float32-representable (Workload.c2)", "ellipse": list(ell),
                    "seconds": time.time() - t0}
            tmp = os.path.join(HERE, f"oracle_{name}.tmp.npz")
            np.savez_compressed(tmp, meta=np.array(json.dumps(meta)), **out)
            os.replace(tmp, os.path.join(HERE, f"oracle_{name}.npz"))


def main(name):
    if name in PML_RUNS:
        return main_pml(name)
    wname, method, order, dt, T, every, what = RUNS[name]
    w = get_workload(wname)
    g = Grid(w.n, w.h, 4, abc_cells=w.abc_cells, sigma_max=w.sigma_max)
    prob = Problem(g, w.c2(), PointSources((w.source_node(),), (1.0,), w.f_peak, w.t_delay))
    nsteps = int(round(T / dt))
    per = int(round(every / dt))
    assert abs(per * dt - every) < 1e-12 and per * (nsteps // per) == nsteps
    kw = {"faber": dict(m=order, p=w.taylor_p, ellipse=prob.ellipse()),
          "krylov": dict(k=order, p=w.taylor_p)}[method]
    U = np.zeros(g.nstate)
    out = {}
    t0 = time.time()
    for n in range(nsteps):
        U = step(prob, method, U, n * dt, dt, **kw)
        if (n + 1) % per == 0:
            k = (n + 1) // per
            p = U[: g.npts]
            if what == "interior":
                out[f"p{k}"] = interior(w, p)
            else:
                for i, pl in enumerate(planes(w, p)):
                    out[f"p{k}_plane{i}"] = pl
            print(f"{name}: t = {(n + 1) * dt:.3f} s after {time.time() - t0:.0f} s", flush=True)
            meta = {"workload": wname, "method": method, "order": order, "dt": dt, "T": T,
                    "snapshot_every": every, "stored": what, "snapshots_done": k,
                    "taylor_p": w.taylor_p, "c2": "float32-representable (Workload.c2)",
                    "ellipse": list(prob.ellipse()), "seconds": time.time() - t0}
            # written after every snapshot, so a long run leaves usable partial files
            tmp = os.path.join(HERE, f"oracle_{name}.tmp.npz")
            np.savez_compressed(tmp, meta=np.array(json.dumps(meta)), **out)
            os.replace(tmp, os.path.join(HERE, f"oracle_{name}.npz"))


if __name__ == "__main__":
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        main(sys.argv[1])
