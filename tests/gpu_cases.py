"""Shared set-up for the GPU parity tests: one seeded case built twice, once
for the oracle (numpy) and once for the HIP library (torch device memory)."""
from dataclasses import dataclass

import numpy as np

from oracle.operator import Grid
from oracle.source import PointSources
from oracle.steppers import Problem
from synthetic import layered_velocity, smooth_state

TOL = {"float64": 1e-11, "float32": 1e-5}   # relative L2 per state / snapshot


@dataclass
class Case:
    prob: Problem
    op: object
    U0: np.ndarray
    nodes: tuple
    p: int
    torch_dtype: object


def make_case(n, dtype="float64", order=4, bc="zero", abc=4, smax=300.0, src=True,
              seed=0, homogeneous=None, max_k=0, p=8, smooth=True, n_src=1, amp=1.0):
    import torch
    from paper_2401_16322_amd.expwave import Operator
    n = tuple(n)
    g = Grid(n, 10.0, order, bc=bc, abc_cells=abc if bc == "zero" else 0,
             sigma_max=smax if bc == "zero" else 0.0)
    if homogeneous is not None:
        c = np.full(g.shape, float(homogeneous))
    else:
        c = layered_velocity(n, 10.0, seed=seed + 100)
    c2 = c ** 2
    if dtype == "float32":
        # the values of the FP32 device array are the input both sides see
        c2 = c2.astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(seed)
    nodes = tuple(int(v) for v in rng.choice(g.npts, size=n_src, replace=False)) if src else ()
    amps = tuple(amp * float(a) for a in rng.uniform(0.5, 1.5, len(nodes)))
    sources = PointSources(nodes, amps, 15.0, 0.05) if src else None
    prob = Problem(g, c2, sources)
    tdt = torch.float64 if dtype == "float64" else torch.float32
    c2_dev = torch.tensor(c2, dtype=tdt, device="cuda")
    op = Operator(n, 10.0, c2_dev, order=order, bc=bc, abc_cells=g.abc_cells,
                  sigma_max=g.sigma_max, max_krylov_k=max_k, max_taylor_p=max(p, 1))
    if src:
        op.set_source_ricker(np.array(nodes), np.array(amps), 15.0, 0.05, p)
    U0 = smooth_state(n, seed=seed + 7, width_cells=max(1.0, min(n) / 8)) if smooth \
        else np.zeros(g.nstate)
    return Case(prob, op, U0, nodes, p, tdt)


def to_dev(case, U):
    import torch
    return torch.tensor(U, dtype=case.torch_dtype, device="cuda")


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a))
