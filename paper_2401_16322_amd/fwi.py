"""Receiver traces of Faber (or Krylov) steps as a differentiable function of
c^2, with checkpointing (the gradient side of the method: large steps mean
few stored wavefields, Sec. 3.3).

Forward: nsteps Faber steps of degree m (or Krylov steps of dimension m)
from U0; traces[n] is the pressure at the receivers after step n. Reverse:
with g[n] = d(loss)/d(traces[n]), lam = 0 and, for n = N-1 down to 0,
lam += g[n] at the receivers, then lam <- (step n)^T lam while the c^2
gradient of each step accumulates (expw_faber_adjoint_step: the exact
transpose of the Faber step; expw_krylov_adjoint_step: the derivatives of
the exponential with each factor in a Krylov space of dimension m). States are kept every `checkpoint_every` steps;
during the reverse sweep each segment is recomputed from its checkpoint, so
the memory is about N/K + K states instead of N. The gradient is taken at a
fixed ellipse (the ellipse of the operator, set from c^2 at creation).

Every step, recomputation and reverse term runs in the library's kernels;
this module only orders the calls.
"""
from __future__ import annotations


def _step(op, method, U, t, dt, m, traces=None):
    if method == "faber":
        op.step_faber(U, t, dt, m, 1, traces=traces)
    elif method == "krylov":
        op.step_krylov(U, t, dt, m, 1, traces=traces)
    else:
        raise ValueError(f"unknown method {method!r} (faber or krylov)")


def _forward(op, U0, t0, dt, nsteps, m, every, keep, method="faber"):
    import torch
    nrec = op._rec.numel()
    U = U0.clone()
    traces = torch.empty(max(nsteps, 1) * nrec, dtype=op.dtype, device=U0.device)
    ck = {0: U0.clone()} if keep else None
    for n in range(nsteps):
        _step(op, method, U, t0 + n * dt, dt, m, traces=traces[n * nrec:])
        if keep and (n + 1) % every == 0 and n + 1 < nsteps:
            ck[n + 1] = U.clone()
    return traces[: nsteps * nrec].view(nsteps, nrec), ck, U


def _reverse(op, ck, g, t0, dt, nsteps, m, every, method="faber"):
    """(dL/dc^2 per point, dL/dU0) for upstream trace gradients g (nsteps x n_rec)."""
    import torch
    dev = g.device
    lam = torch.zeros(op.nstate, dtype=op.dtype, device=dev)
    grad = torch.zeros(op.npts, dtype=op.dtype, device=dev)
    nscratch = (m + 1) if method == "krylov" else max(m - 1, 1)
    scratch = torch.empty(nscratch * op.nstate, dtype=op.dtype, device=dev)
    g = g.to(dtype=op.dtype).contiguous()
    for s0 in sorted(ck, reverse=True):
        s1 = min(s0 + every, nsteps)
        states = [ck[s0]]
        for n in range(s0, s1 - 1):
            u = states[-1].clone()
            _step(op, method, u, t0 + n * dt, dt, m)
            states.append(u)
        for n in range(s1 - 1, s0 - 1, -1):
            op.inject_receivers(g[n], lam)
            if method == "krylov":
                op.krylov_adjoint_step(states[n - s0], lam, t0 + n * dt, dt, m, grad, scratch)
            else:
                op.faber_adjoint_step(states[n - s0], lam, t0 + n * dt, dt, m, grad, scratch)
    return grad, lam


def misfit_gradient(op, U0, t0, dt, nsteps, m, d_obs, checkpoint_every=10, method="faber"):
    """L = 1/2 sum_n |traces[n] - d_obs[n]|^2 and (dL/dc^2, dL/dU0, traces)."""
    every = max(1, int(checkpoint_every))
    traces, ck, _ = _forward(op, U0, t0, dt, nsteps, m, every, True, method)
    resid = traces - d_obs.to(device=traces.device, dtype=traces.dtype)
    L = 0.5 * float((resid.double() ** 2).sum())
    grad, lam = _reverse(op, ck, resid, t0, dt, nsteps, m, every, method)
    return L, grad, lam, traces


def faber_traces(op, c2, U0, t0, dt, nsteps, m, checkpoint_every=10, method="faber"):
    """Receiver traces (nsteps x n_rec) as a torch autograd function of c2
    (the tensor the operator was created with) and U0."""
    import torch

    class _Traces(torch.autograd.Function):
        @staticmethod
        def forward(ctx, c2_, U0_):
            if c2_.data_ptr() != op.c2.data_ptr():
                raise ValueError("c2 must be the tensor the operator was created with")
            every = max(1, int(checkpoint_every))
            tr, ck, _ = _forward(op, U0_.detach(), t0, dt, nsteps, m, every, True, method)
            ctx.ck, ctx.every = ck, every
            return tr.clone()

        @staticmethod
        def backward(ctx, g):
            grad, lam = _reverse(op, ctx.ck, g, t0, dt, nsteps, m, ctx.every, method)
            return grad.view_as(c2), lam

    return _Traces.apply(c2, U0)
