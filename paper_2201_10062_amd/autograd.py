"""Differentiable all-at-once heat-equation solve (torch.autograd.Function).

Forward: f_H from f and u0 (theta scheme, Sec. 1), then preconditioned MINRES on
Y T u = Y f_H for every member of the batch (one batched library call).
Backward: since T^T = Y T Y (Y T is symmetric, eqn:main_system), the adjoint
T^T lambda = dL/du is the same preconditioned MINRES with a flipped right-hand side;
then dL/df, dL/du0 (adjoint of the f_H assembly) and dL/da at the faces or nodes,
dL/da_e = -(tau/h^2) sum_k (D_e lambda_k)(D_e utilde_k).  Every step runs in the
library's HIP kernels; this module only marshals tensors.
"""
from __future__ import annotations

import numpy as np
import torch

from .smr import Batch, Plan


# Plans and batch of the latest (dim, N, n, theta, precond, batch size, device): a call with the
# same coefficient reuses them as they are; a new coefficient rebuilds the plans' tables in the
# same workspaces with the same column-tile widths (no allocation, no tile timing) and keeps the
# batch workspace, so the batched solve replays its captured iterations.
_CACHE: dict = {}


def _plans_for(dim, N, n, theta, precond, B, a_host, dev):
    key = (dim, N, n, float(theta), precond, B, str(dev))
    a_bytes = a_host.tobytes()
    ent = _CACHE.get(key)
    if ent is not None and ent["a"] == a_bytes:
        return ent["plans"], ent["batch"]
    old_plans = ent["plans"] if ent is not None else [None] * B
    plans = []
    for old in old_plans:
        ws = cols = None
        if old is not None:
            ws, cols = old.raw_workspace, (old.tile_cols or None)
            old.release()
        plans.append(Plan(dim, N, n, theta=theta, a_nodal=a_host, precond=precond, device=dev,
                          workspace=ws, tile_cols=cols))
    batch = Batch(plans, workspace=ent["batch"].raw_workspace if ent is not None else None)
    _CACHE.clear()
    _CACHE[key] = {"a": a_bytes, "plans": plans, "batch": batch}
    return plans, batch


def clear_cache():
    """Drop the cached plans (their workspaces are freed with them)."""
    _CACHE.clear()


class HeatSolve(torch.autograd.Function):
    """u = T(a)^{-1} f_H(f, u0).  f: (B, n+1, m) float64 on the GPU; a_nodal: (N+2)^dim
    nodal coefficient (float64, any device); u0: (m,) or None.  Returns u of shape (B, n, m)."""

    @staticmethod
    def forward(ctx, f, a_nodal, u0, dim, N, n, theta, rtol, maxit, precond):
        if f.dim() == 2:
            f = f.unsqueeze(0)
        B = f.shape[0]
        a_host = np.ascontiguousarray(a_nodal.detach().to("cpu", torch.float64).numpy().reshape((N + 2,) * dim))
        dev = f.device
        plans, batch = _plans_for(dim, N, n, theta, precond, B, a_host, dev)
        u0c = None if u0 is None else u0.detach().contiguous().to(dev, torch.float64)
        bs = [p.build_rhs(f[i].contiguous().reshape(-1), u0c) for i, p in enumerate(plans)]
        xs, infos = batch.solve(bs, rtol=rtol, maxit=maxit)
        u = torch.stack(xs).reshape(B, n, -1)
        ctx.plans, ctx.batch, ctx.rtol, ctx.maxit = plans, batch, rtol, maxit
        ctx.infos = infos
        ctx.has_u0 = u0 is not None
        ctx.save_for_backward(u, u0c if u0c is not None else torch.zeros(0, device=dev, dtype=torch.float64))
        ctx.a_device = a_nodal.device
        return u

    @staticmethod
    def backward(ctx, gu):
        if any(p.handle is None for p in ctx.plans):
            raise RuntimeError("the plans of this solve were rebuilt by a later forward call with another "
                               "coefficient; run backward before the next forward with a new coefficient")
        u, u0c = ctx.saved_tensors
        B = u.shape[0]
        gs = [gu[i].contiguous().reshape(-1).to(torch.float64) for i in range(B)]
        lams, ctx.adj_infos = ctx.batch.solve_adjoint(gs, rtol=ctx.rtol, maxit=ctx.maxit)
        u0p = u0c if ctx.has_u0 else None
        gf, ga, gu0 = [], None, None
        for i, p in enumerate(ctx.plans):
            gfi, gu0i = p.rhs_adjoint(lams[i], want_u0=ctx.has_u0)
            _, _, gni = p.grad_a(u[i].reshape(-1).contiguous(), lams[i], u0=u0p)
            gf.append(gfi.reshape(p.n + 1, p.m))
            ga = gni if ga is None else ga + gni
            if ctx.has_u0:
                gu0 = gu0i if gu0 is None else gu0 + gu0i
        grad_f = torch.stack(gf)
        grad_a = ga.reshape((ctx.plans[0].N + 2,) * ctx.plans[0].dim).to(ctx.a_device)
        return grad_f, grad_a, gu0, None, None, None, None, None, None, None


def heat_solve(f, a_nodal, u0=None, *, dim=2, theta=1.0, rtol=1e-8, maxit=500, precond="PH"):
    """Differentiable solve for a batch of sources f (B, n+1, m) with nodal coefficient a."""
    n = f.shape[-2] - 1
    N = a_nodal.shape[-1] - 2
    return HeatSolve.apply(f, a_nodal, u0, dim, N, n, theta, rtol, maxit, precond)
