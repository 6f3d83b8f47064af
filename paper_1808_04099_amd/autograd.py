"""Differentiable projection: torch.autograd.Function wrappers around the C ABI.

Projection           one step (u~, alpha, U_in) -> (u^{n+1}, p); backward calls the hand-written
                     adjoint kernels (transposed correction, transposed Poisson solve, transposed
                     face interpolation / divergence / forcing) through bcm_project_adjoint.
MultiStepProjection  K steps u^{k+1} = P(F(u^k)) with per-step pressure checkpoints (each
                     solve warm-started from the previous step's pressure): forward keeps u^0
                     and p^0..p^{K-1} only; backward recomputes each u^k from u^0 with
                     bcm_project_recompute (forcing + correction, no solve) and runs the
                     adjoint steps in reverse.
"""
from __future__ import annotations

import torch


def _as_field(g, like):
    if g is None:
        return torch.zeros_like(like)
    return g.to(like.dtype).contiguous()


class Projection(torch.autograd.Function):
    @staticmethod
    def forward(ctx, ux, uy, uz, alpha, U_in, plan, dt, rho):
        U = float(U_in)
        out = plan.project([ux, uy, uz], alpha, U, dt, rho)
        ctx.plan, ctx.dt, ctx.rho, ctx.U = plan, dt, rho, U
        ctx.report = out["report"]
        ctx.save_for_backward(ux, uy, uz, alpha)
        u = out["u_new"]
        return u[0], u[1], u[2], out["p"]

    @staticmethod
    def backward(ctx, gx, gy, gz, gp):
        ux, uy, uz, alpha = ctx.saved_tensors
        plan = ctx.plan
        g = [_as_field(x, ux) for x in (gx, gy, gz)]
        g_p = None if gp is None else gp.to(torch.float64).contiguous()
        g_u, g_alpha, gU, _, _ = plan.project_adjoint([ux, uy, uz], alpha, g, ctx.U, ctx.dt,
                                                      ctx.rho, g_p=g_p)
        return (g_u[0], g_u[1], g_u[2], g_alpha,
                torch.tensor(gU, dtype=torch.float64), None, None, None)


class MultiStepProjection(torch.autograd.Function):
    @staticmethod
    def forward(ctx, ux, uy, uz, alpha, U_in, plan, dt, rho, steps):
        U = float(U_in)
        u = [ux, uy, uz]
        ps, reports = [], []
        for _ in range(int(steps)):
            out = plan.project(u, alpha, U, dt, rho, p0=ps[-1] if ps else None)
            ps.append(out["p"])
            reports.append(out["report"])
            u = out["u_new"]
        ctx.plan, ctx.dt, ctx.rho, ctx.U, ctx.steps = plan, dt, rho, U, int(steps)
        ctx.reports = reports
        ctx.save_for_backward(ux, uy, uz, alpha, *ps)
        return u[0], u[1], u[2]

    @staticmethod
    def backward(ctx, gx, gy, gz):
        saved = ctx.saved_tensors
        u0, alpha, ps = list(saved[:3]), saved[3], saved[4:]
        plan = ctx.plan
        g = [_as_field(x, u0[0]) for x in (gx, gy, gz)]
        g_alpha = torch.zeros_like(u0[0]) if alpha is not None else None
        gU = 0.0
        for k in reversed(range(ctx.steps)):
            u = u0
            for j in range(k):      # recompute u^k from the checkpointed pressures
                u = plan.project_recompute(u, alpha, ps[j], ctx.U, ctx.dt, ctx.rho)
            g, ga, gu_in, _, _ = plan.project_adjoint(u, alpha, g, ctx.U, ctx.dt, ctx.rho)
            if g_alpha is not None:
                g_alpha += ga
            gU += gu_in
        return (g[0], g[1], g[2], g_alpha, torch.tensor(gU, dtype=torch.float64),
                None, None, None, None)


def kinetic_energy(u, cell_volume, rho=1.0):
    """J = (rho/2) sum_i V_i |u_i|^2 (torch ops; the objective is user code, not the path)."""
    return 0.5 * rho * sum((cell_volume * (x.to(torch.float64) ** 2)).sum() for x in u)
