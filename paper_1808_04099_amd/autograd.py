"""Differentiable projection: torch.autograd.Function wrappers around the C ABI.

Projection           one step (u~, alpha, U_in) -> (u^{n+1}, p); backward calls the hand-written
                     adjoint kernels (transposed correction, transposed Poisson solve, transposed
                     face interpolation / divergence / forcing) through bcm_project_adjoint.
MultiStepProjection  K steps u^{k+1} = P(F(u^k)) with per-step pressure checkpoints (each
                     solve warm-started from the previous step's pressure): forward keeps u^0
                     and p^0..p^{K-1} only; backward recomputes u^1..u^{K-1} once each with
                     bcm_project_recompute (forcing + correction, no solve) and runs the
                     adjoint steps in reverse, the library summing the cotangents of alpha
                     and U_in over the steps.
KineticEnergy        the objective J = (rho/2) sum V |u|^2 and its seed, by bcm_kinetic_energy.
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
        plan, K = ctx.plan, ctx.steps
        g = [_as_field(x, u0[0]) for x in (gx, gy, gz)]
        # u^1 .. u^{K-1} recomputed once each from the checkpointed pressures (K - 1 calls of
        # forcing + correction, no solve); they are held until the reverse sweep releases them
        hist = [u0]
        for j in range(K - 1):
            hist.append(plan.project_recompute(hist[-1], alpha, ps[j], ctx.U, ctx.dt, ctx.rho))
        g_alpha, gU = None, 0.0
        for k in reversed(range(K)):
            g, g_alpha, gU, _, _ = plan.project_adjoint(
                hist[k], alpha, g, ctx.U, ctx.dt, ctx.rho, g_alpha=g_alpha, g_U_in=gU,
                accumulate=k < K - 1)
            hist[k] = None
        return (g[0], g[1], g[2], g_alpha, torch.tensor(gU, dtype=torch.float64),
                None, None, None, None)


class KineticEnergy(torch.autograd.Function):
    """J = (rho/2) sum_i V_i |u_i|^2 through bcm_kinetic_energy; the backward asks the library
    for the seed cotangent grad_J * rho * V * u."""

    @staticmethod
    def forward(ctx, ux, uy, uz, plan, rho):
        J, _ = plan.kinetic_energy([ux, uy, uz], rho)
        ctx.plan, ctx.rho = plan, rho
        ctx.save_for_backward(ux, uy, uz)
        return torch.tensor(J, dtype=torch.float64, device=ux.device)

    @staticmethod
    def backward(ctx, gJ):
        ux, uy, uz = ctx.saved_tensors
        _, seed = ctx.plan.kinetic_energy([ux, uy, uz], ctx.rho, g_scale=float(gJ),
                                          want_J=False)
        return seed[0], seed[1], seed[2], None, None


def kinetic_energy(u, plan, rho=1.0):
    """Kinetic-energy objective of the velocity fields u [3] on the plan's mesh (differentiable)."""
    return KineticEnergy.apply(u[0], u[1], u[2], plan, rho)
