"""Projection step, its exact adjoint and the multi-step kinetic-energy objective (FP64).

TEST INFRASTRUCTURE ONLY: the product path never imports this package.

One step of the paper's fractional-step method after the momentum sub-step (Sec. 3):
  1. immersed-body forcing  rho (u* - u~)/dt = f,  with the constraint force written per cell as
     f = (rho/dt) alpha (u_s - u~), alpha = solid volume fraction, so u* = (1-alpha) u~ + alpha u_s
     (the Eulerian form of the constraint force; the paper's simplified constraint u = u_s in the
     body, Sec. 2);
  2. Poisson equation  D G p = (rho/dt) D U*   (U* = face velocity of u*);
  3. velocity correction  u^{n+1} = u* - (dt/rho) G_c p  and  U^{n+1} = U* - (dt/rho) G p.
     (The printed correction coefficient is rho/dt; only dt/rho is consistent with the Poisson
     right-hand side, which is the reading used everywhere here.)
The adjoint is the exact transpose of this discrete map with the solve taken as exact.
"""
from __future__ import annotations

import numpy as np


def _us_field(us, C, dtype=np.float64):
    us = np.asarray(us)
    if us.ndim == 1 and us.size == 3:
        return np.broadcast_to(us.astype(dtype)[:, None], (3, C))
    return us.reshape(3, C)


def force(u_tilde, alpha, us):
    """u* = (1 - alpha) u~ + alpha u_s, per cell and component."""
    C = alpha.size
    ut = u_tilde.reshape(3, C)
    a = alpha.reshape(C)
    return (1.0 - a) * ut + a * _us_field(us, C)


def project(ops, u_tilde, alpha, us, U_in, dt, rho, p=None):
    """One projection on an FVMesh; returns every intermediate (flat cube-major arrays)."""
    C = ops.n_cells
    c = dt / rho
    ustar = force(u_tilde, alpha, us)
    Uf = ops.face_velocity(ustar, U_in)
    b = (ops.D @ Uf) / c
    if p is None:
        p = ops.solve(b)
    gp = ops.G @ p
    Uf_new = Uf - c * gp
    u_new = ustar - c * (ops.Gc @ gp).reshape(3, C)
    return dict(u_star=ustar, U_star=Uf, b=b, p=p, U_new=Uf_new, u_new=u_new)


def project_adjoint(ops, u_tilde, alpha, us, U_in, dt, rho, gu_new, gU_new=None, gp=None):
    """Transpose of `project` applied to the output cotangents.

    gu_new: d(obj)/d(u^{n+1}) [3, C]; gU_new: d(obj)/d(U^{n+1}) [faces] or None;
    gp: d(obj)/dp [C] or None.  Returns (g_u_tilde [3, C], g_u_star [3, C], g_U_in, lam) where
    lam = A^{-T}(...) is the adjoint pressure; alpha_gradient(g_u_star, ...) gives
    d(obj)/d(alpha).
    """
    C = ops.n_cells
    c = dt / rho
    a = alpha.reshape(C)
    gu_new = np.asarray(gu_new).reshape(3, C)
    g_face_grad = -c * (ops.Gc.T @ gu_new.reshape(-1))
    if gU_new is not None:
        g_face_grad = g_face_grad - c * gU_new
    g_p = ops.G.T @ g_face_grad
    if gp is not None:
        g_p = g_p + gp
    lam = ops.solve_T(g_p)
    gUf = (ops.D.T @ lam) / c
    if gU_new is not None:
        gUf = gUf + gU_new
    g_ustar = gu_new + (ops.W.T @ gUf).reshape(3, C)
    g_U_in = np.dot(ops.w0, gUf)
    g_ut = (1.0 - a) * g_ustar
    return g_ut, g_ustar, g_U_in, lam


def alpha_gradient(g_ustar, u_tilde, us):
    """d(obj)/d(alpha) = sum over components of g_u* (u_s - u~)."""
    C = g_ustar.shape[1]
    return np.sum(g_ustar * (_us_field(us, C) - u_tilde.reshape(3, C)), axis=0)


def kinetic_energy(ops, u, rho):
    """J = (rho/2) sum_i V_i (u_i . u_i), without complex conjugation (complex-step safe)."""
    u = u.reshape(3, -1)
    return 0.5 * rho * np.sum(ops.V * np.sum(u * u, axis=0))


def initial_velocity(noise, U_in):
    """u^0 = U_in e_x + noise."""
    u0 = np.array(noise, dtype=np.result_type(noise, U_in), copy=True).reshape(3, -1)
    u0[0] = u0[0] + U_in
    return u0


def multistep_objective(ops, noise, alpha, us, U_in, dt, rho, steps):
    """J(alpha, U_in) after `steps` projections u^{k+1} = P(F(u^k)) from u^0 = U_in e_x + noise."""
    u = initial_velocity(noise, U_in)
    for _ in range(steps):
        u = project(ops, u, alpha, us, U_in, dt, rho)["u_new"]
    return kinetic_energy(ops, u, rho), u


def multistep_gradient(ops, noise, alpha, us, U_in, dt, rho, steps):
    """(J, dJ/dalpha [C], dJ/dU_in) by reverse sweeps over the stored velocities."""
    C = ops.n_cells
    u = initial_velocity(noise, U_in)
    hist = []
    for _ in range(steps):
        hist.append(u)
        u = project(ops, u, alpha, us, U_in, dt, rho)["u_new"]
    J = kinetic_energy(ops, u, rho)
    g = rho * ops.V * u.reshape(3, C)
    g_alpha = np.zeros(C)
    g_U = 0.0
    for k in reversed(range(steps)):
        g_ut, g_ustar, gU, _ = project_adjoint(ops, hist[k], alpha, us, U_in, dt, rho, g)
        g_alpha += alpha_gradient(g_ustar, hist[k], us)
        g_U += gU
        g = g_ut
    g_U += float(np.sum(g[0]))      # u^0 = U_in e_x + noise
    return J, g_alpha, g_U


def complex_step_derivative(ops, noise, alpha, us, U_in, dt, rho, steps, v_alpha, v_U,
                            eps=1e-30):
    """Directional derivative of J along (v_alpha, v_U) by the complex step Im J(x + i eps v)/eps.

    Exact to rounding here: the map is polynomial in alpha and affine in U_in, with no
    conjugation anywhere."""
    a = alpha.reshape(-1) + 1j * eps * v_alpha.reshape(-1)
    U = U_in + 1j * eps * v_U
    J, _ = multistep_objective(ops, noise.astype(np.complex128), a, us, U, dt, rho, steps)
    return float(J.imag / eps)
