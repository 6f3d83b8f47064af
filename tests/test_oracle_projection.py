"""Pins of the oracle's projection step, its adjoint and the multi-step gradient.

* identities the projection must satisfy whatever the solve: face divergence after correction
  equals (dt/rho) times the Poisson residual; u^{n+1} independent of dt and rho; face gradients
  annihilated; idempotence on face velocities; alpha = 0 / alpha = 1 special cases;
* the adjoint against a complex-step directional derivative (exact to rounding for this
  polynomial map) and against central finite differences.
"""
import numpy as np
import pytest

from bcm_inputs import CHANNEL_BC, uniform_mesh, uniform_random_velocity
from oracle import FVMesh, projection as P

from test_oracle_operators import _tiny_multilevel


def _setup(which):
    m = uniform_mesh((2, 2, 2), 0.5, 4, CHANNEL_BC) if which == "uniform" else _tiny_multilevel()
    fv = FVMesh(m)
    rng = np.random.default_rng(7)
    u = uniform_random_velocity(m, 8, 0.3, (1.0, 0, 0))
    alpha = rng.uniform(0, 1, m.n_cells)
    return m, fv, u, alpha


@pytest.mark.parametrize("which", ["uniform", "multilevel"])
def test_projection_identities(which):
    m, fv, u, alpha = _setup(which)
    dt, rho, U_in = 0.01, 1.3, 0.8
    r = P.project(fv, u, alpha, (0.1, 0, 0), U_in, dt, rho)
    c = dt / rho
    res = r["b"] - fv.A @ r["p"]
    # face divergence after correction == c * Poisson residual, cell by cell
    assert np.abs(fv.D @ r["U_new"] - c * res).max() <= 1e-12 * np.abs(fv.D @ r["U_star"]).max()
    # with an exact solve the faces are divergence free
    assert np.abs(fv.D @ r["U_new"]).max() <= 1e-10 * np.abs(fv.D @ r["U_star"]).max()
    # velocity independent of dt and rho; pressure scales with rho/dt
    r2 = P.project(fv, u, alpha, (0.1, 0, 0), U_in, 3 * dt, 0.5 * rho)
    assert np.abs(r2["u_new"] - r["u_new"]).max() <= 1e-12
    assert np.allclose(r2["p"] * 6.0, r["p"], rtol=1e-10, atol=1e-12 * np.abs(r["p"]).max())
    # idempotence: projecting the corrected face velocities again yields zero pressure
    p_again = fv.solve(fv.D @ r["U_new"] / c)
    assert np.abs(p_again).max() <= 1e-10 * np.abs(r["p"]).max()
    # gradient annihilation: face fields G phi are removed entirely
    phi = np.random.default_rng(1).standard_normal(m.n_cells)
    Uf = fv.G @ phi
    q = fv.solve(fv.D @ Uf / c)
    assert np.abs(Uf - c * (fv.G @ q)).max() <= 1e-10 * np.abs(Uf).max()


def test_forcing_special_cases():
    m, fv, u, _ = _setup("uniform")
    us = np.array([0.2, -0.1, 0.05])
    assert np.array_equal(P.force(u, np.zeros(m.n_cells), us), u.reshape(3, -1))
    one = np.ones(m.n_cells)
    assert np.allclose(P.force(u, one, us), np.broadcast_to(us[:, None], (3, m.n_cells)))


@pytest.mark.parametrize("which", ["uniform", "multilevel"])
def test_adjoint_matches_complex_step(which):
    m, fv, u, alpha = _setup(which)
    noise = u.copy()
    noise[0] -= 1.0
    dt, rho, U_in, K = 0.02, 1.0, 1.0, 3
    J, ga, gU = P.multistep_gradient(fv, noise, alpha, (0, 0, 0), U_in, dt, rho, K)
    rng = np.random.default_rng(11)
    for _ in range(3):
        va = rng.uniform(-1, 1, m.n_cells)
        vU = float(rng.choice([-1.0, 1.0]))
        cs = P.complex_step_derivative(fv, noise, alpha, (0, 0, 0), U_in, dt, rho, K, va, vU)
        adj = float(np.dot(ga, va) + gU * vU)
        assert abs(adj - cs) <= 1e-10 * abs(cs)


def test_adjoint_matches_central_differences():
    m, fv, u, alpha = _setup("uniform")
    noise = u.copy()
    noise[0] -= 1.0
    dt, rho, U_in, K = 0.02, 1.0, 1.0, 2
    J, ga, gU = P.multistep_gradient(fv, noise, alpha, (0, 0, 0), U_in, dt, rho, K)
    rng = np.random.default_rng(12)
    va = rng.uniform(-1, 1, m.n_cells)
    vU = 1.0
    eps = 1e-6
    Jp, _ = P.multistep_objective(fv, noise, alpha + eps * va, (0, 0, 0), U_in + eps * vU, dt,
                                  rho, K)
    Jm, _ = P.multistep_objective(fv, noise, alpha - eps * va, (0, 0, 0), U_in - eps * vU, dt,
                                  rho, K)
    fd = (Jp - Jm) / (2 * eps)
    adj = float(np.dot(ga, va) + gU * vU)
    assert abs(adj - fd) <= 1e-6 * abs(fd)
