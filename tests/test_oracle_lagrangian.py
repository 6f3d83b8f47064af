"""Pins of the Lagrangian-particle forcing oracle (oracle/lagrangian.py).

* the 3-point function: partition of unity and vanishing first moment for any shift (the
  properties it is built to satisfy), zero beyond 3/2, continuity at 1/2 and 3/2;
* interpolation of a linear velocity field is exact (uniform and three-level meshes);
* spreading conserves the total force and its first moment: sum_i V_i f_i = sum_p dV_p F_p,
  sum_i V_i x_i f_i = sum_p dV_p X_p F_p;
* spreading is the transpose of interpolation: sum_p dV_p (I u)_p . G_p = sum_i V_i u_i . (S G)_i;
* a uniform flow equal to the body velocity is left unchanged by the forcing;
* brute force: the interpolation weights equal the product of phi over all cells of a tiny mesh.
"""
import numpy as np
import pytest

from bcm_inputs import CHANNEL_BC, configs, uniform_mesh
from oracle.lagrangian import ParticleOperator, phi


def test_phi_moments_and_support():
    r = np.random.default_rng(1).uniform(-3, 3, 200)
    j = np.arange(-6, 7)
    s0 = phi(r[:, None] - j[None, :]).sum(axis=1)
    s1 = ((r[:, None] - j[None, :]) * phi(r[:, None] - j[None, :])).sum(axis=1)
    assert np.abs(s0 - 1).max() <= 1e-14 and np.abs(s1).max() <= 1e-14
    assert phi(np.array([1.5, 1.7, -2.0])).max() == 0.0
    for a in (0.5, 1.5):
        assert abs(phi(a - 1e-12) - phi(a + 1e-12)) <= 1e-11
    assert phi(0.0) == 0.75


def _particles(m, n_p, seed, box):
    rng = np.random.default_rng(seed)
    lo, hi = np.array(box[0]), np.array(box[1])
    return lo + (hi - lo) * rng.uniform(size=(n_p, 3))


MESHES = {
    "uniform": (lambda: uniform_mesh((4, 2, 2), 0.25, 8, CHANNEL_BC),
                ((0.1, 0.1, 0.1), (0.9, 0.4, 0.4))),
    "three_level": (lambda: configs.multilevel_small()["mesh"],
                    ((0.62, 0.47, 0.47), (0.78, 0.53, 0.53))),
}


@pytest.mark.parametrize("which", sorted(MESHES))
def test_linear_field_is_interpolated_exactly(which):
    make, box = MESHES[which]
    m = make()
    X = _particles(m, 60, 3, box)
    op = ParticleOperator(m, X)
    xs = m.cell_centres()
    A = np.array([[0.3, -1.2, 0.7], [2.0, 0.1, -0.4], [-0.5, 0.9, 1.1]])
    b = np.array([1.0, -2.0, 0.5])
    u = np.stack([b[d] + sum(A[d, e] * xs[e].ravel() for e in range(3)) for d in range(3)])
    U = op.interpolate(u)
    ref = b[None, :] + X @ A.T
    assert np.abs(U - ref).max() <= 1e-12


@pytest.mark.parametrize("which", sorted(MESHES))
def test_spreading_conserves_force_and_moment_and_is_the_transpose(which):
    make, box = MESHES[which]
    m = make()
    X = _particles(m, 40, 4, box)
    op = ParticleOperator(m, X)
    rng = np.random.default_rng(5)
    F = rng.standard_normal((len(X), 3))
    dV = rng.uniform(0.5, 1.5, len(X)) * op.h_cell.min() ** 3
    f = op.spread(F, dV)
    V = op.h_cell ** 3
    xs = [c.ravel() for c in m.cell_centres()]
    tot = (f * V).sum(axis=1)
    assert np.abs(tot - (F * dV[:, None]).sum(axis=0)).max() <= 1e-12 * np.abs(F).sum()
    for e in range(3):
        mom = (f * V * xs[e]).sum(axis=1)
        ref = (F * (dV * X[:, e])[:, None]).sum(axis=0)
        assert np.abs(mom - ref).max() <= 1e-12 * np.abs(F).sum()
    u = rng.standard_normal((3, m.n_cells))
    lhs = np.sum(dV[:, None] * op.interpolate(u) * F)
    rhs = np.sum(V * u * f)
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(dV[:, None] * F))


def test_body_velocity_flow_is_unchanged():
    m, box = MESHES["uniform"][0](), MESHES["uniform"][1]
    X = _particles(m, 30, 6, box)
    op = ParticleOperator(m, X)
    Us = np.array([0.4, -0.2, 0.1])
    u = np.broadcast_to(Us[:, None], (3, m.n_cells)).copy()
    u_star, U, F = op.force(u, Us, np.full(len(X), 1e-6), 0.01, 1.0)
    assert np.abs(F).max() <= 1e-10 and np.abs(u_star - u).max() <= 1e-14


def test_weights_by_brute_force():
    m = uniform_mesh((2, 2, 1), 0.5, 4, CHANNEL_BC)
    X = np.array([[0.48, 0.52, 0.23], [0.31, 0.69, 0.26]])
    op = ParticleOperator(m, X)
    xs = np.stack([c.ravel() for c in m.cell_centres()], axis=1)
    h = op.h_cell[0]
    for p in range(len(X)):
        w = np.prod(phi((xs - X[p]) / h), axis=1)
        assert np.abs(op.W[p].toarray().ravel() - w).max() <= 1e-15
        assert abs(w.sum() - 1.0) <= 1e-14
