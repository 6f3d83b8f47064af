"""The five synthetic workloads, as concrete seeded inputs.

Each preset returns a dict with the mesh, the velocity to project (u_tilde, [3][c][k][j][i]),
the solid volume fraction alpha ([c][k][j][i]), the body velocity u_s (a constant, zero: the
bodies are stationary), the inflow speed U_in, dt, rho and the solve tolerance.  Only the mesh
shapes, value distributions and seeds are decided here; no projection arithmetic happens.

  small_box     4x4x4 cubes of 16^3 on [0,1]^3, every side open (p = 0); manufactured Poisson
                RHS b = -14 pi^2 sin(pi x) sin(2 pi y) sin(3 pi z) and a U[-1,1] velocity (seed 0)
  sphere_channel  16x8x8 cubes of 16^3 on [0,2]x[0,1]^2, inflow -x (U_in = 1), outflow +x, slip
                y/z sides; sphere r = 0.15 at (0.5,0.5,0.5); u = (1,0,0) + 0.05 U[-1,1] (seed 1)
  mixed_channel 32x16x16 cubes of 16^3, same domain/BCs/sphere; each component a 32-mode smooth
                random field (seeds 2,3,4) plus U_in = 1 along x
  adjoint_channel 32x8x8 cubes of 16^3 on [0,4]x[0,1]^2 (2048 cubes), u0 = U_in e_x +
                0.05 U[-1,1] (seed 5), sphere; 4 steps.  Sub-case: 4x4x4 cubes on [0,1]^3.
  multilevel    3 levels of 16^3 cubes over [0,2]x[0,1]^2 (level-0 edge 1/12), refined near a
                bluff body = box [0.5,0.9]x[0.425,0.575]^2 U ellipsoid centred (0.5,0.5,0.5) with
                semi-axes (0.2,0.08,0.08); u = (1,0,0) + 0.05 U[-1,1] (seed 6); 10 steps.
"""
from __future__ import annotations

import numpy as np

from .fields import Box, Ellipsoid, Sphere, Union, fourier_field, uniform_random_velocity, \
    volume_fraction
from .mesh import CHANNEL_BC, OPEN_BC, build_mesh, uniform_mesh

RHO = 1.0


def _problem(mesh, u, alpha, U_in, tol, **extra):
    h_min = float(mesh.h().min())
    u_ref = U_in if U_in > 0 else 1.0
    d = dict(mesh=mesh, u=u, alpha=alpha, us=(0.0, 0.0, 0.0), U_in=float(U_in),
             dt=0.5 * h_min / u_ref, rho=RHO, tol=tol)
    d.update(extra)
    return d


def manufactured_rhs(mesh):
    """b = -14 pi^2 sin(pi x) sin(2 pi y) sin(3 pi z) at cell centres; p = sin sin sin solves
    the continuous problem with p = 0 on the boundary of [0,1]^3."""
    X, Y, Z = mesh.cell_centres()
    return -14.0 * np.pi ** 2 * np.sin(np.pi * X) * np.sin(2 * np.pi * Y) * np.sin(3 * np.pi * Z)


def small_box(n=16, cubes=4):
    mesh = uniform_mesh((cubes,) * 3, 1.0 / cubes, n, OPEN_BC)
    u = uniform_random_velocity(mesh, seed=0, amp=1.0)
    alpha = np.zeros((mesh.n_cubes, n, n, n))
    return _problem(mesh, u, alpha, 0.0, 1e-10, b=manufactured_rhs(mesh))


def sphere_body():
    return Sphere((0.5, 0.5, 0.5), 0.15)


def sphere_channel(n=16, dims=(16, 8, 8), edge=1.0 / 8, seed=1, quad=32):
    mesh = uniform_mesh(dims, edge, n, CHANNEL_BC)
    u = uniform_random_velocity(mesh, seed=seed, amp=0.05, base=(1.0, 0.0, 0.0))
    alpha = volume_fraction(mesh, sphere_body(), quad=quad)
    return _problem(mesh, u, alpha, 1.0, 1e-10)


def mixed_channel(n=16, dims=(32, 16, 16), edge=1.0 / 16, seeds=(2, 3, 4), quad=32):
    mesh = uniform_mesh(dims, edge, n, CHANNEL_BC)
    u = np.stack([fourier_field(mesh, s) for s in seeds])
    u[0] += 1.0
    alpha = volume_fraction(mesh, sphere_body(), quad=quad)
    return _problem(mesh, u, alpha, 1.0, 1e-10)


def adjoint_channel(n=16, dims=(32, 8, 8), edge=1.0 / 8, seed=5, steps=4, quad=32):
    mesh = uniform_mesh(dims, edge, n, CHANNEL_BC)
    noise = uniform_random_velocity(mesh, seed=seed, amp=0.05)
    alpha = volume_fraction(mesh, sphere_body(), quad=quad)
    return _problem(mesh, noise + np.array([1.0, 0, 0])[:, None, None, None, None], alpha, 1.0,
                    1e-13, noise=noise, steps=steps)


def adjoint_subcase(n=16, seed=5, steps=4, quad=32):
    """The 64-cube sub-case on [0,1]^3 with the channel's boundary kinds."""
    return adjoint_channel(n=n, dims=(4, 4, 4), edge=0.25, seed=seed, steps=steps, quad=quad)


def fd_directions(n_cells, seeds=range(10, 18)):
    """Seeded directions for directional-derivative checks: (v_alpha [n_cells], v_U_in)."""
    out = []
    for s in seeds:
        rng = np.random.default_rng(s)
        out.append((rng.uniform(-1.0, 1.0, size=n_cells), float(rng.choice([-1.0, 1.0]))))
    return out


def bluff_body():
    return Union(Box((0.5, 0.425, 0.425), (0.9, 0.575, 0.575)),
                 Ellipsoid((0.5, 0.5, 0.5), (0.2, 0.08, 0.08)))


def _box_distance(lo, hi, blo, bhi):
    d = np.maximum(0.0, np.maximum(blo - hi, lo - bhi))
    return float(np.sqrt(np.sum(d * d)))


def multilevel(n=16, base=(24, 12, 12), root_edge=1.0 / 12, d1=0.45, d2=0.12, seed=6,
               quad=16):
    """Three-level mesh refined by distance to the body's bounding boxes: level-1 cubes within d1,
    level-2 cubes within d2 (then 2:1 face balance)."""
    bb = [((0.5, 0.425, 0.425), (0.9, 0.575, 0.575)), ((0.3, 0.42, 0.42), (0.7, 0.58, 0.58))]
    bb = [(np.array(a), np.array(b)) for a, b in bb]

    def refine(level, lo, hi):
        dist = min(_box_distance(lo, hi, a, b) for a, b in bb)
        return dist <= (d1 if level == 0 else d2)

    mesh = build_mesh(base, root_edge, n, CHANNEL_BC, refine=refine, max_level=2)
    u = uniform_random_velocity(mesh, seed=seed, amp=0.05, base=(1.0, 0.0, 0.0))
    alpha = volume_fraction(mesh, bluff_body(), quad=quad)
    return _problem(mesh, u, alpha, 1.0, 1e-10, steps=10)


def multilevel_small(n=4, seed=6, quad=8):
    """A scaled-down three-level mesh (same domain and body) that the oracle solves directly."""
    return multilevel(n=n, base=(6, 3, 3), root_edge=1.0 / 3, d1=0.1, d2=0.01, seed=seed,
                      quad=quad)
