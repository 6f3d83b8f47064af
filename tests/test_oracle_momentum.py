"""Pins of the momentum sub-step oracle (oracle/momentum.py): closed forms and brute force.

* QUICK: the face value is exact for quadratics, so with a uniform advecting velocity the
  convective term of a quadratic field is U v'(x) exactly, for either flow direction, in cells
  whose stencil stays inside the domain;
* diffusion: exact second derivative of a quadratic; separable sine (Dirichlet walls) and
  cosine (zero-gradient walls) modes are eigenfunctions of the operator with the two-layer
  mirror ghosts, so one Euler step multiplies them by 1 + nu dt lambda and one Crank-Nicolson
  step by (1 + nu dt lambda/2) / (1 - nu dt lambda/2), lambda = sum_d (2 cos(w_d h) - 2)/h^2;
* free stream: u = (U_in, 0, 0) in the inflow/slip/outflow channel is steady under every scheme;
* brute force: H written cell by cell from the ghost and upwind rules on a tiny mesh with every
  boundary kind, and the Crank-Nicolson system solved densely, agree with the array form and
  the BiCGSTAB solve;
* AB2 with H(u^{n-1}) = H(u^n) reduces to the Euler step.
"""
import numpy as np
import pytest

from bcm_inputs import CHANNEL_BC, OPEN_BC, uniform_mesh, uniform_random_velocity
from oracle.momentum import MomentumGrid, step

INFLOW_BOX = ("inflow",) * 6


def _coords(mg):
    Nz, Ny, Nx = mg.shape
    h = mg.h
    z, y, x = np.meshgrid((np.arange(Nz) + 0.5) * h, (np.arange(Ny) + 0.5) * h,
                          (np.arange(Nx) + 0.5) * h, indexing="ij")
    return x, y, z


@pytest.mark.parametrize("U", [0.7, -0.45])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_quick_convection_exact_for_quadratics(U, axis):
    m = uniform_mesh((2, 2, 2), 0.5, 8, CHANNEL_BC)
    mg = MomentumGrid(m)
    X = _coords(mg)
    s = X[axis]
    a = [np.zeros(mg.shape) for _ in range(3)]
    a[axis][:] = U
    v = [1.0 + 2.0 * s - 3.0 * s * s, 0.5 * s * s, -s]
    H = mg.H(v, a, 0.0, 0.0)
    dv = [2.0 - 6.0 * s, s, -np.ones_like(s)]
    ax = 2 - axis
    N = mg.shape[ax]
    inner = [slice(None)] * 3
    inner[ax] = slice(2, N - 2)
    for c in range(3):
        assert np.abs(H[c][tuple(inner)] + U * dv[c][tuple(inner)]).max() <= 1e-12


def test_diffusion_exact_for_quadratics():
    m = uniform_mesh((2, 2, 2), 0.5, 8, OPEN_BC)
    mg = MomentumGrid(m)
    x, y, z = _coords(mg)
    v = [x * x + 2 * y * y - z * z, x * y, 3 * z * z]
    zero = [np.zeros(mg.shape) for _ in range(3)]
    H = mg.H(v, zero, 1.3, 0.0)
    lap = [1.3 * 2 * (1 + 2 - 1) * np.ones_like(x), np.zeros_like(x), 1.3 * 6 * np.ones_like(x)]
    inner = (slice(1, -1),) * 3
    for c in range(3):
        assert np.abs(H[c][inner] - lap[c][inner]).max() <= 1e-9


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
def test_diffusion_eigenmode_amplification(bc):
    sides = INFLOW_BOX if bc == "dirichlet" else OPEN_BC
    m = uniform_mesh((2, 2, 2), 0.5, 8, sides)
    mg = MomentumGrid(m)
    X = _coords(mg)
    L = 1.0
    h = mg.h
    k = (1, 2, 3)
    nu, dt = 0.02, 0.01
    w = [np.pi * (k[d] + (0 if bc == "dirichlet" else 0)) / L for d in range(3)]
    f = np.sin if bc == "dirichlet" else np.cos
    mode = f(w[0] * X[0]) * f(w[1] * X[1]) * f(w[2] * X[2])
    lam = sum((2 * np.cos(wd * h) - 2) / h ** 2 for wd in w)
    u = [mode, 0.5 * mode, -mode]
    zero = [np.zeros(mg.shape) for _ in range(3)]
    ue, _ = mg.euler(u, nu, 0.0, dt, a=zero)
    ucn, _ = mg.cn(u, nu, 0.0, dt, a=zero)
    ge = 1 + nu * dt * lam
    gcn = (1 + 0.5 * nu * dt * lam) / (1 - 0.5 * nu * dt * lam)
    for c in range(3):
        assert np.abs(ue[c] - ge * u[c]).max() <= 1e-13
        assert np.abs(ucn[c] - gcn * u[c]).max() <= 1e-12


@pytest.mark.parametrize("scheme", ["euler", "ab2", "cn"])
def test_free_stream_is_steady(scheme):
    m = uniform_mesh((3, 2, 2), 0.25, 4, CHANNEL_BC)
    U_in = 1.3
    u = np.zeros((3, m.n_cells))
    u[0] = U_in
    hp = np.zeros((3, m.n_cells))
    ut, Hn = step(m, u, 0.01, U_in, 0.05, scheme, h_prev=hp)
    assert np.abs(Hn).max() <= 1e-12
    assert np.abs(ut - u).max() <= 1e-12


def _brute_H(m, v, a, nu, U_in):
    """H cell by cell: ghost values by mirroring about the boundary face per axis (Dirichlet
    2 g - v, Neumann v), QUICK upwinded on the face velocity, 7-point diffusion."""
    mg = MomentumGrid(m)
    Nz, Ny, Nx = mg.shape
    N = (Nx, Ny, Nz)
    h = mg.h
    side_bc = mg.side_bc

    def val(F, comp, idx):
        idx = list(idx)
        for d in range(3):
            if idx[d] < 0 or idx[d] >= N[d]:
                side = 0 if idx[d] < 0 else 1
                layer = -idx[d] - 1 if side == 0 else idx[d] - N[d]
                mirror = layer if side == 0 else N[d] - 1 - layer
                idx[d] = mirror
                inner = F[comp][idx[2], idx[1], idx[0]]
                kind = side_bc[2 * d + side]
                if kind == 1 or (kind == 3 and comp != d):
                    return inner
                g = 0.0
                if kind == 2 and comp == d:
                    g = -U_in if side else U_in
                return 2 * g - inner
        return F[comp][idx[2], idx[1], idx[0]]

    out = [np.zeros(mg.shape) for _ in range(3)]
    for k in range(Nz):
        for j in range(Ny):
            for i in range(Nx):
                for c in range(3):
                    acc = 0.0
                    for d in range(3):
                        e = [0, 0, 0]
                        e[d] = 1
                        at = lambda o: (i + o * e[0], j + o * e[1], k + o * e[2])
                        fl = []
                        for lo in (-1, 0):          # faces i-1/2 (lo=-1) and i+1/2 (lo=0)
                            U = 0.5 * (val(a, d, at(lo)) + val(a, d, at(lo + 1)))
                            if U >= 0:
                                q = (0.75 * val(v, c, at(lo)) + 0.375 * val(v, c, at(lo + 1))
                                     - 0.125 * val(v, c, at(lo - 1)))
                            else:
                                q = (0.75 * val(v, c, at(lo + 1)) + 0.375 * val(v, c, at(lo))
                                     - 0.125 * val(v, c, at(lo + 2)))
                            fl.append(U * q)
                        acc -= (fl[1] - fl[0]) / h
                        acc += nu * (val(v, c, at(1)) - 2 * val(v, c, at(0))
                                     + val(v, c, at(-1))) / h ** 2
                    out[c][k, j, i] = acc
    return out


@pytest.mark.parametrize("sides", [CHANNEL_BC, OPEN_BC, ("outflow", "inflow", "slip",
                                                         "outflow", "inflow", "slip")])
def test_operator_matches_cell_by_cell_and_dense_cn(sides):
    m = uniform_mesh((2, 1, 1), 0.5, 4, sides)
    mg = MomentumGrid(m)
    rng = np.random.default_rng(71)
    v = [rng.standard_normal(mg.shape) for _ in range(3)]
    a = [rng.uniform(-1, 1, mg.shape) for _ in range(3)]
    nu, U_in = 0.05, 0.8
    H = mg.H(v, a, nu, U_in)
    Hb = _brute_H(m, v, a, nu, U_in)
    for c in range(3):
        assert np.abs(H[c] - Hb[c]).max() <= 1e-12 * np.abs(Hb[c]).max()
    it, _ = mg.cn(v, nu, U_in, 0.03, a=a)
    de, _ = mg.cn(v, nu, U_in, 0.03, a=a, dense=True)
    for c in range(3):
        assert np.abs(it[c] - de[c]).max() <= 1e-12 * np.abs(de[c]).max()


def test_ab2_with_equal_histories_is_euler():
    m = uniform_mesh((2, 2, 1), 0.5, 4, CHANNEL_BC)
    u = uniform_random_velocity(m, 72, 0.3, (1.0, 0, 0)).reshape(3, -1)
    ue, Hn = step(m, u, 0.01, 1.0, 0.02, "euler")
    ua, Ha = step(m, u, 0.01, 1.0, 0.02, "ab2", h_prev=Hn)
    assert np.abs(Ha - Hn).max() == 0.0
    assert np.abs(ua - ue).max() <= 1e-14
