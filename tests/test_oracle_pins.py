"""Closed-form pins of the oracle's cell gradient, kinetic energy and array-form projection.

* cell gradient G_c (the correction's per-cell gradient, Sec. 3 velocity correction): on a
  single-level mesh the mean of the two face gradients of a separable DST-II / DCT-II / DCT-IV
  basis function along axis d is the closed form (sin(theta_d h) / h) times the derivative mode,
  boundary cells included (the ghost rules of each boundary kind continue the mode exactly).
  Both the assembled form (fv.Gc @ fv.G) and the array form (UniformGrid.cell_grad) are pinned.
  On the three-level mesh G_c of a field linear along axis d is that slope exactly in every cell
  whose two d-faces are interior, which pins the 2:1 face distance (3h/2) and the coarse-side
  weighting of the four fine sub-faces.
* kinetic energy J = (rho/2) sum_i V_i |u_i|^2: a constant velocity gives (rho/2)|u|^2 times
  the domain volume on any mesh (every level's V_i), and u_x = x on a uniform grid gives the
  midpoint-rule closed form (rho/2) * Ly Lz * (Lx^3/3 - Lx h^2/12).
* UniformGrid.project (the array-form oracle used at full size) against projection.project
  (the assembled sparse form) on a channel and on the open box.
"""
import numpy as np
import pytest

from bcm_inputs import CHANNEL_BC, OPEN_BC, configs, uniform_mesh, uniform_random_velocity
from oracle import FVMesh, UniformGrid, projection as P

BCS = {"open": OPEN_BC, "channel": CHANNEL_BC,
       "mixed": ("outflow", "inflow", "slip", "outflow", "inflow", "slip")}


def _basis(kind, k, L):
    """(mode, derivative of mode, angular frequency w) of one separable basis function."""
    w = {"dst2": np.pi * (k + 1), "dct2": np.pi * k, "dct4": np.pi * (k + 0.5),
         "dst4": np.pi * (k + 0.5)}[kind] / L
    if kind in ("dst2", "dst4"):
        return (lambda x: np.sin(w * x)), (lambda x: w * np.cos(w * x)), w
    return (lambda x: np.cos(w * x)), (lambda x: -w * np.sin(w * x)), w


def _kind(lo, hi):
    dl, dh = lo == "outflow", hi == "outflow"
    return {(True, True): "dst2", (False, False): "dct2", (False, True): "dct4",
            (True, False): "dst4"}[(dl, dh)]


@pytest.mark.parametrize("bc", sorted(BCS))
@pytest.mark.parametrize("k", [(0, 1, 2), (3, 0, 1), (5, 4, 3)])
def test_cell_gradient_closed_form(bc, k):
    m = uniform_mesh((3, 2, 2), 0.25, 4, BCS[bc])
    fv, ug = FVMesh(m), UniformGrid(m)
    X, Y, Z = m.cell_centres()
    C = (X.ravel(), Y.ravel(), Z.ravel())
    L = np.subtract(m.domain_hi, m.domain_lo)
    h = float(m.h()[0])
    parts = [_basis(_kind(BCS[bc][2 * d], BCS[bc][2 * d + 1]), k[d], L[d]) for d in range(3)]
    p = np.prod([parts[d][0](C[d]) for d in range(3)], axis=0)
    gc = (fv.Gc @ (fv.G @ p)).reshape(3, -1)
    scale = max(np.abs(p).max(), 1e-300) / h
    for d in range(3):
        f, df, w = parts[d]
        # discrete derivative of the mode: (f(x+h) - f(x-h)) / 2h = f'(x) sin(w h) / (w h)
        expect = df(C[d]) * (np.sin(w * h) / (w * h) if w else 1.0)
        for e in range(3):
            if e != d:
                expect = expect * parts[e][0](C[e])
        assert np.abs(gc[d] - expect).max() <= 1e-12 * scale, (bc, k, d)
        arr = ug.to_cubes(ug.cell_grad(ug.to_global(p), d)).ravel()
        assert np.abs(arr - expect).max() <= 1e-12 * scale, (bc, k, d)


def test_cell_gradient_linear_on_three_levels():
    m = configs.multilevel_small()["mesh"]
    assert set(np.unique(m.level)) == {0, 1, 2}
    fv = FVMesh(m)
    X, Y, Z = m.cell_centres()
    C = (X.ravel(), Y.ravel(), Z.ravel())
    for d, slope in enumerate((1.7, -0.6, 2.3)):
        p = slope * C[d] + 0.3
        gc = (fv.Gc @ (fv.G @ p)).reshape(3, -1)
        # cells with a domain-boundary face normal to d see the boundary rule, not the slope
        bnd = ((fv.L < 0) | (fv.R < 0)) & (fv.axis == d)
        touch = np.zeros(m.n_cells, bool)
        touch[fv.L[bnd & (fv.L >= 0)]] = True
        touch[fv.R[bnd & (fv.R >= 0)]] = True
        # cells next to a 2:1 interface normal to d are included: that is what is pinned
        inner = (fv.L >= 0) & (fv.R >= 0) & (fv.axis == d)
        iface = inner & (np.abs(fv.dist - fv.h_cell[np.maximum(fv.L, 0)]) > 1e-12)
        assert iface.any()
        ok = ~touch
        assert np.abs(gc[d][ok] - slope).max() <= 1e-11 * abs(slope)


@pytest.mark.parametrize("which", ["uniform", "multilevel_small"])
def test_kinetic_energy_of_constant_velocity(which):
    m = (uniform_mesh((4, 2, 2), 0.25, 4, CHANNEL_BC) if which == "uniform"
         else configs.multilevel_small()["mesh"])
    fv = FVMesh(m)
    U = np.array([1.3, -0.4, 0.7])
    u = np.broadcast_to(U[:, None], (3, m.n_cells)).copy()
    rho = 1.7
    vol = float(np.prod(np.subtract(m.domain_hi, m.domain_lo)))
    J = P.kinetic_energy(fv, u, rho)
    assert abs(J - 0.5 * rho * float(U @ U) * vol) <= 1e-13 * J


def test_kinetic_energy_of_linear_velocity():
    m = uniform_mesh((4, 2, 2), 0.25, 8, CHANNEL_BC)
    fv = FVMesh(m)
    X, _, _ = m.cell_centres()
    u = np.zeros((3, m.n_cells))
    u[0] = X.ravel()
    h = float(m.h()[0])
    Lx, Ly, Lz = np.subtract(m.domain_hi, m.domain_lo)
    rho = 0.9
    expect = 0.5 * rho * Ly * Lz * (Lx ** 3 / 3 - Lx * h ** 2 / 12)
    assert abs(P.kinetic_energy(fv, u, rho) - expect) <= 1e-13 * expect


@pytest.mark.parametrize("bc", ["channel", "open"])
def test_uniform_projection_matches_assembled(bc):
    m = uniform_mesh((4, 2, 2), 0.25, 8, BCS[bc])
    fv, ug = FVMesh(m), UniformGrid(m)
    rng = np.random.default_rng(21)
    u = uniform_random_velocity(m, 22, 0.4, (1.0, 0.0, 0.0))
    alpha = rng.uniform(0.0, 1.0, (m.n_cubes, m.n, m.n, m.n))
    us, U_in, dt, rho = (0.1, -0.2, 0.05), 0.8, 0.01, 1.2
    a = P.project(fv, u, alpha.ravel(), us, U_in, dt, rho)
    b = ug.project(u, alpha, us, U_in, dt, rho)
    for key in ("b", "p"):
        ref = a[key]
        assert np.abs(b[key].ravel() - ref).max() <= 1e-13 * np.abs(ref).max(), key
    ref = a["u_new"]
    assert np.abs(b["u_new"].reshape(3, -1) - ref).max() <= 1e-13 * np.abs(ref).max()
