"""Pins of the FP64 oracle's operators against closed forms and independent formulations.

* two independently written formulations agree: assembled finite-volume faces (fv.py) and
  array slicing on one global grid (uniform.py);
* discrete eigenmodes: the 7-point operator maps the DST/DCT basis functions of each boundary
  kind to lambda * mode (closed form);
* brute force: a per-cell ghost-value loop written from the boundary and 2:1 interface rules
  reproduces the assembled operator, including a three-level mesh;
* identities: V A symmetric, telescoping divergence, consistency on constants.
"""
import numpy as np
import pytest

from bcm_inputs import CHANNEL_BC, OPEN_BC, build_mesh, uniform_mesh, uniform_random_velocity
from oracle import FVMesh, UniformGrid

BCS = {"open": OPEN_BC, "channel": CHANNEL_BC,
       "mixed": ("outflow", "inflow", "slip", "outflow", "inflow", "slip")}


@pytest.mark.parametrize("bc", sorted(BCS))
def test_fv_and_array_forms_agree(bc):
    m = uniform_mesh((3, 2, 2), 0.25, 4, BCS[bc])
    fv, ug = FVMesh(m), UniformGrid(m)
    rng = np.random.default_rng(1)
    p = rng.standard_normal(m.n_cells)
    a1 = fv.A @ p
    a2 = ug.to_cubes(ug.laplacian(ug.to_global(p))).ravel()
    assert np.abs(a1 - a2).max() <= 1e-13 * np.abs(a1).max()
    u = uniform_random_velocity(m, 2)
    U_in = 0.7
    Uf = fv.face_velocity(u, U_in)
    d1 = fv.D @ Uf
    d2 = ug.to_cubes(ug.div([ug.face_velocity(ug.to_global(u[d]), d, U_in)
                             for d in range(3)])).ravel()
    assert np.abs(d1 - d2).max() <= 1e-13 * np.abs(d1).max()
    gc = (fv.Gc @ (fv.G @ p)).reshape(3, -1)
    for d in range(3):
        g2 = ug.to_cubes(ug.cell_grad(ug.to_global(p), d)).ravel()
        assert np.abs(gc[d] - g2).max() <= 1e-13 * np.abs(g2).max()


def _mode(x, L, kind, k):
    t = x / L
    if kind == "dst2":
        return np.sin(np.pi * (k + 1) * t)
    if kind == "dct2":
        return np.cos(np.pi * k * t)
    if kind == "dct4":
        return np.cos(np.pi * (k + 0.5) * t)
    return np.sin(np.pi * (k + 0.5) * t)


def _kind(lo, hi):
    dl, dh = lo == "outflow", hi == "outflow"
    return {(True, True): "dst2", (False, False): "dct2", (False, True): "dct4",
            (True, False): "dst4"}[(dl, dh)]


@pytest.mark.parametrize("bc", sorted(BCS))
@pytest.mark.parametrize("k", [(0, 0, 0), (1, 2, 3), (5, 0, 2), (11, 7, 6)])
def test_eigenmodes_closed_form(bc, k):
    """A applied to a separable basis function returns sum_d (2 cos theta_d - 2)/h^2 times it."""
    m = uniform_mesh((3, 2, 2), 0.25, 4, BCS[bc])
    fv = FVMesh(m)
    X, Y, Z = m.cell_centres()
    L = np.subtract(m.domain_hi, m.domain_lo)
    N = np.rint(L / m.h()[0]).astype(int)
    h = m.h()[0]
    mode = np.ones_like(X)
    lam = 0.0
    for d, C in enumerate((X, Y, Z)):
        kind = _kind(BCS[bc][2 * d], BCS[bc][2 * d + 1])
        kd = k[d] % N[d]
        mode = mode * _mode(C, L[d], kind, kd)
        shift = {"dst2": 1.0, "dct2": 0.0, "dct4": 0.5, "dst4": 0.5}[kind]
        lam += (2 * np.cos(np.pi * (kd + shift) / N[d]) - 2) / h ** 2
    Am = fv.A @ mode.ravel()
    assert np.abs(Am - lam * mode.ravel()).max() <= 1e-11 * max(abs(lam), 1.0)


def test_manufactured_solution_closed_form():
    """p = sin(pi x) sin(2 pi y) sin(3 pi z) is an eigenmode of the discrete operator on the
    open unit box, so the discrete solution is p_h = (-14 pi^2 / lambda_h) p exactly."""
    from bcm_inputs.configs import small_box
    pr = small_box()
    m = pr["mesh"]
    fv = FVMesh(m)
    h = 1.0 / 64
    lam_h = sum(2 * np.cos(k * np.pi * h) - 2 for k in (1, 2, 3)) / h ** 2
    assert abs(lam_h - (-137.98037223710435)) < 1e-9
    X, Y, Z = m.cell_centres()
    pe = (np.sin(np.pi * X) * np.sin(2 * np.pi * Y) * np.sin(3 * np.pi * Z)).ravel()
    p = fv.solve(pr["b"].ravel())
    ratio = -14 * np.pi ** 2 / lam_h
    assert abs(ratio - 1 - 1.40664e-3) < 1e-8
    assert np.abs(p - ratio * pe).max() <= 1e-13
    assert fv.residual_norm(p, pr["b"].ravel()) <= 1e-13


# ---------------------------------------------------------------------------------------------
# Brute force: the operator written cell by cell with ghost values (boundary and 2:1 rules).
# ---------------------------------------------------------------------------------------------
def _brute_laplacian(m, p):
    """(A p)_i = sum over the 6 sides of (g - p_i)/h^2 with ghost g from the neighbour cells:
    same level -> neighbour cell; open boundary -> -p_i; Neumann boundary -> p_i;
    fine cell next to a coarse cell P -> p_i/3 + 2 P/3; coarse cell next to 4 fine cells ->
    4/3 mean(fine) - p_i/3.  Cells are located by their centre coordinates."""
    n = m.n
    X, Y, Z = m.cell_centres()
    cen = np.stack([X, Y, Z], -1).reshape(-1, 3)
    h = np.repeat(m.h(), n ** 3)
    lo = np.asarray(m.domain_lo)
    hi = np.asarray(m.domain_hi)
    # locate cells: integer index of each cell's centre on its own level grid
    index = {}
    for i in range(cen.shape[0]):
        key = (round(h[i] * 1e9),) + tuple(np.floor((cen[i] - lo) / h[i]).astype(int))
        index[key] = i
    side_bc = m.meta["side_bc"]
    out = np.zeros_like(p)
    for i in range(cen.shape[0]):
        acc = 0.0
        for f in range(6):
            d, s = divmod(f, 2)
            sgn = 1 if s else -1
            q = cen[i].copy()
            q[d] += sgn * h[i]
            if q[d] < lo[d] or q[d] > hi[d]:
                g = -p[i] if side_bc[f] == "outflow" else p[i]
            else:
                same = (round(h[i] * 1e9),) + tuple(np.floor((q - lo) / h[i]).astype(int))
                if same in index:
                    g = p[index[same]]
                else:
                    H = 2 * h[i]
                    qc = cen[i].copy()
                    qc[d] += sgn * (h[i] / 2 + h[i])        # centre of the coarse cell
                    coarse = (round(H * 1e9),) + tuple(np.floor((qc - lo) / H).astype(int))
                    if coarse in index:
                        g = p[i] / 3 + 2 * p[index[coarse]] / 3
                    else:
                        hf = h[i] / 2
                        vals = []
                        for a in (-0.5, 0.5):
                            for b in (-0.5, 0.5):
                                qf = cen[i].copy()
                                qf[d] += sgn * (h[i] / 2 + hf / 2)
                                t1, t2 = [t for t in range(3) if t != d]
                                qf[t1] += a * hf
                                qf[t2] += b * hf
                                key = (round(hf * 1e9),) + tuple(
                                    np.floor((qf - lo) / hf).astype(int))
                                vals.append(p[index[key]])
                        g = 4.0 / 3.0 * np.mean(vals) - p[i] / 3
            acc += (g - p[i]) / h[i] ** 2
        out[i] = acc
    return out


def _tiny_multilevel():
    # one level-0 cube split in two steps next to an unsplit neighbour -> 3 levels
    def refine(level, lo, hi):
        return lo[0] < 0.5 and (level == 0 or (lo[0] < 0.2 and lo[1] < 0.2 and lo[2] < 0.2))
    return build_mesh((2, 1, 1), 0.5, 2, ("inflow", "outflow", "slip", "outflow", "slip",
                                          "slip"), refine=refine, max_level=2)


@pytest.mark.parametrize("which", ["uniform", "multilevel"])
def test_brute_force_ghost_loop_matches_assembled(which):
    m = uniform_mesh((2, 2, 2), 0.5, 4, CHANNEL_BC) if which == "uniform" else _tiny_multilevel()
    if which == "multilevel":
        assert set(np.unique(m.level)) == {0, 1, 2}
    fv = FVMesh(m)
    rng = np.random.default_rng(3)
    p = rng.standard_normal(m.n_cells)
    a = fv.A @ p
    assert np.abs(a - _brute_laplacian(m, p)).max() <= 1e-12 * np.abs(a).max()
    # dense solve agrees with the oracle's solve
    b = rng.standard_normal(m.n_cells)
    dense = np.linalg.solve(fv.A.toarray(), b)
    assert np.abs(dense - fv.solve(b)).max() <= 1e-11 * np.abs(dense).max()


def test_multilevel_identities():
    from bcm_inputs.configs import multilevel_small
    m = multilevel_small()["mesh"]
    assert set(np.unique(m.level)) == {0, 1, 2}
    fv = FVMesh(m)
    VA = fv.A.T.multiply(fv.V[None, :]).T.tocsr()
    assert abs(VA - VA.T).max() <= 1e-12 * abs(VA).max()
    # telescoping: sum_i V_i (D U)_i = net outward flux through the domain boundary
    rng = np.random.default_rng(4)
    U = rng.standard_normal(fv.n_faces)
    bnd = (fv.L < 0) | (fv.R < 0)
    outward = np.where(fv.R < 0, 1.0, -1.0)
    lhs = np.sum(fv.V * (fv.D @ U))
    rhs = np.sum((outward * fv.area * U)[bnd])
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(fv.area * U))
    # a constant velocity has zero divergence in every cell away from the domain boundary
    u = np.zeros((3, m.n_cells))
    u[0] = 1.3
    u[1] = -0.4
    u[2] = 0.25
    div = fv.D @ fv.face_velocity(u, 0.0)
    touches = np.zeros(m.n_cells, bool)
    touches[fv.L[bnd & (fv.L >= 0)]] = True
    touches[fv.R[bnd & (fv.R >= 0)]] = True
    assert np.abs(div[~touches]).max() <= 1e-10
    # constants are annihilated by the Laplacian in cells with no open boundary face
    ones = np.ones(m.n_cells)
    assert np.abs((fv.A @ ones)[~touches]).max() <= 1e-8
