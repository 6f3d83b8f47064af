"""The whole-array composite operators (oracle/composite.py) against the assembled
finite-volume operators (oracle/fv.py), which the closed-form, brute-force and identity tests
pin: Laplacian, face-velocity divergence with every boundary kind and the inflow term, and
the volume-weighted residual norm, on uniform and three-level meshes."""
import numpy as np
import pytest

from bcm_inputs import CHANNEL_BC, OPEN_BC, configs, uniform_mesh, uniform_random_velocity
from oracle import FVMesh
from oracle.composite import CompositeMesh

from test_oracle_operators import _tiny_multilevel

MESHES = {
    "channel": lambda: uniform_mesh((3, 2, 2), 0.25, 4, CHANNEL_BC),
    "open": lambda: uniform_mesh((2, 2, 2), 0.5, 8, OPEN_BC),
    "mixed_bc": lambda: uniform_mesh((2, 3, 2), 0.25, 4, ("outflow", "inflow", "slip",
                                                          "outflow", "inflow", "slip")),
    "tiny_3level": _tiny_multilevel,
    "multilevel_small": lambda: configs.multilevel_small()["mesh"],
}


@pytest.mark.parametrize("which", sorted(MESHES))
def test_composite_operators_match_assembled(which):
    m = MESHES[which]()
    fv, cm = FVMesh(m), CompositeMesh(m)
    rng = np.random.default_rng(61)
    p = rng.standard_normal(m.n_cells)
    a1 = fv.A @ p
    a2 = cm.laplacian(p).ravel()
    assert np.abs(a1 - a2).max() <= 1e-12 * np.abs(a1).max()
    u = uniform_random_velocity(m, 62, 0.5, (0.3, -0.1, 0.2)).reshape(3, -1)
    U_in = 0.85
    d1 = fv.D @ fv.face_velocity(u, U_in)
    d2 = cm.divergence(u, U_in).ravel()
    assert np.abs(d1 - d2).max() <= 1e-12 * np.abs(d1).max()
    b = rng.standard_normal(m.n_cells)
    assert abs(cm.residual_norm(p, b) - fv.residual_norm(p, b)) <= 1e-12
