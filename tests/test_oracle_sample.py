"""The per-cell oracle (sample.py) against the assembled finite-volume oracle (fv.py)."""
import numpy as np
import pytest

from bcm_inputs import CHANNEL_BC, configs, uniform_mesh, uniform_random_velocity
from oracle import FVMesh
from oracle.sample import CellSampler

from test_oracle_operators import _tiny_multilevel


@pytest.mark.parametrize("which", ["channel", "tiny_3level", "multilevel_small"])
def test_sampler_matches_assembled_operators(which):
    m = {"channel": lambda: uniform_mesh((3, 2, 2), 0.25, 4, CHANNEL_BC),
         "tiny_3level": _tiny_multilevel,
         "multilevel_small": lambda: configs.multilevel_small()["mesh"]}[which]()
    fv = FVMesh(m)
    cs = CellSampler(m)
    rng = np.random.default_rng(2)
    p = rng.standard_normal(m.n_cells)
    u = uniform_random_velocity(m, 3).reshape(3, -1)
    U_in = 0.7
    Ap = fv.A @ p
    div = fv.D @ fv.face_velocity(u, U_in)
    gc = (fv.Gc @ (fv.G @ p)).reshape(3, -1)
    cells = np.unique(np.concatenate([rng.integers(0, m.n_cells, 60),
                                      cs.interface_cells(limit=60)]))
    for g in cells:
        assert abs(cs.laplacian(p, g) - Ap[g]) <= 1e-11 * np.abs(Ap).max()
        assert abs(cs.divergence(u, g, U_in) - div[g]) <= 1e-11 * np.abs(div).max()
        for d in range(3):
            assert abs(cs.cell_gradient(p, g, d) - gc[d, g]) <= 1e-11 * np.abs(gc).max()
