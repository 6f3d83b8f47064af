"""The no-allocation objective (bcm_kinetic_energy_noalloc) through the C ABI against
bcm_kinetic_energy: the same J bit for bit and the same seed cotangent, on two calls in a row,
the second on a smaller mesh (the file-scope scratch array keeps the first call's contents)."""
import ctypes

import numpy as np
import pytest
import torch

from bcm_inputs import CHANNEL_BC, configs, uniform_mesh, uniform_random_velocity

from gpu_util import dev, log, plan_for, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]


def _call(plan, name, u, rho, g_scale):
    from paper_1808_04099_amd import _lib as L
    lib = L.load()
    seed = [plan.empty() for _ in range(3)]
    J = ctypes.c_double(0.0)
    st = getattr(lib, name)(plan.handle, (ctypes.c_void_p * 3)(*[x.data_ptr() for x in u]),
                            float(rho), float(g_scale), ctypes.byref(J),
                            (ctypes.c_void_p * 3)(*[x.data_ptr() for x in seed]),
                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, lib.bcm_last_error().decode()
    torch.cuda.synchronize()
    return J.value, seed


@pytest.mark.parametrize("precision", ["fp64", "mixed_f32fields"])
def test_noalloc_objective_matches_workspace_objective(precision):
    meshes = [configs.multilevel_small()["mesh"], uniform_mesh((2, 1, 1), 0.5, 8, CHANNEL_BC)]
    assert meshes[1].n_cells < meshes[0].n_cells
    for k, m in enumerate(meshes):
        plan = plan_for(m, precision)
        u = uniform_random_velocity(m, 91 + k, 0.6, (1.0, 0.2, -0.3)).reshape(3, -1)
        ut = [dev(u[d], plan.field_dtype) for d in range(3)]
        J0, s0 = _call(plan, "bcm_kinetic_energy", ut, 1.2, 0.7)
        J1, s1 = _call(plan, "bcm_kinetic_energy_noalloc", ut, 1.2, 0.7)
        log(f"  call {k}: {m.n_cells} cells, J {J0:.15e} / {J1:.15e}")
        assert J1 == J0
        for d in range(3):
            assert torch.equal(s0[d], s1[d])
