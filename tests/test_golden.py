"""Stored expected values (tests/golden/, written by tests/golden/make_golden.py from closed
forms and the oracle only): the oracle must keep reproducing them, and the GPU must match."""
import json
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

from make_golden import SAMPLE, tiny_channel_inputs  # noqa: E402

from gpu_util import dev, host, plan_for, requires_gpu  # noqa: E402


def _gold(name):
    return json.load(open(os.path.join(HERE, "golden", name)))


def test_manufactured_constants():
    g = _gold("manufactured_box.json")
    assert abs(g["lambda_h"] - (-137.98037)) < 1e-5
    assert abs(g["ratio_minus_one"] - 1.40664e-3) < 1e-8


def test_oracle_reproduces_tiny_channel():
    from oracle import FVMesh, projection as OP
    g = _gold("tiny_channel.json")
    m, u, alpha, prm = tiny_channel_inputs()
    fv = FVMesh(m)
    r = OP.project(fv, u, alpha, (0, 0, 0), prm["U_in"], prm["dt"], prm["rho"])
    assert np.allclose(r["p"][SAMPLE], g["p"], rtol=1e-12, atol=1e-14)
    assert np.allclose(r["u_new"][:, SAMPLE], g["u_new"], rtol=1e-12, atol=1e-14)


@pytest.mark.gpu
@requires_gpu
def test_gpu_matches_tiny_channel_golden():
    import torch
    from paper_1808_04099_amd import MultiStepProjection, kinetic_energy
    g = _gold("tiny_channel.json")
    m, u, alpha, prm = tiny_channel_inputs()
    plan = plan_for(m, "fp64", tol=1e-13)
    out = plan.project([dev(u[d]) for d in range(3)], dev(alpha), prm["U_in"], prm["dt"],
                       prm["rho"])
    assert np.allclose(host(out["p"])[SAMPLE], g["p"], rtol=1e-9, atol=1e-12)
    un = np.stack([host(x) for x in out["u_new"]])
    assert np.allclose(un[:, SAMPLE], g["u_new"], rtol=1e-9, atol=1e-12)
    noise = u.reshape(3, -1).copy()
    noise[0] -= prm["U_in"]
    a_t = dev(alpha).requires_grad_(True)
    U = torch.tensor(prm["U_in"], dtype=torch.float64, requires_grad=True)
    nz = [dev(noise[d]) for d in range(3)]
    ul = MultiStepProjection.apply(nz[0] + U, nz[1], nz[2], a_t, U, plan, prm["dt"], prm["rho"],
                                   prm["steps"])
    vol = dev(np.repeat(m.h() ** 3, m.n ** 3))
    J = kinetic_energy(ul, plan, prm["rho"])
    J.backward()
    assert abs(J.item() - g["J"]) <= 1e-10 * abs(g["J"])
    assert np.allclose(host(a_t.grad)[SAMPLE], g["g_alpha"], rtol=1e-7,
                       atol=1e-9 * np.abs(g["g_alpha"]).max())
    assert abs(U.grad.item() - g["g_U_in"]) <= 1e-8 * abs(g["g_U_in"])
