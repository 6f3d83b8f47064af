"""The three-level workload at full size (32,380 cubes of 16^3, 132.6M cells), as configured.

* one projection, FP32 fields with FP64 refinement and all-FP64: the pressure's residual over
  every cell, evaluated by the oracle's whole-array operator (oracle/composite.py):
      ||b - A p||_V / ||b||_V <= 1.2e-10
  with b the right-hand side the GPU solved (FP32 fields: its u* is rounded to FP32) or the
  oracle's own b (FP64); and the GPU's b against the oracle's divergence of the same u* over
  every cell (2e-6 of max |b| with FP32 u*, 1e-12 in FP64).
* ten projections forward and their adjoint (pressure checkpoints, recompute in the
  backward), kinetic-energy objective: in FP64 with 1e-13 solves, the directional derivative
  along two seeded directions (alpha part U[-1, 1] per cell, U_in part +-1) against central
  finite differences of the FP64 forward, step 1e-6, to 1e-6 relative; with FP32 fields at
  the configured 1e-10, the gradient against the FP64 one (elementwise, relative to its
  largest value; FP32 storage of u, alpha and the cotangents bounds the agreement).
"""
import numpy as np
import pytest
import torch

from bcm_inputs import configs
from oracle.composite import CompositeMesh

from gpu_util import dev, host, log, plan_for, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

_CACHE = {}


def _inputs():
    if "pr" not in _CACHE:
        pr = configs.multilevel()
        _CACHE["pr"] = pr
        _CACHE["cm"] = CompositeMesh(pr["mesh"])
    return _CACHE["pr"], _CACHE["cm"]


@pytest.mark.parametrize("precision", ["mixed_f32fields", "fp64"])
def test_full_size_residual_over_every_cell(precision):
    pr, cm = _inputs()
    m = pr["mesh"]
    f32 = precision == "mixed_f32fields"
    log(f"multilevel full size {precision}: {m.n_cubes} cubes, {m.n_cells} cells")
    ft = torch.float32 if f32 else torch.float64
    u = pr["u"].reshape(3, -1)
    a = pr["alpha"].reshape(-1)
    if f32:
        u = u.astype(np.float32)
        a = a.astype(np.float32)
    plan = plan_for(m, precision)
    out = plan.project([dev(u[d], ft) for d in range(3)], dev(a, ft), pr["U_in"], pr["dt"],
                       pr["rho"], want_b=True)
    rep = out["report"]
    log(f"  its={rep.n_inner} outer={rep.n_outer} rel.res={rep.final_rel_res:.2e}")
    assert rep.status == 0 and rep.final_rel_res <= pr["tol"]
    p = host(out["p"])
    b = host(out["b"])
    del out, plan
    torch.cuda.empty_cache()
    c = pr["dt"] / pr["rho"]
    a64 = a.astype(np.float64)
    ustar = [(1.0 - a64) * u[d].astype(np.float64) for d in range(3)]
    del a64
    b_ref = cm.divergence(ustar, pr["U_in"]).ravel() / c
    del ustar
    bmax = np.abs(b_ref).max()
    db = np.abs(b - b_ref).max() / bmax
    res = cm.residual_norm(p, b if f32 else b_ref)
    log(f"  oracle: rel.res {res:.3e} over every cell; max|b - b_oracle|/max|b| {db:.2e}")
    assert db <= (2e-6 if f32 else 1e-12)
    assert res <= 1.2 * pr["tol"]


def _J(plan, pr, noise, alpha_t, U, steps):
    from paper_1808_04099_amd import MultiStepProjection, kinetic_energy
    u = MultiStepProjection.apply(noise[0] + U.to(noise[0].dtype), noise[1], noise[2], alpha_t,
                                  U, plan, pr["dt"], pr["rho"], steps)
    return kinetic_energy(u, plan, pr["rho"])


def test_full_size_ten_step_gradient():
    pr, _ = _inputs()
    m = pr["mesh"]
    K = pr["steps"]
    noise64 = pr["u"].reshape(3, -1).copy()
    noise64[0] -= pr["U_in"]
    alpha64 = pr["alpha"].reshape(-1)
    grads = {}
    for precision, tol in (("fp64", 1e-13), ("mixed_f32fields", pr["tol"])):
        f32 = precision == "mixed_f32fields"
        ft = torch.float32 if f32 else torch.float64
        log(f"multilevel full size, {K} steps forward + adjoint, {precision}, tol {tol}")
        plan = plan_for(m, precision, tol=tol, max_iter=80)
        noise = [dev(noise64[d], ft) for d in range(3)]
        a_t = dev(alpha64, ft).requires_grad_(True)
        U = torch.tensor(pr["U_in"], dtype=torch.float64, requires_grad=True)
        J = _J(plan, pr, noise, a_t, U, K)
        J.backward()
        torch.cuda.synchronize()
        grads[precision] = (J.item(), a_t.grad.detach().to(torch.float64), U.grad.item())
        log(f"  J={J.item():.15e} dJ/dU_in={U.grad.item():.12e}")
        if precision == "fp64":
            eps = 1e-6
            for k, (va, vU) in enumerate(configs.fd_directions(m.n_cells, seeds=(10, 11))):
                v = dev(va)
                with torch.no_grad():
                    Jp = _J(plan, pr, noise, dev(alpha64) + eps * v,
                            torch.tensor(pr["U_in"] + eps * vU, dtype=torch.float64), K).item()
                    Jm = _J(plan, pr, noise, dev(alpha64) - eps * v,
                            torch.tensor(pr["U_in"] - eps * vU, dtype=torch.float64), K).item()
                fd = (Jp - Jm) / (2 * eps)
                adj = float(torch.dot(grads["fp64"][1], v).item() + grads["fp64"][2] * vU)
                rel = abs(adj - fd) / abs(fd)
                log(f"  direction {k}: adjoint {adj:.12e} fd {fd:.12e} rel {rel:.2e}")
                assert rel <= 1e-6
                del v
        del plan, noise, a_t, J
        torch.cuda.empty_cache()
    J64, ga64, gU64 = grads["fp64"]
    J32, ga32, gU32 = grads["mixed_f32fields"]
    dJ = abs(J32 - J64) / abs(J64)
    dga = float((ga32 - ga64).abs().max() / ga64.abs().max())
    dgU = abs(gU32 - gU64) / abs(gU64)
    log(f"  FP32 fields vs FP64: J {dJ:.2e}, dJ/dalpha {dga:.2e} (max-relative), "
        f"dJ/dU_in {dgU:.2e}")
    assert dJ <= 1e-6 and dga <= 1e-5 and dgU <= 1e-5
