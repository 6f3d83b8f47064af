"""Three-level meshes with 2:1 interfaces on the GPU.

* full size (32,380 cubes of 16^3, 132.6M cells), FP32 fields with FP64 refinement: the
  returned pressure, right-hand side, velocities and face velocities are checked at sampled
  cells (random cells plus cells on 2:1 interfaces and the domain boundary) with the per-cell
  oracle, using bounds that hold at any size:
    |r_i| sqrt(V_i) <= tol ||b||_V            (one cell's share of the 2-norm bound)
    |b_i - b_oracle_i| <= 2e-6 max|b|          (u* stored in FP32: 6e-8 relative rounding)
    |u_new - u_oracle| <= 1e-5 max|u|          (FP32 fields)
    |div_f U^{n+1} - (dt/rho) r_i| <= 1e-6 max|U| / h  (face identity, FP32 face velocities)
  The oracle evaluates everything from the FP32-rounded inputs the GPU receives.
* scaled-down three-level mesh: the 10-step kinetic-energy gradient (forward + adjoint with
  per-step pressure checkpoints) against the oracle's exact gradient, FP64 (1e-7) and FP32
  fields (1e-5: the FP32 storage of u, alpha and the cotangents bounds the agreement).
"""
import numpy as np
import pytest
import torch

from bcm_inputs import configs
from oracle import FVMesh, projection as OP
from oracle.sample import CellSampler

from gpu_util import dev, host, log, plan_for, rel_err, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]


def _cells(cs, m, seed=3, n_random=400, n_interface=400):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([rng.integers(0, m.n_cells, n_random),
                                     cs.interface_cells(limit=n_interface)]))


def test_full_size_multilevel_projection_sampled():
    pr = configs.multilevel()
    m = pr["mesh"]
    log(f"multilevel full size: {m.n_cubes} cubes, {m.n_cells} cells")
    u32 = pr["u"].astype(np.float32)
    a32 = pr["alpha"].astype(np.float32)
    plan = plan_for(m, "mixed_f32fields")
    out = plan.project([dev(u32[d], torch.float32) for d in range(3)], dev(a32, torch.float32),
                       pr["U_in"], pr["dt"], pr["rho"], face_u=True, want_b=True)
    rep = out["report"]
    log(f"  its={rep.n_inner} outer={rep.n_outer} rel.res={rep.final_rel_res:.2e}")
    assert rep.status == 0 and rep.final_rel_res <= pr["tol"]
    c = pr["dt"] / pr["rho"]
    vol = torch.from_numpy(np.repeat(m.h() ** 3, m.n ** 3)).to("cuda")
    bnorm = float(torch.sqrt((vol * out["b"] ** 2).sum()))
    bmax = float(out["b"].abs().max())
    cs = CellSampler(m)
    cells = _cells(cs, m)
    idx = torch.from_numpy(cells).to("cuda")
    # gather what the per-cell oracle needs: the sampled cells and their neighbours
    need = set(cells.tolist())
    for g in cells:
        for f in range(6):
            for nb, *_ in cs.subfaces(g, f):
                if nb is not None:
                    need.add(nb)
    need = np.array(sorted(need))
    nt = torch.from_numpy(need).to("cuda")
    p_s = dict(zip(need.tolist(), host(out["p"][nt]).tolist()))
    ustar = [dict(zip(need.tolist(), ((1 - a32.ravel()[need].astype(np.float64))
                                      * u32[d].ravel()[need].astype(np.float64)).tolist()))
             for d in range(3)]
    b_g = host(out["b"][idx])
    un = [host(out["u_new"][d][idx]) for d in range(3)]
    n = m.n
    fu = [out["face_u"][d].view(m.n_cubes, *[(n + (2 - d == a)) for a in range(3)])
          for d in range(3)]
    umax = float(np.abs(u32).max())
    worst = dict(res=0.0, b=0.0, u=0.0, div=0.0)
    for t, g in enumerate(cells):
        cb, i, j, k = cs.cell_of(g)
        V = cs.h_cube[cb] ** 3
        h = cs.h_cube[cb]
        r = b_g[t] - cs.laplacian(p_s, g)
        worst["res"] = max(worst["res"], abs(r) * np.sqrt(V) / (pr["tol"] * bnorm))
        b_ref = cs.divergence(ustar, g, pr["U_in"]) / c
        worst["b"] = max(worst["b"], abs(b_g[t] - b_ref) / (2e-6 * bmax))
        for d in range(3):
            u_ref = ustar[d][g] - c * cs.cell_gradient(p_s, g, d)
            worst["u"] = max(worst["u"], abs(un[d][t] - u_ref) / (1e-5 * umax))
        div = ((fu[0][cb, k, j, i + 1] - fu[0][cb, k, j, i]) + (fu[1][cb, k, j + 1, i]
               - fu[1][cb, k, j, i]) + (fu[2][cb, k + 1, j, i] - fu[2][cb, k, j, i])).item() / h
        worst["div"] = max(worst["div"], abs(div - c * r) / (1e-6 * umax / h))
    log(f"  sampled {cells.size} cells, worst ratio to bound: {worst}")
    assert all(v <= 1.0 for v in worst.values()), worst


@pytest.mark.parametrize("precision", ["fp64", "mixed_f32fields"])
def test_multilevel_multistep_gradient_matches_oracle(precision):
    from paper_1808_04099_amd import MultiStepProjection, kinetic_energy
    pr = configs.multilevel_small()
    m = pr["mesh"]
    steps = pr["steps"]
    f32 = precision == "mixed_f32fields"
    noise = pr["u"].reshape(3, -1).copy()
    noise[0] -= pr["U_in"]
    alpha = pr["alpha"].ravel()
    if f32:
        noise = noise.astype(np.float32).astype(np.float64)
        alpha = alpha.astype(np.float32).astype(np.float64)
    log(f"multilevel small gradient {precision}: {m.n_cubes} cubes, {steps} steps")
    fv = FVMesh(m)
    J_ref, ga_ref, gU_ref = OP.multistep_gradient(fv, noise, alpha, (0, 0, 0), pr["U_in"],
                                                  pr["dt"], pr["rho"], steps)
    plan = plan_for(m, precision, tol=1e-12)
    ft = plan.field_dtype
    vol = dev(np.repeat(m.h() ** 3, m.n ** 3))
    nz = [dev(noise[d], ft) for d in range(3)]
    a_t = dev(alpha, ft).requires_grad_(True)
    U = torch.tensor(pr["U_in"], dtype=torch.float64, requires_grad=True)
    u0 = [nz[0] + U.to(ft), nz[1], nz[2]]
    u = MultiStepProjection.apply(u0[0], u0[1], u0[2], a_t, U, plan, pr["dt"], pr["rho"], steps)
    J = kinetic_energy(u, plan, pr["rho"])
    J.backward()
    tol = 1e-5 if f32 else 1e-7
    log(f"  J gpu={J.item():.12e} oracle={J_ref:.12e}; dJ/dU gpu={U.grad.item():.10e} "
        f"oracle={gU_ref:.10e}; |dJ/dalpha| err={rel_err(host(a_t.grad), ga_ref):.2e}")
    assert abs(J.item() - J_ref) <= tol * abs(J_ref)
    assert rel_err(host(a_t.grad), ga_ref) <= tol
    assert abs(U.grad.item() - gU_ref) <= tol * abs(gU_ref)
