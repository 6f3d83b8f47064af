"""GPU parity of the momentum sub-step (bcm_momentum) against the oracle (oracle/momentum.py).

* H(u^n) and one Euler step, element by element, on meshes with every boundary kind, cube
  sizes 4, 8 and 16 and several cubes per workgroup (ragged last group): 1e-12 relative in
  FP64 fields, 2e-6 with FP32 fields (the oracle evaluates the FP32-rounded inputs);
* AB2 from the H of a previous step;
* Crank-Nicolson: Jacobi iterations to 1e-13 against the oracle's exact solve (BiCGSTAB to
  1e-14), with the iteration history; an iteration limit gives BCM_NOT_CONVERGED;
* multi-level meshes are refused (BCM_ERR_UNSUPPORTED);
* one whole fractional step on the 16x8x8-cube sphere channel (4.2M cells): Crank-Nicolson
  momentum, then forcing, Poisson solve and correction, against the oracle's momentum step
  followed by its exact spectral projection.
"""
import numpy as np
import pytest
import torch

from bcm_inputs import CHANNEL_BC, OPEN_BC, configs, uniform_mesh, uniform_random_velocity
from oracle import UniformGrid
from oracle.momentum import step

from gpu_util import dev, host, log, plan_for, rel_err, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

MESHES = {
    "channel_n8": lambda: uniform_mesh((4, 2, 2), 0.25, 8, CHANNEL_BC),
    "open_n4_ragged": lambda: uniform_mesh((3, 3, 2), 1.0 / 3, 4, OPEN_BC),
    "mixed_bc_n4": lambda: uniform_mesh((2, 3, 2), 0.25, 4, ("outflow", "inflow", "slip",
                                                             "outflow", "inflow", "slip")),
    "channel_n16": lambda: uniform_mesh((3, 2, 1), 0.5, 16, CHANNEL_BC),
}


def _inputs(m, seed=81):
    u = uniform_random_velocity(m, seed, 0.4, (0.8, 0.1, -0.1)).reshape(3, -1)
    hp = uniform_random_velocity(m, seed + 1, 2.0).reshape(3, -1)
    return u, hp


def _run(plan, u, **kw):
    ft = plan.field_dtype
    out = plan.momentum([dev(u[d], ft) for d in range(3)], **kw)
    return np.stack([host(x) for x in out["u_tilde"]]), (
        np.stack([host(x) for x in out["h"]]) if out["h"] else None), out["report"]


@pytest.mark.parametrize("precision", ["fp64", "mixed_f32fields"])
@pytest.mark.parametrize("name", sorted(MESHES))
def test_euler_and_operator_match_oracle(name, precision):
    m = MESHES[name]()
    f32 = precision == "mixed_f32fields"
    u, _ = _inputs(m)
    if f32:
        u = u.astype(np.float32).astype(np.float64)
    nu, U_in, dt = 0.02, 0.9, 0.01
    log(f"momentum euler {name} {precision}")
    plan = plan_for(m, precision)
    ut, H, rep = _run(plan, u, U_in=U_in, dt=dt, nu=nu, scheme="euler", want_h=True)
    ut_ref, H_ref = step(m, u, nu, U_in, dt, "euler")
    tol = 2e-6 if f32 else 1e-12
    eh, eu = rel_err(H, H_ref), rel_err(ut, ut_ref)
    log(f"  H err {eh:.2e}, u~ err {eu:.2e}")
    assert rep.status == 0 and eh <= tol and eu <= tol


@pytest.mark.parametrize("name", ["channel_n8", "mixed_bc_n4"])
def test_ab2_matches_oracle(name):
    m = MESHES[name]()
    u, hp = _inputs(m, 83)
    nu, U_in, dt = 0.01, 1.1, 0.02
    plan = plan_for(m, "fp64")
    ft = plan.field_dtype
    ut, H, rep = _run(plan, u, U_in=U_in, dt=dt, nu=nu, scheme="ab2",
                      h_prev=[dev(hp[d], ft) for d in range(3)], want_h=True)
    ut_ref, H_ref = step(m, u, nu, U_in, dt, "ab2", h_prev=hp)
    assert rel_err(H, H_ref) <= 1e-12 and rel_err(ut, ut_ref) <= 1e-12
    # without h_prev (first step) AB2 is the Euler step
    ut1, _, _ = _run(plan, u, U_in=U_in, dt=dt, nu=nu, scheme="ab2")
    ue, _ = step(m, u, nu, U_in, dt, "euler")
    assert rel_err(ut1, ue) <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "mixed_f32fields"])
@pytest.mark.parametrize("name", ["channel_n8", "open_n4_ragged", "channel_n16"])
def test_crank_nicolson_matches_oracle(name, precision):
    m = MESHES[name]()
    f32 = precision == "mixed_f32fields"
    u, _ = _inputs(m, 85)
    if f32:
        u = u.astype(np.float32).astype(np.float64)
    h = float(m.h()[0])
    nu, U_in = 0.01, 0.9
    dt = 0.5 * h / 1.0
    log(f"momentum cn {name} {precision}")
    plan = plan_for(m, precision)
    ut, H, rep = _run(plan, u, U_in=U_in, dt=dt, nu=nu, scheme="cn", cn_tol=1e-6 if f32 else 1e-13,
                      want_h=True)
    ut_ref, H_ref = step(m, u, nu, U_in, dt, "cn")
    err = rel_err(ut, ut_ref)
    log(f"  its {rep.n_inner} final {rep.final_rel_res:.2e} history {len(rep.history)}; "
        f"u~ err {err:.2e}")
    assert rep.status == 0 and rep.n_inner == len(rep.history)
    assert rep.final_rel_res <= (1e-6 if f32 else 1e-13)
    assert err <= (2e-6 if f32 else 1e-11)
    assert rel_err(H, H_ref) <= (2e-6 if f32 else 1e-12)


def test_crank_nicolson_iteration_limit():
    m = MESHES["channel_n8"]()
    u, _ = _inputs(m, 87)
    plan = plan_for(m, "fp64")
    _, _, rep = _run(plan, u, U_in=1.0, dt=0.02, nu=0.01, scheme="cn", cn_tol=1e-14,
                     cn_max_iter=3)
    assert rep.status == 1 and rep.n_inner == 3 and rep.final_rel_res > 1e-14


def test_multilevel_mesh_is_refused():
    from paper_1808_04099_amd import BCMError
    m = configs.multilevel_small()["mesh"]
    plan = plan_for(m, "fp64")
    u = np.zeros((3, m.n_cells))
    with pytest.raises(BCMError) as e:
        _run(plan, u, U_in=1.0, dt=0.01, nu=0.01, scheme="euler")
    assert e.value.status == -6


def test_fractional_step_sphere_channel():
    """16x8x8 cubes of 16^3 (4.2M cells): u^n -> Crank-Nicolson momentum -> forcing -> Poisson
    (1e-10) -> correction, against the oracle's momentum step and exact spectral projection."""
    pr = configs.sphere_channel()
    m = pr["mesh"]
    nu = 1e-3
    u = pr["u"].reshape(3, -1)
    log(f"fractional step: {m.n_cells} cells, nu {nu}, dt {pr['dt']}")
    plan = plan_for(m, "fp64")
    mo = plan.momentum([dev(u[d]) for d in range(3)], U_in=pr["U_in"], dt=pr["dt"], nu=nu,
                       scheme="cn", cn_tol=1e-13)
    rep_m = mo["report"]
    out = plan.project(mo["u_tilde"], dev(pr["alpha"]), pr["U_in"], pr["dt"], pr["rho"])
    rep = out["report"]
    log(f"  momentum: {rep_m.n_inner} iterations, {rep_m.final_rel_res:.1e}; "
        f"projection: {rep.n_inner} its, {rep.final_rel_res:.1e}")
    assert rep_m.status == 0 and rep.status == 0
    ut_ref, _ = step(m, u, nu, pr["U_in"], pr["dt"], "cn")
    ut = np.stack([host(x) for x in mo["u_tilde"]])
    e_ut = rel_err(ut, ut_ref)
    ref = UniformGrid(m).project(ut_ref.reshape(3, m.n_cubes, m.n, m.n, m.n), pr["alpha"],
                                 (0.0, 0.0, 0.0), pr["U_in"], pr["dt"], pr["rho"])
    un = np.stack([host(x) for x in out["u_new"]])
    e_u = rel_err(un, ref["u_new"].reshape(3, -1))
    e_p = rel_err(host(out["p"]), ref["p"].ravel())
    log(f"  u~ err {e_ut:.2e}, u^(n+1) err {e_u:.2e}, p err {e_p:.2e}")
    assert e_ut <= 1e-11 and e_u <= 1e-7 and e_p <= 1e-7
