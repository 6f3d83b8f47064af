"""GPU parity of the projection step (forcing -> Poisson -> correction) against the oracle.

Tolerances: the pressure comes from a solve to relative residual tol, so the GPU result
differs from the oracle's exact solve by at most ||e|| <= ||r|| / lambda_min; the velocity
error is c G_c e.  Both are checked with a fixed 1e-7 relative bound (FP64 fields) or 1e-5
(FP32 fields, which round u to 6e-8 relative).  The face velocities are checked against the
exact discrete identity div_f U^{n+1} = (dt/rho) r of the returned pressure.
"""
import numpy as np
import pytest

from bcm_inputs import CHANNEL_BC, configs, uniform_mesh, uniform_random_velocity
from oracle import FVMesh, projection as OP

from gpu_util import dev, host, log, plan_for, rel_err, requires_gpu
from test_oracle_operators import _tiny_multilevel

pytestmark = [pytest.mark.gpu, requires_gpu]


def _case(name):
    if name == "channel_n8":
        m = uniform_mesh((4, 2, 2), 0.25, 8, CHANNEL_BC)
    elif name == "tiny_3level_n2":
        m = _tiny_multilevel()
    elif name == "multilevel_small_n4":
        m = configs.multilevel_small()["mesh"]
    elif name == "box_open_n16":
        m = configs.small_box()["mesh"]
    rng = np.random.default_rng(21)
    u = uniform_random_velocity(m, 22, 0.3, (1.0, 0.0, 0.0))
    alpha = np.clip(rng.uniform(-0.5, 1.5, m.n_cells), 0.0, 1.0)
    return m, u, alpha


def _face_divergence(m, face_u):
    """div of the returned per-cube face velocities, per cell (cube-local differences)."""
    n = m.n
    h = np.repeat(m.h(), n ** 3).reshape(m.n_cubes, n, n, n)
    fx = face_u[0].reshape(m.n_cubes, n, n, n + 1)
    fy = face_u[1].reshape(m.n_cubes, n, n + 1, n)
    fz = face_u[2].reshape(m.n_cubes, n + 1, n, n)
    return ((np.diff(fx, axis=3) + np.diff(fy, axis=2) + np.diff(fz, axis=1)) / h).ravel()


@pytest.mark.parametrize("name", ["channel_n8", "tiny_3level_n2", "multilevel_small_n4",
                                  "box_open_n16"])
@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_f32fields"])
def test_projection_matches_oracle(name, precision):
    m, u, alpha = _case(name)
    log(f"projection {name} {precision}: {m.n_cubes} cubes")
    U_in, dt, rho, us = 1.0, 0.3 * float(m.h().min()), 1.2, (0.05, -0.02, 0.01)
    f32 = precision == "mixed_f32fields"
    if f32:   # the oracle sees exactly the fields the GPU sees
        u = u.astype(np.float32).astype(np.float64)
        alpha = alpha.astype(np.float32).astype(np.float64)
    fv = FVMesh(m)
    ref = OP.project(fv, u, alpha, us, U_in, dt, rho)
    plan = plan_for(m, precision)
    ft = plan.field_dtype
    out = plan.project([dev(u[d], ft) for d in range(3)], dev(alpha, ft), U_in, dt, rho, us=us,
                       face_u=True, want_b=True)
    rep = out["report"]
    p = host(out["p"])
    b = host(out["b"])
    unew = np.stack([host(x) for x in out["u_new"]])
    rr = fv.residual_norm(p, b)
    log(f"  its={rep.n_inner} outer={rep.n_outer} reported={rep.final_rel_res:.2e} "
        f"oracle={rr:.2e} |b-b_ref|={rel_err(b, ref['b']):.2e}")
    # the solve: residual of the returned pressure for the right-hand side it solved
    assert rep.status == 0 and rr <= 1.2e-10
    # the right-hand side: FP64 fields agree to rounding; FP32 fields store u* rounded to
    # 6e-8 relative, which the divergence turns into ~1e-7 of max|b|
    assert rel_err(b, ref["b"]) <= (2e-6 if f32 else 1e-12)
    tol = 1e-5 if f32 else 1e-7
    assert rel_err(unew, ref["u_new"]) <= tol
    assert rel_err(p, ref["p"]) <= tol
    # the corrected face velocities are divergence free up to c times the final residual
    div = _face_divergence(m, [host(x) for x in out["face_u"]])
    c = dt / rho
    res = c * (b - fv.A @ p)
    scale = np.abs(fv.D @ ref["U_star"]).max()
    assert np.abs(div - res).max() <= (1e-6 if f32 else 1e-10) * scale


@pytest.mark.parametrize("precision", ["fp64", "mixed_f32fields"])
def test_cell_only_correction_matches_face_output_path(precision):
    """16^3 cubes: the correction without face output (column kernels) and with it (tile
    kernels) give the same cell velocities; forcing and divergence against the oracle."""
    m = uniform_mesh((4, 2, 2), 0.25, 16, CHANNEL_BC)
    rng = np.random.default_rng(5)
    u = uniform_random_velocity(m, 6, 0.3, (1.0, 0.0, 0.0))
    alpha = rng.uniform(0.0, 1.0, m.n_cells)
    f32 = precision == "mixed_f32fields"
    if f32:
        u = u.astype(np.float32).astype(np.float64)
        alpha = alpha.astype(np.float32).astype(np.float64)
    plan = plan_for(m, precision)
    ft = plan.field_dtype
    args = ([dev(u[d], ft) for d in range(3)], dev(alpha, ft), 0.8, 0.004, 1.0)
    a = plan.project(*args, face_u=True, want_b=True)
    b = plan.project(*args, face_u=False, want_b=True)
    ua = np.stack([host(x) for x in a["u_new"]])
    ub = np.stack([host(x) for x in b["u_new"]])
    assert rel_err(ub, ua) <= (1e-6 if f32 else 1e-13)
    fv = FVMesh(m)
    ref = OP.project(fv, u, alpha, (0, 0, 0), 0.8, 0.004, 1.0)
    assert rel_err(host(b["b"]), ref["b"]) <= (2e-6 if f32 else 1e-12)
    assert rel_err(ub, ref["u_new"]) <= (1e-5 if f32 else 1e-7)


@pytest.mark.parametrize("precision", ["fp64", "mixed_f32fields"])
def test_body_cube_forcing_matches_full_forcing(precision):
    """16^3 cubes with the body in a few cubes only: the forcing kernel then stores u* only in
    those cubes and passes u~ on elsewhere (u* = u~ where alpha = 0).  With the face-velocity
    output every cube is forced and stored; the right-hand side and the pressure must be
    bit-identical, the cell velocities equal to the correction kernels' rounding."""
    m = uniform_mesh((4, 2, 2), 0.25, 16, CHANNEL_BC)
    rng = np.random.default_rng(9)
    u = uniform_random_velocity(m, 10, 0.3, (1.0, 0.0, 0.0))
    alpha = np.zeros((m.n_cubes, m.n ** 3))
    alpha[[3, 6]] = rng.uniform(0.0, 1.0, (2, m.n ** 3))   # two body cubes of 16
    alpha[9, :100] = 1.0                                   # one partly covered cube
    alpha = alpha.ravel()
    f32 = precision == "mixed_f32fields"
    if f32:
        u = u.astype(np.float32).astype(np.float64)
    plan = plan_for(m, precision)
    ft = plan.field_dtype
    args = ([dev(u[d], ft) for d in range(3)], dev(alpha, ft), 0.8, 0.004, 1.0)
    full = plan.project(*args, face_u=True, want_b=True)
    sel = plan.project(*args, face_u=False, want_b=True)
    assert np.array_equal(host(full["b"]), host(sel["b"]))
    assert np.array_equal(host(full["p"]), host(sel["p"]))
    uf = np.stack([host(x) for x in full["u_new"]])
    us = np.stack([host(x) for x in sel["u_new"]])
    assert rel_err(us, uf) <= (1e-6 if f32 else 1e-13)
    ref = OP.project(FVMesh(m), u, alpha, (0, 0, 0), 0.8, 0.004, 1.0)
    assert rel_err(us, ref["u_new"]) <= (1e-5 if f32 else 1e-7)


@pytest.mark.parametrize("precision", ["fp64", "mixed_f32fields"])
def test_recompute_matches_projection(precision):
    m, u, alpha = _case("multilevel_small_n4")
    plan = plan_for(m, precision)
    ft = plan.field_dtype
    args = ([dev(u[d], ft) for d in range(3)], dev(alpha, ft), 1.0, 0.01, 1.0)
    out = plan.project(*args)
    again = plan.project_recompute(args[0], args[1], out["p"], *args[2:])
    for d in range(3):
        assert np.array_equal(host(again[d]), host(out["u_new"][d]))


def test_sphere_channel_full_size_fp64():
    """The 1024-cube (4.2M cells) sphere channel, FP64, against the exact spectral oracle."""
    from oracle import UniformGrid
    pr = configs.sphere_channel()
    m = pr["mesh"]
    log(f"sphere_channel full: {m.n_cells} cells")
    plan = plan_for(m, "fp64")
    out = plan.project([dev(pr["u"][d]) for d in range(3)], dev(pr["alpha"]), pr["U_in"],
                       pr["dt"], pr["rho"])
    ug = UniformGrid(m)
    ref = ug.project(pr["u"], pr["alpha"], (0.0, 0.0, 0.0), pr["U_in"], pr["dt"], pr["rho"])
    p = host(out["p"])
    r = ref["b_global"] - ug.laplacian(ug.to_global(p))
    rr = np.linalg.norm(r) / np.linalg.norm(ref["b_global"])
    rep = out["report"]
    log(f"  its={rep.n_inner} reported={rep.final_rel_res:.2e} oracle={rr:.2e}")
    assert rep.status == 0 and rr <= 1.2e-10
    # ||p - p*|| <= ||r|| / lambda_min (closed form on one level)
    err = np.linalg.norm(ug.to_global(p) - ref["p_global"])
    assert err <= 1.01 * np.linalg.norm(r) / ug.lambda_min_abs()
    unew = np.stack([host(x) for x in out["u_new"]])
    assert rel_err(unew, ref["u_new"].reshape(3, -1)) <= 1e-7


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_mixed_channel_full_size(precision):
    """The 8192-cube (33.5M cells) channel of the benchmark, in the benchmark's launch
    configuration, against the exact spectral oracle: residual, the closed-form error bound,
    and the corrected velocity."""
    from oracle import UniformGrid
    pr = configs.mixed_channel()
    m = pr["mesh"]
    log(f"mixed_channel full {precision}: {m.n_cells} cells")
    plan = plan_for(m, precision)
    out = plan.project([dev(pr["u"][d]) for d in range(3)], dev(pr["alpha"]), pr["U_in"],
                       pr["dt"], pr["rho"])
    ug = UniformGrid(m)
    ref = ug.project(pr["u"], pr["alpha"], (0.0, 0.0, 0.0), pr["U_in"], pr["dt"], pr["rho"])
    p = host(out["p"])
    r = ref["b_global"] - ug.laplacian(ug.to_global(p))
    rr = np.linalg.norm(r) / np.linalg.norm(ref["b_global"])
    rep = out["report"]
    log(f"  its={rep.n_inner} outer={rep.n_outer} reported={rep.final_rel_res:.2e} "
        f"oracle={rr:.2e}")
    assert rep.status == 0 and rr <= 1.2e-10
    err = np.linalg.norm(ug.to_global(p) - ref["p_global"])
    assert err <= 1.01 * np.linalg.norm(r) / ug.lambda_min_abs()
    unew = np.stack([host(x) for x in out["u_new"]])
    assert rel_err(unew, ref["u_new"].reshape(3, -1)) <= 1e-7
