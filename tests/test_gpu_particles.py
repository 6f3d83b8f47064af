"""GPU parity of the Lagrangian-particle forcing (bcm_ib_force) against the oracle
(oracle/lagrangian.py): interpolated velocities, constraint forces and the forced field u*,
element by element, on a uniform channel (FP64 and FP32 fields) and inside the finest level of
the three-level mesh; particles outside the mesh or with a support that leaves the level or
the domain are skipped and reported; and one whole fractional step on the 16x8x8-cube sphere
channel with about 4.6k particles on the sphere surface (forcing, Poisson solve, correction)
against the oracle's forcing followed by its exact spectral projection.
The GPU spread adds with atomics (no fixed order), so the forced field agrees to rounding."""
import numpy as np
import pytest
import torch

from bcm_inputs import CHANNEL_BC, configs, sphere_particles, uniform_mesh, uniform_random_velocity
from oracle import UniformGrid
from oracle.lagrangian import ParticleOperator

from gpu_util import dev, host, log, plan_for, rel_err, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]


def _box_particles(n_p, seed, box):
    rng = np.random.default_rng(seed)
    lo, hi = np.array(box[0]), np.array(box[1])
    return lo + (hi - lo) * rng.uniform(size=(n_p, 3))


CASES = {
    "channel": (lambda: uniform_mesh((4, 2, 2), 0.25, 8, CHANNEL_BC),
                lambda m: sphere_particles((0.5, 0.25, 0.25), 0.12, float(m.h()[0]))),
    "three_level": (lambda: configs.multilevel_small()["mesh"],
                    lambda m: (_box_particles(150, 7, ((0.62, 0.47, 0.47), (0.78, 0.53, 0.53))),
                               None)),
}


@pytest.mark.parametrize("precision", ["fp64", "mixed_f32fields"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_particle_forcing_matches_oracle(name, precision):
    make, parts = CASES[name]
    m = make()
    X, dV = parts(m)
    f32 = precision == "mixed_f32fields"
    u = uniform_random_velocity(m, 95, 0.5, (1.0, 0.0, 0.0)).reshape(3, -1)
    if f32:
        u = u.astype(np.float32).astype(np.float64)
    op = ParticleOperator(m, X)
    h3 = op.h_cell[op.W.indices[op.W.indptr[:-1]]] ** 3      # h^3 at each particle's cells
    dV_ref = dV if dV is not None else h3
    Us = np.array([0.1, -0.05, 0.0])
    dt, rho = 0.01, 1.2
    us_ref, U_ref, F_ref = op.force(u, Us, dV_ref, dt, rho)
    plan = plan_for(m, precision)
    out = plan.ib_force([dev(u[d], plan.field_dtype) for d in range(3)], dev(X), dt, rho,
                        dV=dev(dV) if dV is not None else None, Us=tuple(Us), want_UF=True)
    us = np.stack([host(x) for x in out["u_star"]])
    eU, eF = rel_err(host(out["U_p"]), U_ref), rel_err(host(out["F_p"]), F_ref)
    du = np.abs(us - us_ref).max() / np.abs(us_ref - u).max()   # relative to the forcing
    log(f"  {name} {precision}: {len(X)} particles; U_p {eU:.2e} F_p {eF:.2e} u* {du:.2e}")
    tol = 2e-6 if f32 else 1e-12
    assert eU <= tol and eF <= (2e-5 if f32 else 1e-12) and du <= (1e-5 if f32 else 1e-12)


def test_particles_off_the_mesh_or_level_are_skipped_and_reported():
    from paper_1808_04099_amd import BCMError
    m = uniform_mesh((4, 2, 2), 0.25, 8, CHANNEL_BC)
    X = np.array([[0.5, 0.25, 0.25],      # fine
                  [1.5, 0.25, 0.25],      # outside the mesh
                  [0.01, 0.25, 0.25],     # support crosses the inflow wall
                  [0.5, 0.49, 0.25]])     # support crosses a slip wall
    plan = plan_for(m, "fp64")
    u = [torch.zeros(m.n_cells, dtype=torch.float64, device="cuda") for _ in range(3)]
    with pytest.raises(BCMError) as e:
        plan.ib_force(u, dev(X).reshape(-1, 3), 0.01, 1.0, Us=(1.0, 0.0, 0.0))
    assert e.value.status == -1 and "3 particles skipped" in str(e.value)
    # the valid particle's forcing is applied: one particle, u~ = 0, U_s = (1, 0, 0)
    out_ok = plan.ib_force(u, dev(X[:1]).reshape(-1, 3), 0.01, 1.0, Us=(1.0, 0.0, 0.0))
    tot = float(out_ok["u_star"][0].sum()) * float(m.h()[0]) ** 3
    assert abs(tot - float(m.h()[0]) ** 3) <= 1e-14     # spread conserves dV (U_s - U_p)


def test_fractional_step_with_particles_sphere_channel():
    """16x8x8 cubes of 16^3 (4.2M cells): Lagrangian forcing of the sphere (one particle per
    h^2 of surface), then the projection without a volume fraction, against the oracle."""
    pr = configs.sphere_channel()
    m = pr["mesh"]
    h = float(m.h()[0])
    X, dV = sphere_particles((0.5, 0.5, 0.5), 0.15, h)
    u = pr["u"].reshape(3, -1)
    log(f"fractional step with particles: {m.n_cells} cells, {len(X)} particles")
    plan = plan_for(m, "fp64")
    fo = plan.ib_force([dev(u[d]) for d in range(3)], dev(X), pr["dt"], pr["rho"], dV=dev(dV))
    out = plan.project(fo["u_star"], None, pr["U_in"], pr["dt"], pr["rho"])
    rep = out["report"]
    assert rep.status == 0
    op = ParticleOperator(m, X)
    us_ref, _, _ = op.force(u, (0.0, 0.0, 0.0), dV, pr["dt"], pr["rho"])
    ref = UniformGrid(m).project(us_ref.reshape(3, m.n_cubes, m.n, m.n, m.n),
                                 np.zeros((m.n_cubes, m.n, m.n, m.n)), (0.0, 0.0, 0.0),
                                 pr["U_in"], pr["dt"], pr["rho"])
    e_us = rel_err(np.stack([host(x) for x in fo["u_star"]]), us_ref)
    e_u = rel_err(np.stack([host(x) for x in out["u_new"]]), ref["u_new"].reshape(3, -1))
    e_p = rel_err(host(out["p"]), ref["p"].ravel())
    log(f"  projection {rep.n_inner} its {rep.final_rel_res:.1e}; u* {e_us:.2e}, "
        f"u^(n+1) {e_u:.2e}, p {e_p:.2e}")
    assert e_us <= 1e-13 and e_u <= 1e-7 and e_p <= 1e-7
