"""GPU parity of the Poisson operator and solve (FP64 and mixed) against the FP64 oracle.

Tolerances: the FP64 operator apply is one stencil evaluation, compared to 1e-12 of the
largest value.  Solves run to a V-weighted relative residual of 1e-10 (the workload target);
the oracle re-evaluates the residual of the returned pressure in FP64 (<= 1.2e-10, the slack
covering the different summation order), and the error against the exact discrete solution
is bounded by ||e|| <= ||r|| / lambda_min(-A) with lambda_min in closed form on one level.
"""
import numpy as np
import pytest

from bcm_inputs import CHANNEL_BC, OPEN_BC, configs, uniform_mesh
from oracle import FVMesh, UniformGrid

from gpu_util import dev, host, log, plan_for, rel_err, requires_gpu
from test_oracle_operators import _tiny_multilevel

pytestmark = [pytest.mark.gpu, requires_gpu]


def _meshes():
    return {
        "channel_n4": uniform_mesh((3, 2, 2), 0.25, 4, CHANNEL_BC),
        "open_n8": uniform_mesh((2, 2, 2), 0.5, 8, OPEN_BC),
        "channel_n16": uniform_mesh((4, 2, 2), 0.25, 16, CHANNEL_BC),
        "tiny_3level_n2": _tiny_multilevel(),
        "multilevel_small_n4": configs.multilevel_small()["mesh"],
    }


@pytest.mark.parametrize("name", sorted(_meshes()))
def test_laplacian_apply_matches_oracle(name):
    m = _meshes()[name]
    log(f"laplacian {name}: {m.n_cubes} cubes n={m.n}")
    fv = FVMesh(m)
    p = np.random.default_rng(5).standard_normal(m.n_cells)
    plan = plan_for(m)
    ap = host(plan.apply_laplacian(dev(p)))
    ref = fv.A @ p
    assert rel_err(ap, ref) <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_manufactured_solution_small_box(precision):
    """4x4x4 cubes of 16^3, open box: p_h = (-14 pi^2 / lambda_h) sin sin sin exactly."""
    pr = configs.small_box()
    m = pr["mesh"]
    log(f"manufactured {precision}")
    plan = plan_for(m, precision)
    p, rep = plan.poisson_solve(dev(pr["b"]))
    p = host(p)
    fv = FVMesh(m)
    rr = fv.residual_norm(p, pr["b"].ravel())
    log(f"  iters={rep.n_inner} outer={rep.n_outer} reported={rep.final_rel_res:.3e} "
        f"oracle={rr:.3e}")
    assert rep.status == 0 and rep.final_rel_res <= 1e-10
    assert rr <= 1.2e-10
    h = 1.0 / 64
    lam_h = sum(2 * np.cos(k * np.pi * h) - 2 for k in (1, 2, 3)) / h ** 2
    X, Y, Z = m.cell_centres()
    ph = (-14 * np.pi ** 2 / lam_h) * (np.sin(np.pi * X) * np.sin(2 * np.pi * Y)
                                        * np.sin(3 * np.pi * Z)).ravel()
    ug = UniformGrid(m)
    bound = rr * np.linalg.norm(pr["b"]) / ug.lambda_min_abs()
    assert np.linalg.norm(p - ph) <= 1.01 * bound


@pytest.mark.parametrize("name", ["channel_n4", "open_n8", "tiny_3level_n2",
                                  "multilevel_small_n4"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_poisson_matches_oracle(name, precision):
    m = _meshes()[name]
    log(f"poisson {name} {precision}")
    fv = FVMesh(m)
    b = np.random.default_rng(9).standard_normal(m.n_cells)
    plan = plan_for(m, precision)
    p, rep = plan.poisson_solve(dev(b))
    p = host(p)
    rr = fv.residual_norm(p, b)
    log(f"  iters={rep.n_inner} outer={rep.n_outer} reported={rep.final_rel_res:.3e} "
        f"oracle={rr:.3e}")
    assert rep.status == 0
    assert rr <= 1.2e-10
    ref = fv.solve(b)
    # ||e||_V <= ||r||_V / lambda_min of the V-symmetric operator; checked loosely via the
    # residual and directly against the exact solve
    assert rel_err(p, ref) <= 1e-7


@pytest.mark.parametrize("name", ["channel_n4", "multilevel_small_n4", "tiny_3level_n2"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_split_graph_multigrid_matches_oracle(name, precision):
    """graph_split = 0 smooths every cube-graph level but the last with the multi-workgroup
    kernels (the path large multi-level meshes take by default)."""
    m = _meshes()[name]
    log(f"split graph {name} {precision}")
    fv = FVMesh(m)
    b = np.random.default_rng(19).standard_normal(m.n_cells)
    p, rep = plan_for(m, precision, graph_split=0).poisson_solve(dev(b))
    p = host(p)
    rr = fv.residual_norm(p, b)
    log(f"  iters={rep.n_inner} outer={rep.n_outer} oracle={rr:.3e}")
    assert rep.status == 0 and rr <= 1.2e-10
    assert rel_err(p, fv.solve(b)) <= 1e-7


@pytest.mark.parametrize("name", ["channel_n16", "multilevel_small_n4"])
@pytest.mark.parametrize("opts", [dict(coarse_solver=0, max_iter=200), dict(krylov=0, max_iter=200),
                                  dict(coarse_cycles=2), dict(pre_sweeps=1, post_sweeps=3),
                                  dict(pre_sweeps=0, post_sweeps=2, max_iter=200),
                                  dict(pre_sweeps=3, post_sweeps=1),
                                  dict(prolong=0), dict(krylov=2), dict(check_every=3)],
                         ids=["paper_cg", "vcycle_iteration", "two_graph_cycles", "sweeps_1_3",
                              "sweeps_0_2", "sweeps_3_1",
                              "constant_prolongation", "standard_pcg", "checks_every_3"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solver_variants_match_oracle(name, opts, precision):
    """The paper's scheme (CG capped at coarse_iters on the one-cell-per-cube level, plain
    V-cycle iteration) and other option settings reach the same solution."""
    m = _meshes()[name]
    log(f"variant {name} {opts} {precision}")
    fv = FVMesh(m)
    b = np.random.default_rng(23).standard_normal(m.n_cells)
    p, rep = plan_for(m, precision, **opts).poisson_solve(dev(b))
    p = host(p)
    rr = fv.residual_norm(p, b)
    log(f"  iters={rep.n_inner} outer={rep.n_outer} oracle={rr:.3e}")
    assert rep.status == 0 and rr <= 1.2e-10
    assert rel_err(p, fv.solve(b)) <= 1e-7


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_check_every_reads_back_less_often(precision):
    """check_every = 3 tests convergence every third Krylov iteration: the solve still reaches
    the tolerance, with fewer history entries (one per check) than checking every iteration,
    and every inner solve ends on a check."""
    m = _meshes()["channel_n16"]
    fv = FVMesh(m)
    b = np.random.default_rng(37).standard_normal(m.n_cells)
    p1, r1 = plan_for(m, precision).poisson_solve(dev(b))
    p3, r3 = plan_for(m, precision, check_every=3).poisson_solve(dev(b))
    log(f"check_every 1: {r1.n_inner} its, {len(r1.history)} entries; "
        f"3: {r3.n_inner} its, {len(r3.history)} entries ({precision})")
    assert r1.status == 0 and r3.status == 0
    assert fv.residual_norm(host(p3), b) <= 1.2e-10
    assert len(r3.history) < len(r1.history)
    # one entry per outer residual plus one per check (ceil(inner iterations / 3) per solve)
    assert len(r3.history) <= r3.n_outer + 1 + (r3.n_inner + 2 * (r3.n_outer + 1)) // 3
    assert rel_err(host(p3), fv.solve(b)) <= 1e-7


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_trilinear_prolongation_needs_fewer_iterations(precision):
    """On a single-level channel of 16^3 cubes the trilinear prolongation (default) reaches the
    tolerance in fewer Krylov iterations than the piecewise-constant one, at the same solution."""
    m = uniform_mesh((8, 4, 4), 0.125, 16, CHANNEL_BC)
    b = np.random.default_rng(31).standard_normal(m.n_cells)
    its, sols = {}, {}
    for pro in (0, 1):
        p, rep = plan_for(m, precision, prolong=pro).poisson_solve(dev(b))
        assert rep.status == 0
        its[pro], sols[pro] = rep.n_inner, host(p)
    log(f"trilinear {its[1]} vs constant {its[0]} iterations ({precision})")
    assert its[1] < its[0]
    assert rel_err(sols[1], sols[0]) <= 1e-6
