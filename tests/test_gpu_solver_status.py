"""Solver limits and failure detection on the GPU.

Every return path of the Poisson solve reports the true FP64 relative residual of the pressure
it returns; the oracle's residual of that pressure (assembled operator, FP64) must agree with
final_rel_res.  Cases:
  * max_iter = 1 (FP64 and mixed): BCM_NOT_CONVERGED with a filled history;
  * max_outer = 1: FP64 converges in its single Krylov pass (BCM_OK); mixed stops after one
    refinement step (BCM_NOT_CONVERGED, residual about inner_tol);
  * a tolerance below what FP64 can resolve: BCM_STAGNATED long before the iteration limits,
    with the residual at the FP64 floor.
"""
import numpy as np
import pytest

from bcm_inputs import CHANNEL_BC, uniform_mesh
from bcm_inputs.fields import fourier_field
from oracle import FVMesh

from gpu_util import dev, host, log, plan_for, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

OK, NOT_CONVERGED, STAGNATED = 0, 1, 2


def _problem():
    m = uniform_mesh((4, 2, 2), 0.25, 8, CHANNEL_BC)
    b = fourier_field(m, 41).ravel()
    return m, b


def _solve(m, b, precision, **opts):
    from paper_1808_04099_amd.api import BCMError
    plan = plan_for(m, precision, **opts)
    try:
        p, rep = plan.poisson_solve(dev(b))
    except BCMError as e:   # warnings are returned, errors raise
        raise AssertionError(str(e))
    return host(p), rep


def _check_report(m, b, p, rep):
    """final_rel_res and the last history entry against the oracle's residual of the returned
    pressure; 5e-15 of slack covers the rounding of A p (near the FP64 floor the residual is
    made of that rounding)."""
    fv = FVMesh(m)
    res = fv.residual_norm(p, b)
    log(f"  status={rep.status} its={rep.n_inner} outer={rep.n_outer} "
        f"final={rep.final_rel_res:.3e} oracle={res:.3e} history={len(rep.history)}")
    assert abs(rep.final_rel_res - res) <= 1e-6 * res + 5e-15
    assert rep.history and rep.history[-1] == rep.final_rel_res


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_max_iter_one_is_not_converged(precision):
    m, b = _problem()
    log(f"max_iter=1 {precision}")
    p, rep = _solve(m, b, precision, max_iter=1, max_outer=2)
    assert rep.status == NOT_CONVERGED
    assert rep.final_rel_res > 1e-10
    assert len(rep.history) >= 2
    _check_report(m, b, p, rep)


def test_max_outer_one_fp64_converges():
    m, b = _problem()
    log("max_outer=1 fp64")
    p, rep = _solve(m, b, "fp64", max_outer=1)
    assert rep.status == OK and rep.final_rel_res <= 1e-10
    _check_report(m, b, p, rep)


def test_max_outer_one_mixed_reports_its_residual():
    m, b = _problem()
    log("max_outer=1 mixed")
    p, rep = _solve(m, b, "mixed", max_outer=1)
    assert rep.status == NOT_CONVERGED
    assert 1e-8 < rep.final_rel_res < 1e-2
    _check_report(m, b, p, rep)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_unreachable_tolerance_stagnates(precision):
    m, b = _problem()
    log(f"tol=1e-18 {precision}")
    p, rep = _solve(m, b, precision, tol=1e-18, max_iter=200, max_outer=40)
    assert rep.status == STAGNATED
    assert rep.n_inner < 100 and rep.n_outer < 20
    assert rep.final_rel_res <= 1e-13
    _check_report(m, b, p, rep)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sampled_kernel_timing(precision):
    """bcm_timing_sample(every): one launch in each run of `every` is timed.  The operator apply
    runs once per Krylov iteration, so ceil(n_inner / every) of its launches carry events."""
    m, b = _problem()
    plan = plan_for(m, precision, tol=1e-10)
    for every in (1, 3):
        plan.timing_enable("apply8", every)
        p, rep = plan.poisson_solve(dev(b))
        n, ms = plan.timing_read()
        plan.timing_enable(None)
        log(f"  {precision}: every {every}: {n} timed of {rep.n_inner} launches, {ms:.3f} ms")
        assert rep.status == OK
        assert n == -(-rep.n_inner // every) and ms > 0.0


def test_r_update_rides_in_the_next_first_presmoother():
    """The r update of each Krylov iteration is applied by the first pre-smoother of the next
    V-cycle (timer class preupd8), after which the convergence check runs.  Where the last
    reduction factor predicts convergence at that check, a probe (rprobe) computes the check's
    <r, r> first without writing r, and the fused launch follows only if the solve goes on (it
    then skips the check).  So every iteration is checked once, there is no separate r update,
    and the plain pre-smoother runs only in the first V-cycle.  After the last allowed
    iteration the probe does the final check."""
    m, b = _problem()
    plan = plan_for(m, "fp64", tol=1e-10)
    counts = {}
    for cls in ("preupd8", "rprobe", "update", "presmooth8"):
        plan.timing_enable(cls)
        p, rep = plan.poisson_solve(dev(b))
        counts[cls] = plan.timing_read()[0]
        plan.timing_enable(None)
        assert rep.status == OK
    log(f"  converged: {counts}, n_inner {rep.n_inner}")
    assert counts["update"] == 0 and counts["presmooth8"] == 1 and counts["rprobe"] >= 1
    assert rep.n_inner in (counts["preupd8"], counts["preupd8"] + 1)
    _check_report(m, b, host(p), rep)
    plan = plan_for(m, "fp64", max_iter=3, max_outer=1)
    for cls in ("rprobe", "update"):
        plan.timing_enable(cls)
        p, rep = plan.poisson_solve(dev(b))
        counts[cls] = plan.timing_read()[0]
        plan.timing_enable(None)
    log(f"  max_iter 3: status {rep.status}, {counts['rprobe']} probe(s), {counts['update']} update(s)")
    assert rep.status == NOT_CONVERGED and rep.n_inner == 3
    assert counts["rprobe"] == 1 and counts["update"] == 0
    _check_report(m, b, host(p), rep)
