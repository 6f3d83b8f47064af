"""Building-cube projection path on MI355X: HIP kernels behind a C ABI (include/bcm.h).

    from paper_1808_04099_amd import Mesh, Plan
    plan = Plan(Mesh(mesh_desc), precision="mixed")
    out = plan.project(u, alpha, U_in, dt, rho)

The compiled library must exist (python -m paper_1808_04099_amd.build); there is no CPU
fallback.
"""
from .api import BCMError, Mesh, Plan, SolveReport, timing_names
from .autograd import KineticEnergy, MultiStepProjection, Projection, kinetic_energy

__all__ = ["BCMError", "Mesh", "Plan", "SolveReport", "timing_names", "Projection",
           "MultiStepProjection", "KineticEnergy", "kinetic_energy"]
