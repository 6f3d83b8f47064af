"""Plain, slow FP64 CPU oracle of the building-cube projection path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package; the product path (the HIP library and its Python binding)
never does, and shares no code with it.

  fv.py          finite-volume operators assembled as sparse matrices from the mesh geometry
                 (any number of levels, 2:1 interfaces), exact sparse-LU solves
  uniform.py     the same operators on one global array for single-level meshes, exact
                 spectral (DST/DCT) Poisson solve
  projection.py  forcing -> Poisson -> correction step, its exact transpose, the multi-step
                 kinetic-energy objective, its gradient and a complex-step directional derivative
  sample.py      stencil rows evaluated at individually chosen cells (for meshes too large to
                 assemble)
  momentum.py    the momentum sub-step (QUICK convection, diffusion; Euler, AB2, Crank-Nicolson)
                 on single-level meshes, array form with two-layer ghost cells
  lagrangian.py  the Lagrangian-particle forcing: 3-point discrete delta interpolation, constraint
                 force and spreading, as an assembled particle x cell weight matrix
  codec.py       per-cube lossy wavelet compression of checkpoints (CDF 5/3 lifting, uniform
                 quantisation, adaptive bit packing) and its byte stream
  composite.py   the Laplacian, divergence and residual norm of any mesh as whole-array
                 expressions over the cube-major fields (full-size residuals of the 3-level mesh)

Parity status of each function is stated in its module; everything here is pinned by the
`-m "not gpu"` tests (closed forms, identities, brute force, two independent formulations).
"""
from .fv import FVMesh
from .uniform import UniformGrid
from . import projection
