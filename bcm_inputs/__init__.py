"""Seeded synthetic inputs (meshes and fields) used by both the oracle and the GPU path.

Nothing here computes any step of the projection method; see mesh.py for the array conventions.
"""
from .mesh import (BC_INFLOW, BC_NONE, BC_OUTFLOW, BC_SLIP, CHANNEL_BC, OPEN_BC, Mesh,
                   build_mesh, morton3, uniform_mesh)
from .fields import (Box, Ellipsoid, Sphere, Union, fourier_field, sphere_particles,
                     uniform_random_velocity, volume_fraction)
from . import configs
