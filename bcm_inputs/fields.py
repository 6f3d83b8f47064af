"""Seeded synthetic fields: immersed-body volume fractions and velocity fields.

Inputs only (no arithmetic of the projection method).  Every array is cube-major [c][k][j][i];
velocity fields are component-major [3][c][k][j][i] (one scalar array per component).
"""
from __future__ import annotations

import numpy as np

from .mesh import Mesh


# ---------------------------------------------------------------------------------------------
# Immersed bodies.  A body classifies axis-aligned boxes (inside / outside / straddling) and gives
# the exact length of its intersection with a z-segment at a given (x, y).  The volume fraction of
# a straddling cell is the x-y midpoint-quadrature integral of that exact z-chord over the cell.
# ---------------------------------------------------------------------------------------------
IN, OUT, STRADDLE = 1, 0, 2


class Ellipsoid:
    def __init__(self, centre, semi_axes):
        self.c = np.asarray(centre, dtype=np.float64)
        self.a = np.asarray(semi_axes, dtype=np.float64)

    def classify(self, lo, hi):
        lo = (lo - self.c) / self.a
        hi = (hi - self.c) / self.a
        near = np.clip(0.0, lo, hi)
        far = np.maximum(np.abs(lo), np.abs(hi))
        dn = np.sum(near ** 2, axis=-1)
        df = np.sum(far ** 2, axis=-1)
        out = np.full(dn.shape, STRADDLE, dtype=np.int8)
        out[df <= 1.0] = IN
        out[dn >= 1.0] = OUT
        return out

    def z_interval(self, x, y):
        s = 1.0 - ((x - self.c[0]) / self.a[0]) ** 2 - ((y - self.c[1]) / self.a[1]) ** 2
        half = self.a[2] * np.sqrt(np.maximum(s, 0.0))
        valid = s > 0.0
        return self.c[2] - half, self.c[2] + half, valid


class Sphere(Ellipsoid):
    def __init__(self, centre, radius):
        super().__init__(centre, (radius, radius, radius))


class Box:
    def __init__(self, lo, hi):
        self.lo = np.asarray(lo, dtype=np.float64)
        self.hi = np.asarray(hi, dtype=np.float64)

    def classify(self, lo, hi):
        out = np.full(lo.shape[:-1], STRADDLE, dtype=np.int8)
        inside = np.all((lo >= self.lo) & (hi <= self.hi), axis=-1)
        outside = np.any((hi <= self.lo) | (lo >= self.hi), axis=-1)
        out[inside] = IN
        out[outside] = OUT
        return out

    def z_interval(self, x, y):
        valid = (x > self.lo[0]) & (x < self.hi[0]) & (y > self.lo[1]) & (y < self.hi[1])
        a = np.full(np.shape(x), self.lo[2])
        b = np.full(np.shape(x), self.hi[2])
        return a, b, valid


class Union:
    def __init__(self, *parts):
        self.parts = parts

    def classify(self, lo, hi):
        cls = [p.classify(lo, hi) for p in self.parts]
        out = np.full(cls[0].shape, STRADDLE, dtype=np.int8)
        out[np.all(np.stack(cls) == OUT, axis=0)] = OUT
        out[np.any(np.stack(cls) == IN, axis=0)] = IN
        return out

    def z_chord(self, x, y, z0, z1):
        segs = []
        for p in self.parts:
            a, b, v = p.z_interval(x, y)
            a = np.clip(a, z0, z1)
            b = np.clip(b, z0, z1)
            segs.append((np.where(v, a, z0), np.where(v, np.maximum(b, a), z0)))
        # union length of the clipped intervals (at most a handful of parts)
        total = np.zeros(np.shape(x))
        for i, (a, b) in enumerate(segs):
            total += b - a
            for a2, b2 in segs[:i]:
                total -= np.maximum(0.0, np.minimum(b, b2) - np.maximum(a, a2))
        return total


def _as_union(body):
    return body if isinstance(body, Union) else Union(body)


def volume_fraction(mesh: Mesh, body, quad: int = 32, chunk: int = 4096,
                    cube_chunk: int = 512) -> np.ndarray:
    """Per-cell solid volume fraction alpha in [0, 1] (float64 [n_c, n, n, n]).

    Cells wholly inside/outside the body get exactly 1/0.  A straddling cell gets the mean, over
    a quad x quad midpoint grid in x-y, of the exact z-chord length through the body divided by h.
    Cubes are classified first so that only cubes touching the body are visited cell by cell.
    """
    body = _as_union(body)
    n = mesh.n
    alpha = np.zeros((mesh.n_cubes, n ** 3))
    edge = mesh.edge()
    ccls = body.classify(mesh.origin, mesh.origin + edge[:, None])
    alpha[ccls == IN] = 1.0
    todo = np.nonzero(ccls == STRADDLE)[0]
    s = (np.arange(quad) + 0.5) / quad
    g = np.arange(n, dtype=np.float64)
    for c0 in range(0, todo.size, cube_chunk):
        cubes = todo[c0:c0 + cube_chunk]
        h = mesh.h()[cubes][:, None, None, None]
        o = mesh.origin[cubes]
        lo = np.stack(np.broadcast_arrays(o[:, 0, None, None, None] + g[None, None, None, :] * h,
                                          o[:, 1, None, None, None] + g[None, None, :, None] * h,
                                          o[:, 2, None, None, None] + g[None, :, None, None] * h),
                      axis=-1).reshape(-1, 3)
        hf = np.broadcast_to(h, (cubes.size, n, n, n)).reshape(-1)
        cls = body.classify(lo, lo + hf[:, None])
        a = np.zeros(lo.shape[0])
        a[cls == IN] = 1.0
        idx = np.nonzero(cls == STRADDLE)[0]
        for start in range(0, idx.size, chunk):
            sel = idx[start:start + chunk]
            l = lo[sel]
            hh = hf[sel][:, None, None]
            x = l[:, 0, None, None] + s[None, :, None] * hh
            y = l[:, 1, None, None] + s[None, None, :] * hh
            x, y = np.broadcast_arrays(x, y)
            z0 = np.broadcast_to(l[:, 2, None, None], x.shape)
            ch = body.z_chord(x, y, z0, z0 + hh)
            a[sel] = ch.mean(axis=(1, 2)) / hf[sel]
        alpha[cubes] = a.reshape(cubes.size, n ** 3)
    return alpha.reshape(mesh.n_cubes, n, n, n)


# ---------------------------------------------------------------------------------------------
# Velocity fields
# ---------------------------------------------------------------------------------------------
def uniform_random_velocity(mesh: Mesh, seed: int, amp: float = 1.0, base=(0.0, 0.0, 0.0)):
    """base + amp * U[-1, 1] per cell and component, drawn in [3][c][k][j][i] order."""
    rng = np.random.default_rng(seed)
    n = mesh.n
    u = rng.uniform(-1.0, 1.0, size=(3, mesh.n_cubes, n, n, n)) * amp
    for d in range(3):
        u[d] += base[d]
    return u


def fourier_modes(seed: int, n_modes: int = 32, kmax: int = 8):
    """Mode table (k [m,3] int, a [m], phi [m]) for a smooth random field."""
    rng = np.random.default_rng(seed)
    k = rng.integers(1, kmax + 1, size=(n_modes, 3))
    a = rng.standard_normal(n_modes) / np.sum(k.astype(np.float64) ** 2, axis=1)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)
    return k, a, phi


def fourier_field(mesh: Mesh, seed: int, n_modes: int = 32, kmax: int = 8, length=None):
    """sum_m a_m cos(2 pi (k1 x/Lx + k2 y/Ly + k3 z/Lz) + phi_m) at cell centres (float64)."""
    k, a, phi = fourier_modes(seed, n_modes, kmax)
    L = np.asarray(length if length is not None else
                   np.subtract(mesh.domain_hi, mesh.domain_lo), dtype=np.float64)
    if np.all(mesh.level == mesh.level[0]):
        return _fourier_field_uniform(mesh, k, a, phi, L)
    X, Y, Z = mesh.cell_centres()
    out = np.zeros_like(X)
    for m in range(n_modes):
        out += a[m] * np.cos(2.0 * np.pi * (k[m, 0] * X / L[0] + k[m, 1] * Y / L[1]
                                            + k[m, 2] * Z / L[2]) + phi[m])
    return out


def _fourier_field_uniform(mesh: Mesh, k, a, phi, L):
    """Same sum on a single-level mesh, evaluated separably on the global grid:
    sum_m a_m Re(e^{i phi_m} e^{i kx x} e^{i ky y} e^{i kz z}) as one (x,y) x m x z product."""
    n = mesh.n
    h = float(mesh.h()[0])
    lo = np.asarray(mesh.domain_lo, dtype=np.float64)
    cijk = np.rint((mesh.origin - lo) / (h * n)).astype(np.int64)
    dims = cijk.max(axis=0) + 1
    N = dims * n
    xs = [lo[d] + (np.arange(N[d]) + 0.5) * h for d in range(3)]
    ex = np.exp(1j * 2.0 * np.pi * np.outer(k[:, 0], xs[0]) / L[0]) * (a * np.exp(1j * phi))[:, None]
    ey = np.exp(1j * 2.0 * np.pi * np.outer(k[:, 1], xs[1]) / L[1])
    ez = np.exp(1j * 2.0 * np.pi * np.outer(k[:, 2], xs[2]) / L[2])
    # M[(y, x), m] = ey[m, y] ex[m, x];  G[z, y, x] = Re(sum_m ez[m, z] M[(y, x), m])
    M = (ey[:, :, None] * ex[:, None, :]).reshape(ex.shape[0], -1)       # [m, y*x]
    G = (ez.T @ M).real.reshape(N[2], N[1], N[0])
    out = np.empty((mesh.n_cubes, n, n, n))
    for c in range(mesh.n_cubes):
        x, y, z = cijk[c]
        out[c] = G[z * n:(z + 1) * n, y * n:(y + 1) * n, x * n:(x + 1) * n]
    return out


# ---------------------------------------------------------------------------------------------
# Surface particles of an immersed body (the paper's Lagrangian points: about one per Eulerian
# cell that the surface crosses).
# ---------------------------------------------------------------------------------------------
def sphere_particles(centre, radius, spacing):
    """Points on a sphere on a Fibonacci lattice with about one point per spacing^2 of surface,
    and the Lagrangian volume of each (its surface share times the spacing): (X [n, 3], dV [n])."""
    area = 4.0 * np.pi * radius ** 2
    n = max(1, int(round(area / spacing ** 2)))
    k = np.arange(n, dtype=np.float64) + 0.5
    z = 1.0 - 2.0 * k / n
    r = np.sqrt(np.maximum(1.0 - z * z, 0.0))
    ang = np.pi * (3.0 - np.sqrt(5.0)) * k
    X = np.asarray(centre, dtype=np.float64)[None, :] + radius * np.stack(
        [r * np.cos(ang), r * np.sin(ang), z], axis=1)
    dV = np.full(n, area / n * spacing)
    return X, dV
