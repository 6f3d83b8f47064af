"""Lagrangian-particle immersed-boundary forcing (FP64): interpolation, constraint force and
spreading with the 3-point smoothed discrete delta function.

TEST INFRASTRUCTURE ONLY: the product path never imports this package.

Sec. 2.3-2.4 and the forcing sub-step of Sec. 3:
  interpolation (Eq. (ddeltai))  U_p = sum_i u_i delta_h(x_i - X_p) h_i^3
  constraint force (Sec. 3)      F_p = (rho/dt) (U_s,p - U_p)
  spreading (Eq. (ddeltap))      f_i = sum_p F_p delta_h(x_i - X_p) dV_p
  forcing sub-step (Sec. 3)      u* = u~ + (dt/rho) f
with delta_h(x) = prod_n phi(x_n / h) / h (h = the cell width of cell i) and the 3-point
function phi(r) = 3/4 - r^2 (|r| <= 1/2), (9/4 - 3|r| + r^2)/2 (1/2 < |r| <= 3/2), 0 beyond.
dV_p is the particle's Lagrangian volume (the paper's dc_1 dc_2 dc_3).
Readings (the paper does not spell them out):
  l1  the sums run over every cell of the mesh; a particle's support is the 3 x 3 x 3 cells
      around the cell centre nearest to it, all of one level (bodies sit in the finest cubes),
      and the support must stay inside the domain (no mirrored weights at walls);
  l2  the interpolation and the spreading use the same weights, so spreading is the
      transpose of interpolation in the volume-weighted inner products.
Implemented by assembling the interpolation matrix W (particles x cells, entries
prod_n phi((x_i,n - X_p,n)/h)) from the cell geometry: the definition written out.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def phi(r):
    """The 3-point smoothed one-dimensional discrete delta function (Sec. 2.4)."""
    a = np.abs(np.asarray(r, dtype=np.float64))
    out = np.where(a <= 0.5, 0.75 - a * a, 0.5 * (2.25 - 3.0 * a + a * a))
    return np.where(a <= 1.5, out, 0.0)


class ParticleOperator:
    """Interpolation / spreading between the cells of a mesh and a set of particles."""

    def __init__(self, mesh, X):
        self.mesh = mesh
        n = mesh.n
        X = np.asarray(X, dtype=np.float64).reshape(-1, 3)
        self.X = X
        h_cube = mesh.root_edge / 2.0 ** mesh.level.astype(np.float64) / n
        self.h_cell = np.repeat(h_cube, n ** 3)
        lo = np.asarray(mesh.domain_lo, dtype=np.float64)
        # every cell by (level, global integer cell index on its level's lattice)
        edge = h_cube * n
        cijk = np.rint((mesh.origin - lo) / edge[:, None]).astype(np.int64)
        lookup = {}
        for c in range(mesh.n_cubes):
            lookup[(int(mesh.level[c]), *map(int, cijk[c]))] = c
        self._lookup = lookup
        self._levels = sorted(set(int(v) for v in mesh.level), reverse=True)
        rows, cols, vals = [], [], []
        self.cell_of = np.empty(len(X), dtype=np.int64)
        for p, x in enumerate(X):
            found = None
            for L in self._levels:                     # finest level first
                e = mesh.root_edge / 2.0 ** L
                q = np.floor((x - lo) / e).astype(np.int64)
                c = lookup.get((L, *map(int, q)))
                if c is not None:
                    found = (L, c)
                    break
            assert found is not None, f"particle {p} lies outside the mesh"
            L, c = found
            h = mesh.root_edge / 2.0 ** L / n
            i0 = np.floor((x - lo) / h).astype(np.int64)    # the cell holding X: nearest centre
            for dz in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        cell = i0 + np.array([dx, dy, dz])
                        cube = lookup.get((L, *map(int, cell // n)))
                        assert cube is not None, f"support of particle {p} leaves its level"
                        loc = cell - (cell // n) * n
                        idx = cube * n ** 3 + (loc[2] * n + loc[1]) * n + loc[0]
                        centre = lo + (cell + 0.5) * h
                        w = float(np.prod(phi((centre - x) / h)))
                        rows.append(p)
                        cols.append(idx)
                        vals.append(w)
            self.cell_of[p] = c
        self.W = sp.csr_matrix((vals, (rows, cols)), shape=(len(X), mesh.n_cells))

    def interpolate(self, u):
        """U_p (particles x 3) of the cell velocity u [3, n_cells]."""
        u = np.asarray(u).reshape(3, -1)
        return np.stack([self.W @ u[d] for d in range(3)], axis=1)

    def spread(self, F, dV):
        """f (3 x n_cells) of the particle forces F (particles x 3) with volumes dV."""
        F = np.asarray(F).reshape(-1, 3)
        g = F * np.asarray(dV, dtype=np.float64).reshape(-1, 1)
        return np.stack([(self.W.T @ g[:, d]) / self.h_cell ** 3 for d in range(3)])

    def force(self, u_tilde, Us, dV, dt, rho):
        """The forcing sub-step: returns (u*, U_p, F_p)."""
        U = self.interpolate(u_tilde)
        F = (rho / dt) * (np.broadcast_to(np.asarray(Us, dtype=np.float64), U.shape) - U)
        u_star = np.asarray(u_tilde).reshape(3, -1) + (dt / rho) * self.spread(F, dV)
        return u_star, U, F
