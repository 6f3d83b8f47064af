"""Finite-volume operators evaluated cell by cell, for meshes too large to assemble.

TEST INFRASTRUCTURE ONLY: the product path never imports this package.

Same definitions as fv.py (cell-centred finite volumes, Sec. 2.2 and Sec. 3), written per
cell: the sub-faces of each side of a cell are found from the geometry (a lookup of cubes by
level and integer position), with
  same-level neighbour: one sub-face, area h^2, distance h, interpolation (1/2, 1/2);
  coarser neighbour:    one sub-face, area h^2, distance 3h/2, weights (2/3 own, 1/3 other);
  finer neighbours:     four sub-faces, area (h/2)^2, distance 3h/4, weights (1/3 own, 2/3);
  domain boundary:      open: p = 0 at distance h/2, U = u_cell; inflow: U = U_in, no flux of
                        p; slip: U = 0, no flux of p.
parity: pinned against fv.FVMesh on small meshes (tests/test_oracle_sample.py).
"""
from __future__ import annotations

import numpy as np

OUTFLOW, INFLOW, SLIP = 1, 2, 3


class CellSampler:
    def __init__(self, mesh):
        self.m = mesh
        self.n = mesh.n
        lo = np.asarray(mesh.domain_lo, dtype=np.float64)
        self.lo = lo
        edge = mesh.root_edge / 2.0 ** mesh.level.astype(np.float64)
        ijk = np.rint((mesh.origin - lo) / edge[:, None]).astype(np.int64)
        self.key = {(int(mesh.level[c]), *map(int, ijk[c])): c for c in range(mesh.n_cubes)}
        self.base = np.asarray(mesh.meta.get("base_dims") or np.rint(
            np.subtract(mesh.domain_hi, mesh.domain_lo) / mesh.root_edge).astype(int))
        self.h_cube = edge / mesh.n

    # ---- geometry ------------------------------------------------------------------------
    def cell_of(self, g):
        n = self.n
        c, r = divmod(int(g), n ** 3)
        k, r = divmod(r, n * n)
        j, i = divmod(r, n)
        return c, i, j, k

    def flat(self, c, i, j, k):
        n = self.n
        return ((c * n + k) * n + j) * n + i

    def _locate(self, level, X):
        """Cell containing point X among cubes of `level` (or None)."""
        e = self.m.root_edge / 2 ** level
        q = np.floor((X - self.lo) / e).astype(int)
        c = self.key.get((level, *map(int, q)))
        if c is None:
            return None
        h = self.h_cube[c]
        loc = np.floor((X - self.m.origin[c]) / h).astype(int)
        loc = np.clip(loc, 0, self.n - 1)
        return self.flat(c, *loc)

    def subfaces(self, g, f):
        """[(neighbour cell or None, area, distance, own weight, other weight, kind)]."""
        c, i, j, k = self.cell_of(g)
        d, s = divmod(f, 2)
        sg = 1 if s else -1
        h = self.h_cube[c]
        lv = int(self.m.level[c])
        cen = self.m.origin[c] + (np.array([i, j, k]) + 0.5) * h
        X = cen.copy()
        X[d] += sg * h
        ext = self.lo + self.base * self.m.root_edge
        if X[d] < self.lo[d] or X[d] > ext[d]:
            return [(None, h * h, h / 2, 1.0, 0.0, int(self.m.face_bc[c, f]))]
        nb = self._locate(lv, X)
        if nb is not None:
            return [(nb, h * h, h, 0.5, 0.5, 0)]
        Xc = cen.copy()
        Xc[d] += sg * 1.5 * h
        if lv > 0:
            nb = self._locate(lv - 1, Xc)
            if nb is not None:
                return [(nb, h * h, 1.5 * h, 2.0 / 3.0, 1.0 / 3.0, 0)]
        out = []
        t1, t2 = [a for a in range(3) if a != d]
        for a in (-0.25, 0.25):
            for b in (-0.25, 0.25):
                Xf = cen.copy()
                Xf[d] += sg * 0.75 * h
                Xf[t1] += a * h
                Xf[t2] += b * h
                nb = self._locate(lv + 1, Xf)
                assert nb is not None, "mesh is not 2:1 balanced"
                out.append((nb, h * h / 4, 0.75 * h, 1.0 / 3.0, 2.0 / 3.0, 0))
        return out

    # ---- operators at one cell -----------------------------------------------------------
    def laplacian(self, p, g):
        """(A p) at cell g."""
        c = self.cell_of(g)[0]
        V = self.h_cube[c] ** 3
        acc = 0.0
        for f in range(6):
            for nb, area, dist, _, _, kind in self.subfaces(g, f):
                if nb is None:
                    if kind == OUTFLOW:
                        acc += area * (0.0 - p[g]) / dist
                else:
                    acc += area * (p[nb] - p[g]) / dist
        return acc / V

    def face_velocity(self, u, g, f, U_in):
        """Outward normal velocity integrated over side f of cell g (sum of area * U)."""
        d, s = divmod(f, 2)
        sg = 1.0 if s else -1.0
        tot = 0.0
        for nb, area, dist, w_own, w_nb, kind in self.subfaces(g, f):
            if nb is None:
                U = {OUTFLOW: u[d][g], INFLOW: (U_in if s == 0 else -U_in), SLIP: 0.0}[kind]
            else:
                U = w_own * u[d][g] + w_nb * u[d][nb]
            tot += sg * area * U
        return tot

    def divergence(self, u, g, U_in):
        c = self.cell_of(g)[0]
        return sum(self.face_velocity(u, g, f, U_in) for f in range(6)) / self.h_cube[c] ** 3

    def face_gradient(self, p, g, f):
        """Area-weighted mean derivative along +axis over side f of cell g."""
        d, s = divmod(f, 2)
        sg = 1.0 if s else -1.0
        tot, A = 0.0, 0.0
        for nb, area, dist, _, _, kind in self.subfaces(g, f):
            if nb is None:
                der = (0.0 - p[g]) / dist if kind == OUTFLOW else 0.0
            else:
                der = (p[nb] - p[g]) / dist
            tot += area * sg * der
            A += area
        return tot / A

    def cell_gradient(self, p, g, d):
        return 0.5 * (self.face_gradient(p, g, 2 * d) + self.face_gradient(p, g, 2 * d + 1))

    def interface_cells(self, limit=None):
        """Flat indices of cells that touch a 2:1 interface or the domain boundary."""
        out = []
        n = self.n
        for c in range(self.m.n_cubes):
            for f in range(6):
                d, s = divmod(f, 2)
                lay = n - 1 if s else 0
                a = n // 3
                ijk = [a, a, a]
                ijk[d] = lay
                g = self.flat(c, *ijk)
                sub = self.subfaces(g, f)
                if sub[0][0] is None or len(sub) == 4 or sub[0][2] == 1.5 * self.h_cube[c]:
                    out.append(g)
                if limit and len(out) >= limit:
                    return out
        return out
