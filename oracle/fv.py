"""Finite-volume form of the projection operators, assembled as sparse matrices (FP64).

TEST INFRASTRUCTURE ONLY: the product path never imports this package.

Everything here is derived from the mesh *geometry* (cube base corners and levels); the
neighbour table handed to the GPU library is not read, so this module also checks it.

Discretisation (the paper's collocated, cell-centred arrangement, Sec. 2.2; fractional step,
Sec. 3).  Every face between two cells (or a cell and the domain boundary) carries:
  area a_f, centre-to-centre distance d_f, interpolation weights (w_L, w_R) and, on the domain
  boundary, a kind.  Same-level faces: a = h^2, d = h, w = (1/2, 1/2).  Faces between a fine cell
  (width h) and a coarse cell (width 2h) across a 2:1 cube interface: a = h^2, d = 3h/2, weights
  (2/3 fine, 1/3 coarse), i.e. linear interpolation to the face.
Operators (cell volume V_i = h_i^3, U_f = normal velocity along +axis):
  face velocity   U_f = w_L u_L + w_R u_R               (Poisson right-hand side, Sec. 3)
  face gradient   G p = (p_R - p_L) / d_f
  divergence      (D U)_i = (1/V_i) sum_f (+/-) a_f U_f   (outward sign)
  Laplacian       A = D G                               (pressure Poisson equation, Sec. 3)
  cell gradient   (G_c p)_i,d = mean of the area-weighted face gradients on the -d and +d sides
Boundary kinds: OUTFLOW (open): U_f = u_cell, p = 0 on the face (G = -+2 p / h);
INFLOW: U_f = U_in into the domain, dp/dn = 0;  SLIP: U_f = 0, dp/dn = 0.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

OUTFLOW, INFLOW, SLIP = 1, 2, 3


def _cube_keys(mesh):
    """Integer cube coordinates at each cube's own level, from the base corners."""
    lo = np.asarray(mesh.domain_lo, dtype=np.float64)
    edge = mesh.root_edge / 2.0 ** mesh.level.astype(np.float64)
    ijk = np.rint((mesh.origin - lo) / edge[:, None]).astype(np.int64)
    return [(int(mesh.level[c]), *map(int, ijk[c])) for c in range(mesh.n_cubes)]


def _tangential(d):
    return [a for a in range(3) if a != d]


class FVMesh:
    """Faces and sparse operators of a building-cube mesh (any number of levels)."""

    def __init__(self, mesh):
        self.mesh = mesh
        n = mesh.n
        self.n = n
        nc = mesh.n_cubes
        self.n_cells = nc * n ** 3
        self.h_cube = mesh.root_edge / 2.0 ** mesh.level.astype(np.float64) / n
        self.V = np.repeat(self.h_cube ** 3, n ** 3)
        self.h_cell = np.repeat(self.h_cube, n ** 3)
        keys = _cube_keys(mesh)
        lookup = {k: c for c, k in enumerate(keys)}
        base = np.asarray(mesh.meta.get("base_dims", None) or
                          np.rint((np.subtract(mesh.domain_hi, mesh.domain_lo))
                                  / mesh.root_edge).astype(int))

        def inside(lv, c):
            ext = base * 2 ** lv
            return all(0 <= c[a] < ext[a] for a in range(3))

        a_idx = np.arange(n)
        A2, B2 = np.meshgrid(a_idx, a_idx, indexing="ij")   # tangential (t1, t2) indices
        A2 = A2.ravel()
        B2 = B2.ravel()

        def cell(c, d, layer, t1v, t2v):
            ijk = [None, None, None]
            ijk[d] = np.full_like(t1v, layer)
            t1, t2 = _tangential(d)
            ijk[t1] = t1v
            ijk[t2] = t2v
            return c * n ** 3 + (ijk[2] * n + ijk[1]) * n + ijk[0]

        L, R, AX, AREA, DIST, WL, WR, BC, BSIDE = ([] for _ in range(9))

        def add(l, r, d, area, dist, wl, wr, bc=0, bside=0):
            m = len(l)
            L.append(l)
            R.append(r)
            AX.append(np.full(m, d))
            AREA.append(np.full(m, area))
            DIST.append(np.full(m, dist))
            WL.append(np.full(m, wl))
            WR.append(np.full(m, wr))
            BC.append(np.full(m, bc))
            BSIDE.append(np.full(m, bside))

        for c, key in enumerate(keys):
            lv = key[0]
            h = self.h_cube[c]
            for d in range(3):          # faces inside the cube, between layers l and l + 1
                lay = np.repeat(np.arange(n - 1), n * n)
                t1v = np.tile(A2, n - 1)
                t2v = np.tile(B2, n - 1)
                lo_c = cell(c, d, 0, t1v, t2v) + lay * (n ** d)
                add(lo_c, lo_c + n ** d, d, h * h, h, 0.5, 0.5)
            for f in range(6):
                d, side = divmod(f, 2)
                nb = list(key[1:])
                nb[d] += 1 if side else -1
                if not inside(lv, nb):
                    kind = int(mesh.face_bc[c, f])
                    assert kind in (OUTFLOW, INFLOW, SLIP), "boundary face without a kind"
                    own = cell(c, d, n - 1 if side else 0, A2, B2)
                    none = -np.ones_like(own)
                    if side:
                        add(own, none, d, h * h, h / 2, 1.0, 0.0, kind, +1)
                    else:
                        add(none, own, d, h * h, h / 2, 0.0, 1.0, kind, -1)
                    continue
                if (lv, *nb) in lookup:
                    if side:           # count each same-level face once, from its minus cube
                        o = lookup[(lv, *nb)]
                        add(cell(c, d, n - 1, A2, B2), cell(o, d, 0, A2, B2), d, h * h, h,
                            0.5, 0.5)
                    continue
                par = (lv - 1, nb[0] >> 1, nb[1] >> 1, nb[2] >> 1)
                if lv > 0 and par in lookup:
                    # this (fine) cube touches a coarser cube: n^2 fine sub-faces
                    o = lookup[par]
                    t1, t2 = _tangential(d)
                    q1 = key[1 + t1] & 1
                    q2 = key[1 + t2] & 1
                    ct1 = q1 * (n // 2) + A2 // 2
                    ct2 = q2 * (n // 2) + B2 // 2
                    fine = cell(c, d, n - 1 if side else 0, A2, B2)
                    coarse = cell(o, d, 0 if side else n - 1, ct1, ct2)
                    if side:
                        add(fine, coarse, d, h * h, 1.5 * h, 2.0 / 3.0, 1.0 / 3.0)
                    else:
                        add(coarse, fine, d, h * h, 1.5 * h, 1.0 / 3.0, 2.0 / 3.0)
                    continue
                # otherwise the neighbour region is finer: its cubes add the shared faces
                t1, t2 = _tangential(d)
                for q in range(4):
                    ch = [2 * v for v in nb]
                    ch[d] += 0 if side else 1
                    ch[t1] += q & 1
                    ch[t2] += q >> 1
                    assert (lv + 1, *ch) in lookup, "mesh is not 2:1 face balanced"

        self.L = np.concatenate(L)
        self.R = np.concatenate(R)
        self.axis = np.concatenate(AX)
        self.area = np.concatenate(AREA)
        self.dist = np.concatenate(DIST)
        self.wL = np.concatenate(WL)
        self.wR = np.concatenate(WR)
        self.bc = np.concatenate(BC)
        self.bside = np.concatenate(BSIDE)
        self.n_faces = self.L.size
        self._build()

    # -------------------------------------------------------------------------------------
    def _build(self):
        F, C = self.n_faces, self.n_cells
        f = np.arange(F)
        hasL = self.L >= 0
        hasR = self.R >= 0
        interior = hasL & hasR
        out = self.bc == OUTFLOW
        # face gradient G (F x C)
        rows, cols, vals = [], [], []
        rows += [f[interior], f[interior]]
        cols += [self.R[interior], self.L[interior]]
        vals += [1.0 / self.dist[interior], -1.0 / self.dist[interior]]
        bl = out & hasL & ~hasR       # domain +side: p_face = 0, derivative (0 - p)/(h/2)
        br = out & hasR & ~hasL       # domain -side: derivative (p - 0)/(h/2)
        rows += [f[bl], f[br]]
        cols += [self.L[bl], self.R[br]]
        vals += [-1.0 / self.dist[bl], 1.0 / self.dist[br]]
        self.G = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows),
                                                       np.concatenate(cols))), shape=(F, C))
        # face velocity W (F x 3C) acting on [u_x; u_y; u_z], and the inflow vector w0 (F)
        rows, cols, vals = [], [], []
        offL = self.axis * C + np.where(hasL, self.L, 0)
        offR = self.axis * C + np.where(hasR, self.R, 0)
        rows += [f[interior], f[interior]]
        cols += [offL[interior], offR[interior]]
        vals += [self.wL[interior], self.wR[interior]]
        rows += [f[out & hasL & ~hasR], f[out & hasR & ~hasL]]
        cols += [offL[out & hasL & ~hasR], offR[out & hasR & ~hasL]]
        vals += [np.ones((out & hasL & ~hasR).sum()), np.ones((out & hasR & ~hasL).sum())]
        self.W = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows),
                                                       np.concatenate(cols))), shape=(F, 3 * C))
        w0 = np.zeros(F)
        inflow = self.bc == INFLOW
        w0[inflow] = np.where(self.bside[inflow] < 0, 1.0, -1.0)
        self.w0 = w0
        # divergence D (C x F)
        rows = np.concatenate([self.L[hasL], self.R[hasR]])
        cols = np.concatenate([f[hasL], f[hasR]])
        vals = np.concatenate([self.area[hasL] / self.V[self.L[hasL]],
                               -self.area[hasR] / self.V[self.R[hasR]]])
        self.D = sp.csr_matrix((vals, (rows, cols)), shape=(C, F))
        # cell gradient averaging Gc (3C x F): half the area-weighted face gradient of each side
        hc = self.h_cell
        rows = np.concatenate([self.axis[hasL] * C + self.L[hasL],
                               self.axis[hasR] * C + self.R[hasR]])
        vals = np.concatenate([0.5 * self.area[hasL] / hc[self.L[hasL]] ** 2,
                               0.5 * self.area[hasR] / hc[self.R[hasR]] ** 2])
        self.Gc = sp.csr_matrix((vals, (rows, cols)), shape=(3 * C, F))
        self.A = (self.D @ self.G).tocsr()
        self._lu = None
        self._luT = None

    # -------------------------------------------------------------------------------------
    def face_velocity(self, u_star, U_in):
        return self.W @ u_star.reshape(-1) + self.w0 * U_in

    LU_MAX_CELLS = 60000

    def _uniform(self):
        if not hasattr(self, "_ug"):
            self._ug = None
            if np.all(self.mesh.level == self.mesh.level[0]):
                from .uniform import UniformGrid
                self._ug = UniformGrid(self.mesh)
        return self._ug

    def solve(self, b):
        """p = A^{-1} b: exact spectral solve on single-level meshes, sparse LU on small
        multi-level meshes, else conjugate gradients on the symmetric -V A to 1e-14."""
        ug = self._uniform()
        if ug is not None:
            return self._spectral(ug, b)
        if self.n_cells <= self.LU_MAX_CELLS:
            if self._lu is None:
                self._lu = spla.splu(self.A.tocsc())
            return self._solve(self._lu, b)
        return self._cg(b)

    def solve_T(self, g):
        """A^{-T} g.  V A is symmetric, so A^{-T} = V A^{-1} V^{-1}."""
        ug = self._uniform()
        if ug is not None:
            return self._spectral(ug, g)          # A itself is symmetric on one level
        if self.n_cells <= self.LU_MAX_CELLS:
            if self._luT is None:
                self._luT = spla.splu(self.A.T.tocsc())
            return self._solve(self._luT, g)
        return self.V * self._cg(g / self.V)

    def _spectral(self, ug, b):
        b = np.asarray(b)
        if np.iscomplexobj(b):
            return self._spectral(ug, b.real) + 1j * self._spectral(ug, b.imag)
        return ug.to_cubes(ug.solve(ug.to_global(b.reshape(-1)))).reshape(-1)

    def _cg(self, b, rtol=1e-14):
        b = np.asarray(b)
        if np.iscomplexobj(b):
            return self._cg(b.real, rtol) + 1j * self._cg(b.imag, rtol)
        M = (-sp.diags(self.V) @ self.A).tocsr()
        x, info = spla.cg(M, -self.V * b, rtol=rtol, maxiter=20000,
                          M=sp.diags(1.0 / M.diagonal()))
        assert info == 0, "oracle CG did not converge"
        return x

    @staticmethod
    def _solve(lu, b):
        b = np.asarray(b)
        if np.iscomplexobj(b):
            return lu.solve(b.real.copy()) + 1j * lu.solve(b.imag.copy())
        return lu.solve(b)

    def residual_norm(self, p, b):
        """Volume-weighted relative residual sqrt(sum V r^2) / sqrt(sum V b^2)."""
        r = b - self.A @ p
        return float(np.sqrt(np.sum(self.V * r * r) / np.sum(self.V * b * b)))
