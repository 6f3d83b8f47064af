"""Single-level meshes as one global 3-D array: array-form operators and an exact spectral solve.

TEST INFRASTRUCTURE ONLY: the product path never imports this package.

A second, independent formulation of the finite-volume operators of fv.py for meshes whose cubes
all share one level and tile a box (every uniform workload).  Fields are scattered from the
cube-major layout into one array g[z, y, x] using the cube base corners, so this module does not
read the neighbour table either.  The Poisson solve is the closed-form eigen-decomposition of the
7-point operator with the boundary kinds of each axis:
  p = 0 on both faces        -> DST-II   basis sin(pi (k+1)(i+1/2)/N)
  dp/dn = 0 on both faces    -> DCT-II   basis cos(pi k (i+1/2)/N)
  dp/dn = 0 low, p = 0 high  -> DCT-IV   basis cos(pi (k+1/2)(i+1/2)/N)
  p = 0 low, dp/dn = 0 high  -> DST-IV   basis sin(pi (k+1/2)(i+1/2)/N)
with eigenvalues (2 cos theta_k - 2)/h^2, theta_k the basis frequency times pi/N.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

OUTFLOW, INFLOW, SLIP = 1, 2, 3


class UniformGrid:
    def __init__(self, mesh, workers=-1):
        assert np.all(mesh.level == mesh.level[0]), "single-level meshes only"
        self.mesh = mesh
        n = mesh.n
        self.n = n
        self.h = float(mesh.root_edge / 2.0 ** int(mesh.level[0]) / n)
        edge = self.h * n
        lo = np.asarray(mesh.domain_lo)
        self.cijk = np.rint((mesh.origin - lo) / edge).astype(np.int64)   # cube coords (x,y,z)
        self.dims_cubes = self.cijk.max(axis=0) + 1
        self.shape = tuple(int(v) for v in (self.dims_cubes[::-1] * n))  # (Nz, Ny, Nx)
        assert np.prod(self.dims_cubes) == mesh.n_cubes, "cubes must tile a box"
        self.workers = workers
        # boundary kind per domain side (-x,+x,-y,+y,-z,+z), read from any cube on that side
        side = []
        for f in range(6):
            d, s = divmod(f, 2)
            on = self.cijk[:, d] == (self.dims_cubes[d] - 1 if s else 0)
            kinds = np.unique(mesh.face_bc[on, f])
            assert kinds.size == 1 and kinds[0] in (OUTFLOW, INFLOW, SLIP)
            side.append(int(kinds[0]))
        self.side_bc = side

    # ---- layout ---------------------------------------------------------------------------
    def to_global(self, f):
        n = self.n
        f = np.asarray(f).reshape(self.mesh.n_cubes, n, n, n)
        g = np.empty(self.shape, dtype=f.dtype)
        for c in range(self.mesh.n_cubes):
            x, y, z = self.cijk[c]
            g[z * n:(z + 1) * n, y * n:(y + 1) * n, x * n:(x + 1) * n] = f[c]
        return g

    def to_cubes(self, g):
        n = self.n
        f = np.empty((self.mesh.n_cubes, n, n, n), dtype=g.dtype)
        for c in range(self.mesh.n_cubes):
            x, y, z = self.cijk[c]
            f[c] = g[z * n:(z + 1) * n, y * n:(y + 1) * n, x * n:(x + 1) * n]
        return f

    @staticmethod
    def _ax(d):
        return 2 - d          # axis d (x=0) lives on array axis 2 - d

    def _dirichlet(self, d):
        return self.side_bc[2 * d] == OUTFLOW, self.side_bc[2 * d + 1] == OUTFLOW

    # ---- operators (array form) --------------------------------------------------------------
    def face_velocity(self, u_d, d, U_in):
        """Normal velocity on the faces of axis d (N_d + 1 along that axis)."""
        ax = self._ax(d)
        u = np.moveaxis(u_d, ax, 0)
        lowbc, highbc = self.side_bc[2 * d], self.side_bc[2 * d + 1]
        U = np.empty((u.shape[0] + 1,) + u.shape[1:], dtype=np.result_type(u, U_in))
        U[1:-1] = 0.5 * (u[:-1] + u[1:])
        U[0] = {OUTFLOW: u[0], INFLOW: U_in, SLIP: 0.0}[lowbc]
        U[-1] = {OUTFLOW: u[-1], INFLOW: -U_in, SLIP: 0.0}[highbc]
        return np.moveaxis(U, 0, ax)

    def div(self, U):
        out = 0.0
        for d in range(3):
            out = out + np.diff(U[d], axis=self._ax(d)) / self.h
        return out

    def face_grad(self, p, d):
        ax = self._ax(d)
        q = np.moveaxis(p, ax, 0)
        G = np.zeros((q.shape[0] + 1,) + q.shape[1:], dtype=p.dtype)
        G[1:-1] = np.diff(q, axis=0) / self.h
        dl, dh = self._dirichlet(d)
        if dl:
            G[0] = q[0] / (self.h / 2)
        if dh:
            G[-1] = -q[-1] / (self.h / 2)
        return np.moveaxis(G, 0, ax)

    def cell_grad(self, p, d):
        G = np.moveaxis(self.face_grad(p, d), self._ax(d), 0)
        return np.moveaxis(0.5 * (G[:-1] + G[1:]), 0, self._ax(d))

    def laplacian(self, p):
        return self.div([self.face_grad(p, d) for d in range(3)])

    # ---- spectral solve ----------------------------------------------------------------------
    def _transform(self, d):
        dl, dh = self._dirichlet(d)
        if dl and dh:
            return "dst", 2, 1.0
        if not dl and not dh:
            return "dct", 2, 0.0
        if dh:
            return "dct", 4, 0.5
        return "dst", 4, 0.5

    def eigenvalues(self, d):
        N = self.shape[self._ax(d)]
        kind, typ, shift = self._transform(d)
        theta = np.pi * (np.arange(N) + shift) / N
        return (2.0 * np.cos(theta) - 2.0) / self.h ** 2

    def solve(self, b):
        bh = np.asarray(b)
        for d in range(3):
            kind, typ, _ = self._transform(d)
            f = sfft.dct if kind == "dct" else sfft.dst
            bh = f(bh, type=typ, axis=self._ax(d), norm="ortho", workers=self.workers)
        lam = (self.eigenvalues(0)[None, None, :] + self.eigenvalues(1)[None, :, None]
               + self.eigenvalues(2)[:, None, None])
        bh = bh / lam
        for d in range(3):
            kind, typ, _ = self._transform(d)
            f = sfft.idct if kind == "dct" else sfft.idst
            bh = f(bh, type=typ, axis=self._ax(d), norm="ortho", workers=self.workers)
        return bh

    def lambda_min_abs(self):
        """Smallest |eigenvalue| of the 7-point operator (bounds ||e|| <= ||r|| / lambda_min)."""
        return float(abs(self.eigenvalues(0)).min() + abs(self.eigenvalues(1)).min()
                     + abs(self.eigenvalues(2)).min())

    # ---- projection (global arrays) ------------------------------------------------------------
    def project(self, u_tilde, alpha, us, U_in, dt, rho):
        """Same step as projection.project, on cube-major inputs; returns cube-major outputs."""
        c = dt / rho
        a = self.to_global(alpha)
        ustar = [(1.0 - a) * self.to_global(u_tilde[d]) + a * us[d] for d in range(3)]
        U = [self.face_velocity(ustar[d], d, U_in) for d in range(3)]
        b = self.div(U) / c
        p = self.solve(b)
        Unew = [U[d] - c * self.face_grad(p, d) for d in range(3)]
        unew = [ustar[d] - c * self.cell_grad(p, d) for d in range(3)]
        return dict(u_star=np.stack([self.to_cubes(x) for x in ustar]), b=self.to_cubes(b),
                    p=self.to_cubes(p), u_new=np.stack([self.to_cubes(x) for x in unew]),
                    U_star_global=U, U_new_global=Unew, p_global=p, b_global=b)
