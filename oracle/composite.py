"""Finite-volume operators of a multi-level building-cube mesh as whole-array NumPy expressions.

TEST INFRASTRUCTURE ONLY: the product path never imports this package.

A third formulation of the operators of fv.py, for meshes too large to assemble (the
three-level mesh of 132.6M cells): fields stay in the cube-major layout [c][k][j][i], the cube
faces are classified once from the geometry (cube base corners and levels, like fv.py; the
neighbour table handed to the GPU library is not read), and each operator is a sum of
  * differences between neighbouring layers inside every cube (one array slice per axis), and
  * one term per cube face, evaluated for all cubes whose face has the same relation at once:
      same level       the neighbour's facing layer;
      coarser (2:1)    the coarse cell covering the fine cell's quadrant, at distance 3h/2;
      finer (2:1)      the four fine cells covering the coarse cell's face;
      domain boundary  open (p = 0 on the face), inflow or slip.
The face rules are those of the finite-volume discretisation of the projection step (Sec. 3,
Eq. (poisson); readings c3-c6 of the face interpolation, divergence and 2:1 interfaces):
  (A p)_i   = sum over the cell's faces of area * (outward face gradient) / V_i
  (D W u)_i = sum over the cell's faces of area * (outward face velocity) / V_i
with the face gradient (p_nb - p_i)/d (d = h, or 3h/2 across a 2:1 face, h/2 to an open
boundary where p = 0) and the face velocity the linear interpolation of the two cell values
(1/2, 1/2 on one level; 2/3 fine + 1/3 coarse across a 2:1 face), u_cell on an open boundary,
U_in into the domain on an inflow boundary and 0 on a slip wall.

Pinned against the assembled operators of fv.py (tests/test_oracle_composite.py) on uniform,
three-level and scaled-down three-level meshes.
"""
from __future__ import annotations

import numpy as np

OUTFLOW, INFLOW, SLIP = 1, 2, 3
SAME, COARSER, FINER, BOUNDARY = 0, 1, 2, 3


def _tangential(d):
    return [a for a in range(3) if a != d]


def face_layer(X, d, side, c):
    """Layer on face (d, side) of the cubes c of the cube fields X [n_c, n, n, n] ([k][j][i]), as
    [len(c), t2, t1] with the tangential axes (t1, t2) in increasing axis order."""
    idx = -1 if side else 0
    if d == 0:
        return X[c, :, :, idx]          # [k][j] = [t2 = z][t1 = y]
    if d == 1:
        return X[c, :, idx, :]          # [k][i] = [t2 = z][t1 = x]
    return X[c, idx, :, :]              # [j][i] = [t2 = y][t1 = x]


def _add_to_layer(out, c, d, side, val):
    """out[c] layer (d, side) += val (the cubes c are distinct)."""
    idx = -1 if side else 0
    if d == 0:
        out[c, :, :, idx] += val
    elif d == 1:
        out[c, :, idx, :] += val
    else:
        out[c, idx, :, :] += val


class CompositeMesh:
    """Face relations of every cube face, grouped for whole-array evaluation."""

    def __init__(self, mesh):
        self.mesh = mesh
        n = self.n = mesh.n
        nc = self.nc = mesh.n_cubes
        self.h = mesh.root_edge / 2.0 ** mesh.level.astype(np.float64) / n   # cell width per cube
        self.V = self.h ** 3
        lo = np.asarray(mesh.domain_lo, dtype=np.float64)
        edge = self.h * n
        ijk = np.rint((mesh.origin - lo) / edge[:, None]).astype(np.int64)
        lv = mesh.level.astype(np.int64)
        lookup = {(int(lv[c]), *map(int, ijk[c])): c for c in range(nc)}
        base = np.rint(np.subtract(mesh.domain_hi, mesh.domain_lo) / mesh.root_edge).astype(int)
        # per face: lists of (cube, ...) by relation
        self.groups = []
        for f in range(6):
            d, side = divmod(f, 2)
            t1, t2 = _tangential(d)
            same, coarser, finer, bnd = [], [], [], []
            for c in range(nc):
                L = int(lv[c])
                q = list(map(int, ijk[c]))
                q[d] += 1 if side else -1
                ext = base * 2 ** L
                if not (0 <= q[d] < ext[d]):
                    bnd.append((c, int(mesh.face_bc[c, f])))
                    continue
                o = lookup.get((L, *q))
                if o is not None:
                    same.append((c, o))
                    continue
                par = lookup.get((L - 1, q[0] >> 1, q[1] >> 1, q[2] >> 1)) if L > 0 else None
                if par is not None:
                    coarser.append((c, par, int(ijk[c][t1] & 1), int(ijk[c][t2] & 1)))
                    continue
                ch = []
                for w in range(4):
                    r = [2 * v for v in q]
                    r[d] += 0 if side else 1
                    r[t1] += w & 1
                    r[t2] += w >> 1
                    ch.append(lookup[(L + 1, *r)])      # KeyError: not 2:1 balanced
                finer.append((c, *ch))
            arr = lambda x, k: np.array(x, dtype=np.int64).reshape(-1, k)
            self.groups.append(dict(d=d, side=side, same=arr(same, 2), coarser=arr(coarser, 4),
                                    finer=arr(finer, 5), bnd=arr(bnd, 2)))

    # -- ghost layers --------------------------------------------------------------------------
    def _coarse_ghost(self, X, g, d, side):
        """Value of the covering coarse cell for every fine cell of the fine cubes' faces."""
        n, H = self.n, self.n // 2
        c, o, q1, q2 = g.T
        lay = face_layer(X, d, 1 - side, o)                     # [m, t2, t1] of the coarse cube
        a = np.arange(n) // 2
        i1 = q1[:, None] * H + a[None, :]                       # coarse t1 index per fine t1
        i2 = q2[:, None] * H + a[None, :]
        m = np.arange(len(c))[:, None, None]
        return lay[m, i2[:, :, None], i1[:, None, :]]

    def _fine_mean(self, X, g, d, side):
        """Mean of the four fine cells facing every coarse cell of the coarse cubes' faces."""
        n, H = self.n, self.n // 2
        out = np.empty((len(g), n, n), dtype=X.dtype)
        for w in range(4):
            lay = face_layer(X, d, 1 - side, g[:, 1 + w])        # [m, t2, t1] of fine cube w
            s = lay.reshape(len(g), H, 2, H, 2)
            mean = ((s[:, :, 0, :, 0] + s[:, :, 0, :, 1]) + s[:, :, 1, :, 0]) + s[:, :, 1, :, 1]
            b, a = w >> 1, w & 1
            out[:, b * H:(b + 1) * H, a * H:(a + 1) * H] = 0.25 * mean
        return out

    # -- operators -----------------------------------------------------------------------------
    def laplacian(self, p):
        """A p for p [n_c * n^3] (or [n_c, n, n, n]); returns [n_c, n, n, n]."""
        n = self.n
        P = np.asarray(p, dtype=np.float64).reshape(self.nc, n, n, n)
        out = np.zeros_like(P)
        for ax in (1, 2, 3):                     # interior faces: (neighbour - own) per side
            sl_lo = [slice(None)] * 4
            sl_hi = [slice(None)] * 4
            sl_lo[ax] = slice(0, n - 1)
            sl_hi[ax] = slice(1, n)
            diff = P[tuple(sl_hi)] - P[tuple(sl_lo)]
            out[tuple(sl_lo)] += diff
            out[tuple(sl_hi)] -= diff
        for g in self.groups:
            d, side = g["d"], g["side"]
            if len(g["same"]):
                c, o = g["same"].T
                own = face_layer(P, d, side, c)
                term = face_layer(P, d, 1 - side, o) - own
                self._scatter(out, c, d, side, term)
            if len(g["coarser"]):               # fine cube: (2/3)(P_coarse - p)
                c = g["coarser"][:, 0]
                own = face_layer(P, d, side, c)
                term = (2.0 / 3.0) * (self._coarse_ghost(P, g["coarser"], d, side) - own)
                self._scatter(out, c, d, side, term)
            if len(g["finer"]):                 # coarse cube: (4/3)(mean of 4 fine - p)
                c = g["finer"][:, 0]
                own = face_layer(P, d, side, c)
                term = (4.0 / 3.0) * (self._fine_mean(P, g["finer"], d, side) - own)
                self._scatter(out, c, d, side, term)
            if len(g["bnd"]):                   # open: p = 0 at h/2 -> -2 p; else no flux
                c, kind = g["bnd"].T
                c = c[kind == OUTFLOW]
                if len(c):
                    self._scatter(out, c, d, side, -2.0 * face_layer(P, d, side, c))
        out /= (self.h ** 2)[:, None, None, None]
        return out

    @staticmethod
    def _scatter(out, c, d, side, term):
        _add_to_layer(out, c, d, side, term)

    def divergence(self, u, U_in):
        """D W u (+ inflow): the face-flux divergence of the interpolated face velocities of the
        cell velocity u [3][n_c * n^3]; returns [n_c, n, n, n]."""
        n = self.n
        U = [np.asarray(u[a], dtype=np.float64).reshape(self.nc, n, n, n) for a in range(3)]
        out = np.zeros_like(U[0])
        for d in range(3):
            ax = 3 - d
            X = U[d]
            sl_lo = [slice(None)] * 4
            sl_hi = [slice(None)] * 4
            sl_lo[ax] = slice(0, n - 1)
            sl_hi[ax] = slice(1, n)
            face = 0.5 * (X[tuple(sl_lo)] + X[tuple(sl_hi)])     # interior faces of axis d
            out[tuple(sl_lo)] += face
            out[tuple(sl_hi)] -= face
        for g in self.groups:
            d, side = g["d"], g["side"]
            X = U[d]
            sgn = 1.0 if side else -1.0          # outward normal along +d or -d
            if len(g["same"]):
                c, o = g["same"].T
                fv = 0.5 * (face_layer(X, d, side, c) + face_layer(X, d, 1 - side, o))
                self._scatter(out, c, d, side, sgn * fv)
            if len(g["coarser"]):
                c = g["coarser"][:, 0]
                fv = (2.0 / 3.0) * face_layer(X, d, side, c) + (1.0 / 3.0) * \
                    self._coarse_ghost(X, g["coarser"], d, side)
                self._scatter(out, c, d, side, sgn * fv)
            if len(g["finer"]):                  # mean of the 4 sub-face velocities
                c = g["finer"][:, 0]
                fv = (2.0 / 3.0) * self._fine_mean(X, g["finer"], d, side) + (1.0 / 3.0) * \
                    face_layer(X, d, side, c)
                self._scatter(out, c, d, side, sgn * fv)
            if len(g["bnd"]):
                c, kind = g["bnd"].T
                for k, val in ((OUTFLOW, None), (INFLOW, U_in)):
                    cc = c[kind == k]
                    if not len(cc):
                        continue
                    if val is None:
                        fv = face_layer(X, d, side, cc)
                        self._scatter(out, cc, d, side, sgn * fv)
                    else:                        # U_in into the domain: +U_in on a minus face
                        fv = np.full((len(cc), n, n), -sgn * val)
                        self._scatter(out, cc, d, side, sgn * fv)
        out /= self.h[:, None, None, None]
        return out

    def residual_norm(self, p, b):
        """Volume-weighted relative residual sqrt(sum V r^2 / sum V b^2) of A p = b."""
        n = self.n
        B = np.asarray(b, dtype=np.float64).reshape(self.nc, n, n, n)
        r = B - self.laplacian(p)
        V = self.V[:, None, None, None]
        return float(np.sqrt(np.sum(V * r * r) / np.sum(V * B * B)))
