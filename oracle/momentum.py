"""Momentum sub-step of the fractional-step method (FP64, single-level meshes).

TEST INFRASTRUCTURE ONLY: the product path never imports this package.

Sec. 3, Eq. (substep1): the intermediate velocity u~ solves a momentum equation without the
body force and without the pressure gradient,
    (u~ - u^n)/dt = (1/2) [H(u~) + H(u^n)]          (Crank-Nicolson, the scheme written out)
with H(v) = -A[v] + nu D[v] (nu = mu/rho), A the advection operator and D the diffusion
operator.  The paper also names explicit Euler and Adams-Bashforth:
    Euler   u~ = u^n + dt H(u^n)
    AB2     u~ = u^n + dt (3/2 H(u^n) - 1/2 H(u^{n-1}))
and uses the QUICK scheme for the convective term (Sec. 6.6, Sec. 7).  Readings (the paper
does not spell the discrete operators out):
  m1  A is linear in its argument: the advecting velocity is frozen at u^n (the same in every
      evaluation of one step), so Crank-Nicolson is one linear system for u~.
  m2  Finite-volume flux form on the cell-centred grid: for component c,
        A[v]_i = (1/h) sum_d ( U_d(i+1/2) q(i+1/2) - U_d(i-1/2) q(i-1/2) ),
      U_d = face-normal advecting velocity = mean of the two cells' u^n_d (the face rule of the
      projection step), q = QUICK face value of v_c: for U >= 0,
        q(i+1/2) = 6/8 v(i) + 3/8 v(i+1) - 1/8 v(i-1),
      and the mirror image (6/8 v(i+1) + 3/8 v(i) - 1/8 v(i+2)) for U < 0.
        D[v]_i = sum_d (v(i+e_d) - 2 v(i) + v(i-e_d)) / h^2.
  m3  Velocity boundary values by ghost cells, two layers deep (QUICK reaches two cells
      upwind), mirrored about the boundary face:
        Dirichlet value g:  ghost_l = 2 g - v_l      (l = 0, 1: first and second interior cell)
        Neumann (zero gradient):  ghost_l = v_l
      inflow face: every component Dirichlet (normal component U_in into the domain,
      tangential 0); slip wall: normal component Dirichlet 0, tangential Neumann; open
      (outflow) face: every component Neumann.  The advecting face velocity on a boundary face
      is then U_in, 0 and the boundary cell's value: the projection step's face rules.
  m4  Crank-Nicolson's linear system is solved exactly (to rounding, BiCGSTAB to 1e-14 on the
      global array; or dense on tiny meshes); the GPU path iterates to a stated tolerance.
Multi-level meshes are not covered (the GPU path rejects them too).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .uniform import UniformGrid

OUTFLOW, INFLOW, SLIP = 1, 2, 3


class MomentumGrid:
    """H(v) on one global array per component, with the ghost rules of m3."""

    def __init__(self, mesh):
        self.ug = UniformGrid(mesh)
        self.h = self.ug.h
        self.shape = self.ug.shape
        self.side_bc = self.ug.side_bc

    # -- ghosts ----------------------------------------------------------------------------
    def _rule(self, f, comp, U_in):
        """(kind, value) of component comp on domain side f: ('D', g) or ('N', None)."""
        d, side = divmod(f, 2)
        kind = self.side_bc[f]
        if kind == OUTFLOW:
            return "N", None
        if kind == INFLOW:
            return "D", ((-U_in if side else U_in) if comp == d else 0.0)
        return ("D", 0.0) if comp == d else ("N", None)

    def padded(self, v, comp, U_in):
        """v [Nz, Ny, Nx] with two ghost layers on every side (edges/corners unused: filled from
        one axis at a time, which the per-axis stencils never read)."""
        g = np.pad(np.asarray(v), 2)
        for d in range(3):
            ax = 2 - d
            for side in (0, 1):
                kind, val = self._rule(2 * d + side, comp, U_in)
                m = np.moveaxis(g, ax, 0)
                for l in (0, 1):
                    src = (2 + l) if side == 0 else (-3 - l)
                    dst = (1 - l) if side == 0 else (-2 + l)
                    if kind == "D":
                        m[dst] = 2.0 * val - m[src]
                    else:
                        m[dst] = m[src]
        return g

    # -- operator ----------------------------------------------------------------------------
    def H(self, v, a, nu, U_in):
        """H(v) = -A[v] + nu D[v] for the three components of v with advecting velocity a
        (each a list of three [Nz, Ny, Nx] arrays); returns the list of three results."""
        h = self.h
        ap = [self.padded(a[d], d, U_in) for d in range(3)]
        out = []
        for c in range(3):
            vp = self.padded(v[c], c, U_in)
            acc = np.zeros(self.shape, dtype=np.result_type(vp, ap[0]))
            for d in range(3):
                ax = 2 - d
                V = np.moveaxis(vp, ax, 0)
                Ad = np.moveaxis(ap[d], ax, 0)
                n = V.shape[0] - 4
                # faces i+1/2 for i = -1 .. n-1 (index f = i + 1): the cell's - and + faces
                L = lambda o: V[1 + o: 1 + o + n + 1]             # v(i + o) for the n+1 faces
                Ua = 0.5 * (Ad[1:2 + n] + Ad[2:3 + n])           # advecting velocity on faces
                q_pos = 0.75 * L(0) + 0.375 * L(1) - 0.125 * L(-1)
                q_neg = 0.75 * L(1) + 0.375 * L(0) - 0.125 * L(2)
                flux = Ua * np.where(Ua >= 0, q_pos, q_neg)
                conv = (flux[1:] - flux[:-1]) / h
                diff = (V[3:3 + n] - 2.0 * V[2:2 + n] + V[1:1 + n]) / (h * h)
                # restore this axis to its place, dropping the other axes' ghost layers
                sl = [slice(2, -2)] * 3
                sl[0] = slice(None)
                term = (nu * diff - conv)[tuple(sl)]
                acc = acc + np.moveaxis(term, 0, ax)
            out.append(acc)
        return out

    # -- schemes -------------------------------------------------------------------------------
    def euler(self, u, nu, U_in, dt, a=None):
        Hn = self.H(u, u if a is None else a, nu, U_in)
        return [u[c] + dt * Hn[c] for c in range(3)], Hn

    def ab2(self, u, h_prev, nu, U_in, dt):
        Hn = self.H(u, u, nu, U_in)
        return [u[c] + dt * (1.5 * Hn[c] - 0.5 * h_prev[c]) for c in range(3)], Hn

    def cn(self, u, nu, U_in, dt, rtol=1e-14, dense=False, a=None):
        """u~ with u~ - (dt/2) H(u~) = u^n + (dt/2) H(u^n), H affine in its argument (m1); the
        advecting velocity a is u^n unless given."""
        a = u if a is None else a
        Hn = self.H(u, a, nu, U_in)
        shape = self.shape
        N = int(np.prod(shape))
        zero = [np.zeros(shape) for _ in range(3)]
        h0 = self.H(zero, a, nu, U_in)               # the affine part (boundary values)
        rhs = np.concatenate([(u[c] + 0.5 * dt * Hn[c] + 0.5 * dt * h0[c]).ravel()
                              for c in range(3)])

        def matvec(x):
            xs = [x[c * N:(c + 1) * N].reshape(shape) for c in range(3)]
            hx = self.H(xs, a, nu, U_in)
            return np.concatenate([(xs[c] - 0.5 * dt * (hx[c] - h0[c])).ravel()
                                   for c in range(3)])

        if dense:
            M = np.stack([matvec(e) for e in np.eye(3 * N)], axis=1)
            x = np.linalg.solve(M, rhs)
        else:
            op = spla.LinearOperator((3 * N, 3 * N), matvec=matvec, dtype=np.float64)
            x0 = np.concatenate([u[c].ravel() for c in range(3)])
            x, info = spla.bicgstab(op, rhs, x0=x0, rtol=rtol, atol=0.0, maxiter=2000)
            assert info == 0, "oracle BiCGSTAB did not converge"
        return [x[c * N:(c + 1) * N].reshape(shape) for c in range(3)], Hn

    # -- cube-major helpers ----------------------------------------------------------------------
    def to_global(self, f):
        return self.ug.to_global(f)

    def to_cubes(self, g):
        return self.ug.to_cubes(g)


def step(mesh, u, nu, U_in, dt, scheme, h_prev=None):
    """One momentum sub-step on cube-major fields u [3][n_c * n^3]; returns (u~, H(u^n)) in the
    same layout (each [3, n_c * n^3])."""
    mg = MomentumGrid(mesh)
    ug = [mg.to_global(np.asarray(u[c]).reshape(-1)) for c in range(3)]
    if scheme == "euler":
        ut, Hn = mg.euler(ug, nu, U_in, dt)
    elif scheme == "ab2":
        hp = [mg.to_global(np.asarray(h_prev[c]).reshape(-1)) for c in range(3)]
        ut, Hn = mg.ab2(ug, hp, nu, U_in, dt)
    elif scheme == "cn":
        ut, Hn = mg.cn(ug, nu, U_in, dt)
    else:
        raise ValueError(scheme)
    return (np.stack([mg.to_cubes(x).reshape(-1) for x in ut]),
            np.stack([mg.to_cubes(x).reshape(-1) for x in Hn]))
