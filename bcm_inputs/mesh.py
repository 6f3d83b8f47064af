"""Building-cube meshes as linear arrays (cube list, levels, neighbour table, boundary kinds).

The paper's mesh representation (Sec. 2.2, "Building Cube Method"): no tree, only per-cube base
corner, size (level), an index, the cell count and neighbour adjacency, with a refinement ratio
of 2 between levels and the same number of cells in every cube.  Cubes are ordered along a
Z-order (Morton) space-filling curve, as the paper's mesh generator does (Sec. 6.1).

This module describes *inputs* only: it does no arithmetic of the projection method.

Conventions shared by every consumer:
  * face f in 0..5 is (-x, +x, -y, +y, -z, +z); axis = f // 2, side = f % 2 (0 = minus, 1 = plus).
  * nbr[c, f, :] (int32, 4 slots):
      - same level or coarser neighbour: slot 0 holds its id, slots 1..3 are -1;
      - finer neighbours (2:1): the 4 sub-neighbours covering the face, slot q = a + 2*b where a/b
        are the half (0 = lower, 1 = upper) along the first/second tangential axis, tangential axes
        taken in increasing axis order (x-face: (y, z); y-face: (x, z); z-face: (x, y));
      - domain boundary: all four slots -1, and face_bc[c, f] gives its kind.
  * face_bc[c, f] (int8): BC_NONE for interior faces, else BC_OUTFLOW (open, p = 0),
    BC_INFLOW (normal velocity U_in into the domain, p Neumann) or BC_SLIP (zero normal
    velocity, p Neumann).
  * cell (i, j, k) of cube c has centre origin[c] + ((i+1/2) h, (j+1/2) h, (k+1/2) h) with
    h = edge(level) / n; fields are stored cube-major as [c][k][j][i] (i fastest).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

BC_NONE, BC_OUTFLOW, BC_INFLOW, BC_SLIP = 0, 1, 2, 3
BC_NAMES = {"none": BC_NONE, "outflow": BC_OUTFLOW, "inflow": BC_INFLOW, "slip": BC_SLIP}


@dataclass
class Mesh:
    n: int                      # cells per cube edge
    root_edge: float            # edge of a level-0 cube
    origin: np.ndarray          # float64 [n_c, 3] base (minimum) corner
    level: np.ndarray           # int8 [n_c]
    nbr: np.ndarray             # int32 [n_c, 6, 4]
    face_bc: np.ndarray         # int8 [n_c, 6]
    domain_lo: tuple = (0.0, 0.0, 0.0)
    domain_hi: tuple = (1.0, 1.0, 1.0)
    meta: dict = field(default_factory=dict)

    @property
    def n_cubes(self) -> int:
        return int(self.origin.shape[0])

    @property
    def n_cells(self) -> int:
        return self.n_cubes * self.n ** 3

    @property
    def max_level(self) -> int:
        return int(self.level.max()) if self.n_cubes else 0

    def edge(self) -> np.ndarray:
        """Cube edge length per cube (float64 [n_c])."""
        return self.root_edge / (2.0 ** self.level.astype(np.float64))

    def h(self) -> np.ndarray:
        """Cell width per cube (float64 [n_c])."""
        return self.edge() / self.n

    def cell_centres(self):
        """(X, Y, Z), each float64 [n_c, n, n, n] in [c][k][j][i] order."""
        n = self.n
        s = np.arange(n, dtype=np.float64) + 0.5
        h = self.h()[:, None, None, None]
        X = self.origin[:, 0, None, None, None] + s[None, None, None, :] * h
        Y = self.origin[:, 1, None, None, None] + s[None, None, :, None] * h
        Z = self.origin[:, 2, None, None, None] + s[None, :, None, None] * h
        X, Y, Z = np.broadcast_arrays(X, Y, Z)
        return X.copy(), Y.copy(), Z.copy()

    def with_bc(self, side_bc) -> "Mesh":
        """Copy with the boundary kind of every domain-boundary face reset from side_bc[6]."""
        out = Mesh(self.n, self.root_edge, self.origin.copy(), self.level.copy(), self.nbr.copy(),
                   self.face_bc.copy(), self.domain_lo, self.domain_hi, dict(self.meta))
        bnd = out.nbr[:, :, 0] < 0
        for f in range(6):
            out.face_bc[bnd[:, f], f] = _bc_code(side_bc[f])
        return out


def _bc_code(v) -> int:
    return BC_NAMES[v] if isinstance(v, str) else int(v)


def morton3(ix, iy, iz, bits: int = 21) -> np.ndarray:
    """Interleave the bits of integer coordinates (x lowest) into a Z-order key."""
    ix = np.asarray(ix, dtype=np.uint64)
    iy = np.asarray(iy, dtype=np.uint64)
    iz = np.asarray(iz, dtype=np.uint64)
    key = np.zeros(ix.shape, dtype=np.uint64)
    for b in range(bits):
        one = np.uint64(1)
        key |= ((ix >> np.uint64(b)) & one) << np.uint64(3 * b)
        key |= ((iy >> np.uint64(b)) & one) << np.uint64(3 * b + 1)
        key |= ((iz >> np.uint64(b)) & one) << np.uint64(3 * b + 2)
    return key


def _tangential(axis: int):
    return [a for a in range(3) if a != axis]


def build_mesh(base_dims, root_edge, n, side_bc, refine=None, max_level=0,
               domain_lo=(0.0, 0.0, 0.0)) -> Mesh:
    """Generate a 2:1 face-balanced building-cube mesh.

    base_dims: level-0 cube counts (nx, ny, nz); root_edge: level-0 cube edge; n: cells per edge;
    side_bc: boundary kind of the six domain sides (-x, +x, -y, +y, -z, +z);
    refine(level, lo, hi) -> bool decides whether a cube at `level` spanning [lo, hi] is split
    (applied level by level up to max_level), after which cubes are split further until no two
    face neighbours differ by more than one level.
    """
    nx, ny, nz = (int(v) for v in base_dims)
    lo0 = np.asarray(domain_lo, dtype=np.float64)
    dims = np.array([nx, ny, nz])
    leaves = {(0, i, j, k) for k in range(nz) for j in range(ny) for i in range(nx)}

    def box(key):
        lv, i, j, k = key
        e = root_edge / 2 ** lv
        lo = lo0 + e * np.array([i, j, k], dtype=np.float64)
        return lo, lo + e

    def split(key):
        lv, i, j, k = key
        leaves.discard(key)
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    leaves.add((lv + 1, 2 * i + dx, 2 * j + dy, 2 * k + dz))

    if refine is not None:
        for lv in range(max_level):
            for key in sorted(k for k in leaves if k[0] == lv):
                lo, hi = box(key)
                if refine(lv, lo, hi):
                    split(key)

    def inside(lv, c):
        ext = dims * 2 ** lv
        return all(0 <= c[a] < ext[a] for a in range(3))

    # 2:1 face balance: a leaf with a face neighbour two or more levels finer is split.
    changed = True
    while changed:
        changed = False
        for key in sorted(leaves):
            if key not in leaves:
                continue
            lv = key[0]
            for f in range(6):
                ax, sd = divmod(f, 2)
                c = list(key[1:])
                c[ax] += 1 if sd else -1
                if not inside(lv, c) or (lv, *c) in leaves:
                    continue
                if lv > 0 and (lv - 1, c[0] >> 1, c[1] >> 1, c[2] >> 1) in leaves:
                    continue
                # the neighbour region is refined: its children facing us must all be leaves
                ok = True
                for q in range(4):
                    ch = [2 * v for v in c]
                    ch[ax] += 0 if sd else 1
                    t1, t2 = _tangential(ax)
                    ch[t1] += q & 1
                    ch[t2] += q >> 1
                    if (lv + 1, *ch) not in leaves:
                        ok = False
                        break
                if not ok:
                    split(key)
                    changed = True
                    break

    keys = sorted(leaves)
    top = max(k[0] for k in keys)
    fine = np.array([[v << (top - k[0]) for v in k[1:]] for k in keys], dtype=np.int64)
    order = np.argsort(morton3(fine[:, 0], fine[:, 1], fine[:, 2]), kind="stable")
    keys = [keys[o] for o in order]
    ids = {k: t for t, k in enumerate(keys)}
    n_c = len(keys)
    origin = np.zeros((n_c, 3))
    level = np.zeros(n_c, dtype=np.int8)
    nbr = -np.ones((n_c, 6, 4), dtype=np.int32)
    face_bc = np.zeros((n_c, 6), dtype=np.int8)
    for t, key in enumerate(keys):
        lv = key[0]
        level[t] = lv
        origin[t] = box(key)[0]
        for f in range(6):
            ax, sd = divmod(f, 2)
            c = list(key[1:])
            c[ax] += 1 if sd else -1
            if not inside(lv, c):
                face_bc[t, f] = _bc_code(side_bc[f])
                continue
            if (lv, *c) in ids:
                nbr[t, f, 0] = ids[(lv, *c)]
                continue
            par = (lv - 1, c[0] >> 1, c[1] >> 1, c[2] >> 1)
            if lv > 0 and par in ids:
                nbr[t, f, 0] = ids[par]
                continue
            t1, t2 = _tangential(ax)
            for q in range(4):
                ch = [2 * v for v in c]
                ch[ax] += 0 if sd else 1
                ch[t1] += q & 1
                ch[t2] += q >> 1
                nbr[t, f, q] = ids[(lv + 1, *ch)]
    hi = tuple(float(v) for v in lo0 + root_edge * dims)
    return Mesh(n, float(root_edge), origin, level, nbr, face_bc, tuple(lo0.tolist()), hi,
                meta={"base_dims": (nx, ny, nz), "side_bc": list(side_bc)})


def uniform_mesh(dims, edge, n, side_bc, domain_lo=(0.0, 0.0, 0.0)) -> Mesh:
    """dims[0] x dims[1] x dims[2] equal cubes of the given edge (one level)."""
    return build_mesh(dims, edge, n, side_bc, domain_lo=domain_lo)


CHANNEL_BC = ("inflow", "outflow", "slip", "slip", "slip", "slip")
OPEN_BC = ("outflow",) * 6
