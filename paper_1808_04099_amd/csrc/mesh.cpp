// Mesh ingest (host only): validation of the building-cube description, per-cube device
// metadata and the workgroup launch order.
//
// The mesh is the paper's linear-array representation (Sec. 2.2): base corners, levels,
// equal cell counts and a neighbour adjacency table; cubes are visited along a Z-order
// space-filling curve (Sec. 6.1) so that neighbouring cubes run close together in time.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>

#include "bcm_internal.hpp"

namespace bcm {

namespace {

thread_local std::string g_last_error;

bool fail(const char* fmt, int c, int f, const char* extra = "") {
  char buf[256];
  std::snprintf(buf, sizeof(buf), fmt, c, f, extra);
  g_last_error = buf;
  return false;
}

int tangential(int d, int which) {  // tangential axes of axis d in increasing order
  static const int t[3][2] = {{1, 2}, {0, 2}, {0, 1}};
  return t[d][which];
}

uint64_t spread3(uint64_t v) {
  uint64_t r = 0;
  for (int b = 0; b < 21; ++b) r |= ((v >> b) & 1ull) << (3 * b);
  return r;
}

// Geometry behind the boundary faces: a face whose four neighbour slots are empty must lie on
// the domain boundary, i.e. no cube of any level may touch it from the outside (otherwise the
// solver would apply a boundary rule where the geometry has a neighbour).  Cubes are hashed by
// (level, integer position on the lattice of their level), anchored at the minimum corner of
// the coarsest level present; every cube must sit on its level's lattice.  For each boundary
// face the lookups are: the same-level cube across it, every coarser cube that would contain
// the cell just across it, and the four cubes one level finer that would cover it (a mesh that
// passed the link checks has no face neighbours two or more levels apart).
bool check_boundary_faces(const HostMesh& M) {
  const int nc = M.n_cubes;
  if (nc == 0) return true;
  int lmin = 127, lmax = 0;
  for (int c = 0; c < nc; ++c) {
    lmin = std::min<int>(lmin, M.level[c]);
    lmax = std::max<int>(lmax, M.level[c]);
  }
  double anchor[3] = {HUGE_VAL, HUGE_VAL, HUGE_VAL};
  for (int c = 0; c < nc; ++c)
    if (M.level[c] == lmin)
      for (int d = 0; d < 3; ++d) anchor[d] = std::min(anchor[d], M.origin[3 * c + d]);
  using Key = std::array<int64_t, 4>;  // level, x, y, z
  std::vector<Key> keys(nc);
  std::vector<int64_t> pos(3 * size_t(nc));
  for (int c = 0; c < nc; ++c) {
    const double e = M.root_edge / std::ldexp(1.0, M.level[c]);
    for (int d = 0; d < 3; ++d) {
      const double off = (M.origin[3 * c + d] - anchor[d]) / e;
      const double r = std::round(off);
      if (std::fabs(off - r) > 1e-6 || std::fabs(r) > 1e15)
        return fail("cube %d: base corner is not on the lattice of its level (axis %d)%s", c, d);
      pos[3 * size_t(c) + d] = int64_t(r);
    }
    keys[c] = Key{M.level[c], pos[3 * size_t(c)], pos[3 * size_t(c) + 1], pos[3 * size_t(c) + 2]};
  }
  std::vector<Key> sorted(keys);
  std::sort(sorted.begin(), sorted.end());
  for (size_t i = 1; i < sorted.size(); ++i)
    if (sorted[i] == sorted[i - 1]) {
      const int c = int(std::find(keys.begin(), keys.end(), sorted[i]) - keys.begin());
      return fail("cube %d: another cube of the same level has the same position%.0d%s", c, 0);
    }
  auto exists = [&](int lv, int64_t x, int64_t y, int64_t z) {
    if (lv < lmin || lv > lmax) return false;
    return std::binary_search(sorted.begin(), sorted.end(), Key{lv, x, y, z});
  };
  for (int c = 0; c < nc; ++c) {
    const int lv = M.level[c];
    const int64_t* p = &pos[3 * size_t(c)];
    for (int f = 0; f < 6; ++f) {
      const int* s = &M.nbr[(size_t(c) * 6 + f) * 4];
      if (s[0] >= 0 || s[1] >= 0 || s[2] >= 0 || s[3] >= 0) continue;
      const int d = f >> 1, side = f & 1;
      int64_t q[3] = {p[0], p[1], p[2]};
      q[d] += side ? 1 : -1;  // same-level position across the face
      bool hit = exists(lv, q[0], q[1], q[2]);
      for (int L = lv - 1; L >= lmin && !hit; --L) {  // coarser cubes containing that cell
        const int sh = lv - L;
        hit = exists(L, q[0] >> sh, q[1] >> sh, q[2] >> sh);
      }
      for (int w = 0; w < 4 && !hit; ++w) {  // one level finer: the four cubes covering the face
        int64_t r[3] = {2 * p[0], 2 * p[1], 2 * p[2]};
        r[d] += side ? 2 : -1;
        r[tangential(d, 0)] += w & 1;
        r[tangential(d, 1)] += w >> 1;
        hit = exists(lv + 1, r[0], r[1], r[2]);
      }
      if (hit) return fail("cube %d face %d: marked as a domain boundary, but a cube lies across it%s", c, f);
    }
  }
  return true;
}

bool validate(HostMesh& M) {
  const int nc = M.n_cubes;
  const double tol = 1e-9 * M.root_edge;
  auto edge = [&](int c) { return M.root_edge / std::ldexp(1.0, M.level[c]); };
  auto org = [&](int c, int d) { return M.origin[3 * c + d]; };
  auto nb = [&](int c, int f, int s) { return M.nbr[(c * 6 + f) * 4 + s]; };
  bool any_outflow = false;
  for (int c = 0; c < nc; ++c) {
    if (M.level[c] < 0 || M.level[c] > 20) return fail("cube %d: level out of range%.0d%s", c, 0);
    for (int d = 0; d < 3; ++d)
      if (!std::isfinite(org(c, d))) return fail("cube %d: non-finite origin%.0d%s", c, 0);
  }
  for (int c = 0; c < nc; ++c) {
    for (int f = 0; f < 6; ++f) {
      const int d = f >> 1, side = f & 1, of = f ^ 1;
      int s[4];
      for (int q = 0; q < 4; ++q) {
        s[q] = nb(c, f, q);
        if (s[q] < -1 || s[q] >= nc) return fail("cube %d face %d: neighbour index out of range%s", c, f);
        if (s[q] == c) return fail("cube %d face %d: cube is its own neighbour%s", c, f);
      }
      const int bc = M.face_bc[c * 6 + f];
      const bool none = s[0] < 0 && s[1] < 0 && s[2] < 0 && s[3] < 0;
      const bool one = s[0] >= 0 && s[1] < 0 && s[2] < 0 && s[3] < 0;
      const bool four = s[0] >= 0 && s[1] >= 0 && s[2] >= 0 && s[3] >= 0;
      if (none) {
        if (bc != BCM_BC_OUTFLOW && bc != BCM_BC_INFLOW && bc != BCM_BC_SLIP)
          return fail("cube %d face %d: boundary face without a boundary kind%s", c, f);
        if (bc == BCM_BC_OUTFLOW) any_outflow = true;
        if (bc == BCM_BC_INFLOW) M.has_inflow = true;
        continue;
      }
      if (bc != BCM_BC_NONE) return fail("cube %d face %d: interior face has a boundary kind%s", c, f);
      const double e = edge(c);
      if (one) {
        const int o = s[0];
        const double eo = edge(o);
        // the neighbour must touch this face from the outside
        const double gap = side ? org(o, d) - (org(c, d) + e) : org(c, d) - (org(o, d) + eo);
        if (std::fabs(gap) > tol) return fail("cube %d face %d: neighbour does not touch the face%s", c, f);
        if (M.level[o] == M.level[c]) {
          for (int w = 0; w < 2; ++w) {
            const int t = tangential(d, w);
            if (std::fabs(org(o, t) - org(c, t)) > tol)
              return fail("cube %d face %d: same-level neighbour is not aligned%s", c, f);
          }
          if (!(nb(o, of, 0) == c && nb(o, of, 1) < 0))
            return fail("cube %d face %d: neighbour link is not reciprocal%s", c, f);
        } else if (M.level[o] == M.level[c] - 1) {
          int q = 0;
          for (int w = 0; w < 2; ++w) {
            const int t = tangential(d, w);
            const double off = (org(c, t) - org(o, t)) / e;
            const double r = std::round(off);
            if (std::fabs(off - r) > 1e-9 || (r != 0.0 && r != 1.0))
              return fail("cube %d face %d: finer cube is not a quadrant of its coarse neighbour%s", c, f);
            q |= int(r) << w;
          }
          if (nb(o, of, q) != c)
            return fail("cube %d face %d: coarse neighbour does not list this cube in its slot%s", c, f);
        } else {
          return fail("cube %d face %d: neighbour differs by more than one level (or is finer in slot 0 only)%s", c, f);
        }
        continue;
      }
      if (four) {
        for (int q = 0; q < 4; ++q) {
          const int o = s[q];
          if (M.level[o] != M.level[c] + 1)
            return fail("cube %d face %d: sub-neighbour is not one level finer%s", c, f);
          if (!(nb(o, of, 0) == c && nb(o, of, 1) < 0))
            return fail("cube %d face %d: sub-neighbour link is not reciprocal%s", c, f);
          for (int w = 0; w < 2; ++w) {
            const int t = tangential(d, w);
            const double want = org(c, t) + ((q >> w) & 1) * 0.5 * e;
            if (std::fabs(org(o, t) - want) > tol)
              return fail("cube %d face %d: sub-neighbour slot does not match its position%s", c, f);
          }
        }
        continue;
      }
      return fail("cube %d face %d: neighbour slots must hold 0, 1 or 4 cubes%s", c, f);
    }
  }
  if (!any_outflow) {
    g_last_error = "mesh has no BCM_BC_OUTFLOW face: the Poisson problem would be singular";
    return false;
  }
  return check_boundary_faces(M);
}

void derive(HostMesh& M) {
  const int nc = M.n_cubes;
  M.max_level = 0;
  for (int c = 0; c < nc; ++c) M.max_level = std::max<int>(M.max_level, M.level[c]);
  M.multilevel = false;
  M.meta.assign(nc, CubeMeta{});
  for (int c = 0; c < nc; ++c) {
    CubeMeta& m = M.meta[c];
    std::memset(&m, 0, sizeof(m));
    const double e = M.root_edge / std::ldexp(1.0, M.level[c]);
    m.level = M.level[c];
    m.h = e / M.n;
    m.vol = std::ldexp(1.0, 3 * (M.max_level - M.level[c]));
    for (int f = 0; f < 6; ++f) {
      for (int q = 0; q < 4; ++q) m.nbr[f][q] = M.nbr[(c * 6 + f) * 4 + q];
      const int o = m.nbr[f][0];
      if (o < 0) {
        const int bc = M.face_bc[c * 6 + f];
        m.kind[f] = bc == BCM_BC_OUTFLOW ? FK_OUTFLOW : bc == BCM_BC_INFLOW ? FK_INFLOW : FK_SLIP;
      } else if (m.nbr[f][1] >= 0) {
        m.kind[f] = FK_FINER;
        M.multilevel = true;
      } else if (M.level[o] < M.level[c]) {
        m.kind[f] = FK_COARSER;
        M.multilevel = true;
        const int d = f >> 1;
        int q = 0;
        for (int w = 0; w < 2; ++w) {
          const int t = tangential(d, w);
          const double off = (M.origin[3 * c + t] - M.origin[3 * o + t]) / e;
          q |= int(std::lround(off)) << w;
        }
        m.quad[f] = int8_t(q);
      } else {
        m.kind[f] = FK_SAME;
      }
    }
  }
  // Z-order of the cube base corners on the finest level's grid, then an XCD-aware
  // interleave: workgroup w is dispatched to XCD w % 8, so XCD x receives the x-th
  // contiguous chunk of the curve and neighbouring cubes share that XCD's L2.
  double lo[3] = {1e300, 1e300, 1e300};
  for (int c = 0; c < nc; ++c)
    for (int d = 0; d < 3; ++d) lo[d] = std::min(lo[d], M.origin[3 * c + d]);
  const double ef = M.root_edge / std::ldexp(1.0, M.max_level);
  std::vector<uint64_t> key(nc);
  for (int c = 0; c < nc; ++c) {
    uint64_t k = 0;
    for (int d = 0; d < 3; ++d) {
      const uint64_t v = uint64_t(std::llround((M.origin[3 * c + d] - lo[d]) / ef));
      k |= spread3(v) << d;
    }
    key[c] = k;
  }
  std::vector<int32_t> order(nc);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key[a] < key[b]; });
  const int X = 8;
  const int chunk = (nc + X - 1) / X;
  M.launch.clear();
  M.launch.reserve(nc);
  for (int i = 0; i < chunk; ++i)
    for (int x = 0; x < X; ++x) {
      const int p = x * chunk + i;
      if (p < nc) M.launch.push_back(order[p]);
    }
  // 27-neighbourhoods for the trilinear prolongation (single-level meshes)
  M.nb27.clear();
  if (!M.multilevel && nc < kNb27MaxCubes) {
    M.nb27.resize(size_t(nc) * 27);
    for (int p = 0; p < nc; ++p)
      for (int e = 0; e < 27; ++e) {
        const int d[3] = {e % 3 - 1, (e / 3) % 3 - 1, e / 9 - 1};
        int c = M.launch[p], clamped = 0;
        bool neg = false;
        for (int a = 0; a < 3; ++a) {
          if (d[a] == 0) continue;
          const int f = 2 * a + (d[a] > 0);
          const CubeMeta& m = M.meta[c];
          if (m.kind[f] == FK_SAME) {
            c = m.nbr[f][0];
          } else {
            clamped |= 1 << a;
            neg ^= m.kind[f] == FK_OUTFLOW;
          }
        }
        M.nb27[size_t(p) * 27 + e] = pack_nb27(c, clamped, neg);
      }
  }
  build_coarse_hierarchy(M, M.coarse, kMaxGraphLevels);
  for (const CoarseLevel& L : M.coarse.levels)
    if (int(L.color_off.size()) - 1 > 8) M.coarse.ok = false;  // device keeps 8 colours
}

}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }
const char* last_error() { return g_last_error.c_str(); }

}  // namespace bcm

extern "C" {

int bcm_mesh_create(const bcm_mesh_desc* desc, bcm_mesh** out) {
  if (!desc || !out || !desc->origin || !desc->level || !desc->nbr || !desc->face_bc) {
    bcm::set_error("bcm_mesh_create: NULL argument");
    return BCM_ERR_INVALID_ARG;
  }
  *out = nullptr;
  const int n = desc->n;
  if (desc->n_cubes <= 0 || !(n == 2 || n == 4 || n == 8 || n == 16)) {
    bcm::set_error("bcm_mesh_create: n_cubes must be > 0 and n one of 2, 4, 8, 16");
    return BCM_ERR_INVALID_ARG;
  }
  if (!(desc->root_edge > 0.0) || !std::isfinite(desc->root_edge)) {
    bcm::set_error("bcm_mesh_create: root_edge must be positive and finite");
    return BCM_ERR_INVALID_ARG;
  }
  auto* mesh = new (std::nothrow) bcm_mesh;
  if (!mesh) {
    bcm::set_error("bcm_mesh_create: out of host memory");
    return BCM_ERR_INVALID_ARG;
  }
  bcm::HostMesh& M = mesh->m;
  const size_t nc = size_t(desc->n_cubes);
  M.n_cubes = desc->n_cubes;
  M.n = n;
  M.root_edge = desc->root_edge;
  M.origin.assign(desc->origin, desc->origin + 3 * nc);
  M.level.assign(desc->level, desc->level + nc);
  M.nbr.assign(desc->nbr, desc->nbr + 24 * nc);
  M.face_bc.assign(desc->face_bc, desc->face_bc + 6 * nc);
  if (!bcm::validate(M)) {
    delete mesh;
    return BCM_ERR_INVALID_MESH;
  }
  bcm::derive(M);
  *out = mesh;
  return BCM_OK;
}

void bcm_mesh_destroy(bcm_mesh* mesh) { delete mesh; }

int64_t bcm_mesh_cells(const bcm_mesh* mesh) {
  if (!mesh) return 0;
  return int64_t(mesh->m.n_cubes) * mesh->m.n * mesh->m.n * mesh->m.n;
}

const char* bcm_last_error(void) { return bcm::last_error(); }

const char* bcm_status_string(int s) {
  switch (s) {
    case BCM_OK: return "BCM_OK";
    case BCM_NOT_CONVERGED: return "BCM_NOT_CONVERGED";
    case BCM_STAGNATED: return "BCM_STAGNATED";
    case BCM_ERR_INVALID_ARG: return "BCM_ERR_INVALID_ARG";
    case BCM_ERR_INVALID_MESH: return "BCM_ERR_INVALID_MESH";
    case BCM_ERR_WORKSPACE: return "BCM_ERR_WORKSPACE";
    case BCM_ERR_NONFINITE: return "BCM_ERR_NONFINITE";
    case BCM_ERR_HIP: return "BCM_ERR_HIP";
    case BCM_ERR_UNSUPPORTED: return "BCM_ERR_UNSUPPORTED";
    default: return "BCM_UNKNOWN_STATUS";
  }
}

}  // extern "C"
