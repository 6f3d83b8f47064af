// Multigrid hierarchy of the cube graph (host only).
//
// Below the per-cube levels the Poisson problem lives on the one-cell-per-cube graph: one
// unknown per cube, 7-point couplings with the same 2:1 interface rules as the cell level.
// The paper solves that level with a few CG iterations (Sec. 7); on meshes of thousands of
// cubes that leaves the smoothest modes unresolved, so here the graph itself is coarsened:
//   1. octree merging: the cubes of the finest level (they always come as 8 siblings in a
//      2:1-balanced mesh) become their parent, until every node is a level-0 cube;
//   2. lattice merging: 2x2x2 blocks of level-0 cubes while every lattice dimension is even.
// Each graph level is re-discretised with the composite rules (same-level 1, fine side 2/3,
// coarse side 4/3 of the mean of the four fine neighbours, open boundary 2, Neumann 0), gets
// a greedy colouring for Gauss-Seidel, and a child list for restriction (volume-weighted
// mean) and prolongation (piecewise constant).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <set>
#include <tuple>
#include <unordered_map>

#include "bcm_internal.hpp"
#include "coarse.hpp"

namespace bcm {

namespace {

struct Key {
  int l, i, j, k;
  bool operator==(const Key& o) const { return l == o.l && i == o.i && j == o.j && k == o.k; }
};
struct KeyHash {
  size_t operator()(const Key& a) const {
    uint64_t h = uint64_t(a.l) * 0x9E3779B97F4A7C15ull;
    h ^= uint64_t(uint32_t(a.i)) + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    h ^= uint64_t(uint32_t(a.j)) + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    h ^= uint64_t(uint32_t(a.k)) + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    return size_t(h);
  }
};

int tang(int d, int w) {
  static const int t[3][2] = {{1, 2}, {0, 2}, {0, 1}};
  return t[d][w];
}

// Build the operator rows, colouring and child lists of one graph level.
void build_level(CoarseLevel& L, const std::vector<Key>& keys, const int dims[3], double root_edge,
                 const int side_kind[6]) {
  const int n = int(keys.size());
  std::unordered_map<Key, int, KeyHash> id;
  id.reserve(n * 2);
  for (int t = 0; t < n; ++t) id[keys[t]] = t;
  L.n = n;
  L.row.assign(1, 0);
  L.col.clear();
  L.val.clear();
  L.diag.assign(n, 0.0);
  L.vol.assign(n, 0.0);
  std::vector<std::vector<int>> adj(n);
  int maxl = 0;
  for (const Key& k : keys) maxl = std::max(maxl, k.l);
  for (int t = 0; t < n; ++t) {
    const Key& K = keys[t];
    const double h = root_edge / std::ldexp(1.0, K.l);
    const double ih2 = 1.0 / (h * h);
    L.vol[t] = std::ldexp(1.0, 3 * (maxl - K.l));
    double own = 0.0;
    for (int f = 0; f < 6; ++f) {
      const int d = f >> 1, s = f & 1;
      int c[3] = {K.i, K.j, K.k};
      c[d] += s ? 1 : -1;
      const int ext = dims[d] << K.l;
      if (c[d] < 0 || c[d] >= ext) {
        own += side_kind[f] == FK_OUTFLOW ? 2.0 : 0.0;
        continue;
      }
      auto it = id.find(Key{K.l, c[0], c[1], c[2]});
      if (it != id.end()) {
        L.col.push_back(it->second);
        L.val.push_back(ih2);
        adj[t].push_back(it->second);
        own += 1.0;
        continue;
      }
      if (K.l > 0) {
        auto ip = id.find(Key{K.l - 1, c[0] >> 1, c[1] >> 1, c[2] >> 1});
        if (ip != id.end()) {
          L.col.push_back(ip->second);
          L.val.push_back(2.0 / 3.0 * ih2);
          adj[t].push_back(ip->second);
          own += 2.0 / 3.0;
          continue;
        }
      }
      for (int q = 0; q < 4; ++q) {
        int ch[3] = {2 * c[0], 2 * c[1], 2 * c[2]};
        ch[d] += s ? 0 : 1;
        ch[tang(d, 0)] += q & 1;
        ch[tang(d, 1)] += q >> 1;
        auto is = id.find(Key{K.l + 1, ch[0], ch[1], ch[2]});
        if (is == id.end()) continue;  // cannot happen on a 2:1-balanced graph
        L.col.push_back(is->second);
        L.val.push_back(4.0 / 3.0 * 0.25 * ih2);
        adj[t].push_back(is->second);
      }
      own += 4.0 / 3.0;
    }
    L.diag[t] = -own * ih2;
    L.row.push_back(int(L.col.size()));
  }
  // greedy colouring in key order (a lattice gets the red-black parity colouring)
  std::vector<int> colour(n, -1);
  int ncol = 0;
  for (int t = 0; t < n; ++t) {
    uint64_t used = 0;
    for (int o : adj[t])
      if (colour[o] >= 0 && colour[o] < 64) used |= 1ull << colour[o];
    int c = 0;
    while (used & (1ull << c)) ++c;
    colour[t] = c;
    ncol = std::max(ncol, c + 1);
  }
  if (ncol > 2) {
    // not bipartite (2:1 interfaces): try saturation-degree order (DSATUR), which usually
    // needs fewer colours, i.e. fewer multi-workgroup launches per sweep
    std::vector<int> dcol(n, -1), deg(n);
    std::vector<uint64_t> sat(n, 0);
    std::set<std::tuple<int, int, int>> pq;  // (saturation, degree, node), largest first
    for (int t = 0; t < n; ++t) {
      deg[t] = int(adj[t].size());
      pq.insert({0, deg[t], t});
    }
    int dn = 0;
    while (!pq.empty()) {
      const int t = std::get<2>(*std::prev(pq.end()));
      pq.erase(std::prev(pq.end()));
      int c = 0;
      while (c < 64 && (sat[t] >> c & 1)) ++c;
      dcol[t] = c;
      dn = std::max(dn, c + 1);
      for (int o : adj[t]) {
        if (dcol[o] >= 0 || c >= 64 || (sat[o] >> c & 1)) continue;
        pq.erase({__builtin_popcountll(sat[o]), deg[o], o});
        sat[o] |= 1ull << c;
        pq.insert({__builtin_popcountll(sat[o]), deg[o], o});
      }
    }
    if (dn < ncol) {
      colour = dcol;
      ncol = dn;
    }
  }
  L.order.clear();
  L.color_off.assign(1, 0);
  for (int c = 0; c < ncol; ++c) {
    for (int t = 0; t < n; ++t)
      if (colour[t] == c) L.order.push_back(t);
    L.color_off.push_back(int(L.order.size()));
  }
}

}  // namespace

// Inverse of the operator of a small level in its device node order (row i: diag_i x_i +
// sum_w val_wi x_col_wi), stored transposed (inv[j * n + i] = (M^-1)_ij) so that the lanes
// that compute consecutive rows read consecutive values.  Gauss-Jordan with partial
// pivoting; empty when the level is too large or the operator is numerically singular.
static std::vector<double> dense_inverse_transposed(const CoarseLevel& L) {
  const int n = L.n;
  if (n <= 0 || n > kBottomDirectMax) return {};
  std::vector<double> a(size_t(n) * n, 0.0), inv(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) {
    a[size_t(i) * n + i] += L.e_diag[i];
    for (int w = 0; w < L.W; ++w) a[size_t(i) * n + L.e_col[size_t(w) * n + i]] += L.e_val[size_t(w) * n + i];
    inv[size_t(i) * n + i] = 1.0;
  }
  double scale = 0.0;
  for (double v : a) scale = std::max(scale, std::fabs(v));
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[size_t(r) * n + c]) > std::fabs(a[size_t(piv) * n + c])) piv = r;
    if (!(std::fabs(a[size_t(piv) * n + c]) > 1e-12 * scale)) return {};
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(a[size_t(piv) * n + k], a[size_t(c) * n + k]);
        std::swap(inv[size_t(piv) * n + k], inv[size_t(c) * n + k]);
      }
    const double d = 1.0 / a[size_t(c) * n + c];
    for (int k = 0; k < n; ++k) {
      a[size_t(c) * n + k] *= d;
      inv[size_t(c) * n + k] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = a[size_t(r) * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        a[size_t(r) * n + k] -= f * a[size_t(c) * n + k];
        inv[size_t(r) * n + k] -= f * inv[size_t(c) * n + k];
      }
    }
  }
  std::vector<double> t(size_t(n) * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) t[size_t(j) * n + i] = inv[size_t(i) * n + j];
  return t;
}

bool build_coarse_hierarchy(const HostMesh& M, CoarseHierarchy& H, int max_levels) {
  H.levels.clear();
  H.ok = false;
  const int nc = M.n_cubes;
  // integer keys of the cubes and the level-0 lattice they tile
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int c = 0; c < nc; ++c)
    for (int d = 0; d < 3; ++d) {
      const double e = M.root_edge / std::ldexp(1.0, M.level[c]);
      lo[d] = std::min(lo[d], M.origin[3 * c + d]);
      hi[d] = std::max(hi[d], M.origin[3 * c + d] + e);
    }
  int dims[3];
  for (int d = 0; d < 3; ++d) dims[d] = int(std::lround((hi[d] - lo[d]) / M.root_edge));
  std::vector<Key> keys(nc);
  double vol = 0.0;
  for (int c = 0; c < nc; ++c) {
    const double e = M.root_edge / std::ldexp(1.0, M.level[c]);
    int v[3];
    for (int d = 0; d < 3; ++d) v[d] = int(std::lround((M.origin[3 * c + d] - lo[d]) / e));
    keys[c] = Key{M.level[c], v[0], v[1], v[2]};
    vol += e * e * e;
  }
  // only box domains (the level-0 lattice fully covered) get the hierarchy
  if (std::fabs(vol - double(dims[0]) * dims[1] * dims[2] * std::pow(M.root_edge, 3)) >
      1e-9 * vol)
    return false;
  // boundary kind of each domain side: open if any cube face on it is open
  int side_kind[6] = {FK_SLIP, FK_SLIP, FK_SLIP, FK_SLIP, FK_SLIP, FK_SLIP};
  for (int c = 0; c < nc; ++c)
    for (int f = 0; f < 6; ++f) {
      const int k = M.meta[c].kind[f];
      if (k == FK_OUTFLOW) side_kind[f] = FK_OUTFLOW;
      else if (k == FK_INFLOW && side_kind[f] != FK_OUTFLOW) side_kind[f] = FK_INFLOW;
    }
  double root = M.root_edge;
  int gd[3] = {dims[0], dims[1], dims[2]};
  std::vector<Key> cur = keys;
  H.levels.emplace_back();
  build_level(H.levels.back(), cur, gd, root, side_kind);
  while (int(H.levels.size()) < max_levels && cur.size() > 64) {
    int maxl = 0;
    for (const Key& k : cur) maxl = std::max(maxl, k.l);
    std::vector<Key> next;
    std::vector<int> parent(cur.size());
    std::unordered_map<Key, int, KeyHash> pid;
    if (maxl > 0) {
      for (size_t t = 0; t < cur.size(); ++t) {
        Key p = cur[t];
        if (p.l == maxl) p = Key{p.l - 1, p.i >> 1, p.j >> 1, p.k >> 1};
        auto it = pid.find(p);
        if (it == pid.end()) {
          pid[p] = int(next.size());
          parent[t] = int(next.size());
          next.push_back(p);
        } else {
          parent[t] = it->second;
        }
      }
    } else {
      if ((gd[0] & 1) || (gd[1] & 1) || (gd[2] & 1)) break;
      for (int d = 0; d < 3; ++d) gd[d] >>= 1;
      root *= 2.0;
      for (size_t t = 0; t < cur.size(); ++t) {
        Key p{0, cur[t].i >> 1, cur[t].j >> 1, cur[t].k >> 1};
        auto it = pid.find(p);
        if (it == pid.end()) {
          pid[p] = int(next.size());
          parent[t] = int(next.size());
          next.push_back(p);
        } else {
          parent[t] = it->second;
        }
      }
    }
    // order the coarse nodes along the Z curve of their keys for locality
    H.levels.emplace_back();
    CoarseLevel& C = H.levels.back();
    build_level(C, next, gd, root, side_kind);
    CoarseLevel& F = H.levels[H.levels.size() - 2];
    F.parent = parent;
    C.child_row.assign(C.n + 1, 0);
    for (int p : parent) C.child_row[p + 1]++;
    for (int t = 0; t < C.n; ++t) C.child_row[t + 1] += C.child_row[t];
    C.child.assign(parent.size(), 0);
    C.child_w.assign(parent.size(), 0.0);
    std::vector<int> fill(C.child_row.begin(), C.child_row.end() - 1);
    for (size_t t = 0; t < parent.size(); ++t) {
      const int p = parent[t];
      C.child[fill[p]] = int(t);
      C.child_w[fill[p]] = F.vol[t] / (C.vol[p] * (maxl > 0 ? 1.0 : 1.0));
      fill[p]++;
    }
    // volume-weighted mean: weights of each parent sum to one
    for (int p = 0; p < C.n; ++p) {
      double s = 0.0;
      for (int e = C.child_row[p]; e < C.child_row[p + 1]; ++e) s += C.child_w[e];
      for (int e = C.child_row[p]; e < C.child_row[p + 1]; ++e) C.child_w[e] /= s;
    }
    cur.swap(next);
  }
  // device form: renumber every level so that each colour is a contiguous node range,
  // then store couplings and child lists as column-major ELL arrays
  std::vector<std::vector<int32_t>> newid(H.levels.size());
  for (size_t g = 0; g < H.levels.size(); ++g) {
    const CoarseLevel& L = H.levels[g];
    newid[g].assign(L.n, 0);
    for (int p = 0; p < L.n; ++p) newid[g][L.order[p]] = p;
  }
  for (size_t g = 0; g < H.levels.size(); ++g) {
    CoarseLevel& L = H.levels[g];
    const std::vector<int32_t>& id = newid[g];
    const int n = L.n;
    int W = 1;
    for (int t = 0; t < n; ++t) W = std::max(W, L.row[t + 1] - L.row[t]);
    L.W = W;
    L.e_col.assign(size_t(W) * n, 0);
    L.e_val.assign(size_t(W) * n, 0.0);
    L.e_diag.assign(n, 0.0);
    L.e_vol.assign(n, 0.0);
    for (int t = 0; t < n; ++t) {
      const int p = id[t];
      L.e_diag[p] = L.diag[t];
      L.e_vol[p] = L.vol[t];
      int w = 0;
      for (int e = L.row[t]; e < L.row[t + 1]; ++e, ++w) {
        L.e_col[size_t(w) * n + p] = id[L.col[e]];
        L.e_val[size_t(w) * n + p] = L.val[e];
      }
      for (; w < W; ++w) L.e_col[size_t(w) * n + p] = p;
    }
    // packed rows: 6 columns as 16-bit indices when every coupling of the level has one value
    L.uval = 0.0;
    L.e_pcol.clear();
    bool uniform = W == 6 && n <= 65535 && !L.val.empty();
    for (size_t e = 0; uniform && e < L.val.size(); ++e) uniform = L.val[e] == L.val[0];
    if (uniform) {
      L.uval = L.val[0];
      L.e_pcol.assign(size_t(3) * n, 0u);
      for (int q = 0; q < 3; ++q)
        for (int p = 0; p < n; ++p)
          L.e_pcol[size_t(q) * n + p] = uint32_t(L.e_col[size_t(2 * q) * n + p]) |
                                        uint32_t(L.e_col[size_t(2 * q + 1) * n + p]) << 16;
    }
    if (!L.parent.empty()) {
      const std::vector<int32_t>& idc = newid[g + 1];
      L.e_parent.assign(n, 0);
      for (int t = 0; t < n; ++t) L.e_parent[id[t]] = idc[L.parent[t]];
    }
    if (g > 0) {
      const std::vector<int32_t>& idf = newid[g - 1];
      int CW = 1;
      for (int t = 0; t < n; ++t) CW = std::max(CW, L.child_row[t + 1] - L.child_row[t]);
      L.CW = CW;
      L.e_child.assign(size_t(CW) * n, -1);
      L.e_child_w.assign(size_t(CW) * n, 0.0);
      for (int t = 0; t < n; ++t) {
        const int p = id[t];
        int w = 0;
        for (int e = L.child_row[t]; e < L.child_row[t + 1]; ++e, ++w) {
          L.e_child[size_t(w) * n + p] = idf[L.child[e]];
          L.e_child_w[size_t(w) * n + p] = L.child_w[e];
        }
      }
    }
    if (g == 0) L.perm = id;
  }
  H.bottom_inv = dense_inverse_transposed(H.levels.back());
  H.ok = true;
  return true;
}

}  // namespace bcm
