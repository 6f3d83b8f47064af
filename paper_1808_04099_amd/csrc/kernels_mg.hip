// Multigrid and Krylov kernels of the pressure Poisson solve (Sec. 3): red-black Gauss-Seidel
// smoothing, residual + restriction, operator apply fused with the search-direction update,
// vector updates with fused norms, FP64 residual for iterative refinement, and the
// conjugate-gradient solve on the one-cell-per-cube level (Sec. 7: at most 10 iterations).
//
// One workgroup (256 lanes = 4 wave64) owns one 16^3 or 8^3 cube, or several smaller cubes,
// staged as an LDS tile with a one-cell halo (tile.hpp).  All sums are accumulated in FP64
// with a fixed reduction order: each workgroup writes one partial, k_finalize sums them.
#include "kernels.hpp"
#include "tile.hpp"

namespace bcm {

namespace {

// ------------------------------------------------------------------------------------------
// Red-black Gauss-Seidel smoothing inside each cube (halo frozen at launch: the sweep is
// Gauss-Seidel within a cube and Jacobi across cube faces).  Optionally starts from zero,
// optionally adds a piecewise-constant prolongation of a coarse correction first, and
// optionally accumulates <x, r_dot>_V and <x, q_dot>_V for the Krylov wrapper.
// ------------------------------------------------------------------------------------------
template <int NL, typename T>
__global__ __launch_bounds__(256) void k_smooth(SmoothArgs<T> a) {
  using L = Lv<NL>;
  constexpr int R = (L::CPB * L::N3 + WG - 1) / WG;
  __shared__ CubeMeta sm[L::CPB];
  __shared__ int cube[L::CPB];
  __shared__ T tile[L::CPB * L::TILE];
  __shared__ double red[8];
  load_meta<NL>(sm, cube, a.g.meta, a.g.launch, a.g.n_cubes);
  T bv[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int e = threadIdx.x + r * WG;
    bv[r] = T(0);
    if (e >= L::CPB * L::N3) continue;
    int s, i, j, k;
    cell_of<NL>(e, s, i, j, k);
    const int c = cube[s];
    if (c < 0) continue;
    const size_t g = (size_t)c * L::N3 + (e - s * L::N3);
    T v = a.zero_init ? T(0) : a.x[g];
    if (a.xc) {
      constexpr int NC = NL / 2;
      v += a.xc[(size_t)c * (NC * NC * NC) + ((k >> 1) * NC + (j >> 1)) * NC + (i >> 1)];
    }
    tile[s * L::TILE + ti<NL>(i, j, k)] = v;
    bv[r] = a.b[g];
  }
  if (a.xc)
    fill_halo<NL, RULE_P, T>(tile, sm, cube,
                             FaceGetProlong<NL, T>{a.zero_init ? nullptr : a.xf_in, a.xcf},
                             BcZero<T>{});
  else if (a.zero_init)
    zero_halo<NL, T>(tile, cube);
  else
    fill_halo<NL, RULE_P, T>(tile, sm, cube, FaceGet<NL, T>{a.xf_in}, BcZero<T>{});
  __syncthreads();
  for (int sw = 0; sw < a.sweeps; ++sw) {
    for (int col = 0; col < 2; ++col) {
      const int colour = col ^ a.black_first;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e = threadIdx.x + r * WG;
        if (e >= L::CPB * L::N3) continue;
        int s, i, j, k;
        cell_of<NL>(e, s, i, j, k);
        if (((i + j + k) & 1) != colour || cube[s] < 0) continue;
        const CubeMeta& m = sm[s];
        const T h = T(m.h * a.g.hscale);
        T nb, dg;
        stencil_p<NL, T>(tile + s * L::TILE, m, i, j, k, nb, dg);
        tile[s * L::TILE + ti<NL>(i, j, k)] = (nb - h * h * bv[r]) / dg;
      }
      __syncthreads();
    }
  }
  double zr = 0.0, zq = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int e = threadIdx.x + r * WG;
    if (e >= L::CPB * L::N3) continue;
    int s, i, j, k;
    cell_of<NL>(e, s, i, j, k);
    const int c = cube[s];
    if (c < 0) continue;
    const size_t g = (size_t)c * L::N3 + (e - s * L::N3);
    const T v = tile[s * L::TILE + ti<NL>(i, j, k)];
    a.x[g] = v;
    if (a.part_zr) {
      const double w = sm[s].vol;
      zr += w * double(v) * double(a.r_dot[g]);
      if (a.q_dot) zq += w * double(v) * double(a.q_dot[g]);
    }
  }
  export_faces<NL, T, T>(a.xf_out, tile, cube);
  if (a.part_zr) {
    const double t0 = block_sum(zr, red);
    __syncthreads();
    const double t1 = block_sum(zq, red);
    if (threadIdx.x == 0) {
      a.part_zr[blockIdx.x] = t0;
      if (a.part_zq) a.part_zq[blockIdx.x] = t1;
    }
  }
}

// Residual r = b - A x, restricted to the next level by the mean of the 8 children.
template <int NL, typename T>
__global__ __launch_bounds__(256) void k_restrict(RestrictArgs<T> a) {
  using L = Lv<NL>;
  constexpr int NC = NL / 2, NC3 = NC * NC * NC;
  __shared__ CubeMeta sm[L::CPB];
  __shared__ int cube[L::CPB];
  __shared__ T tile[L::CPB * L::TILE];
  load_meta<NL>(sm, cube, a.g.meta, a.g.launch, a.g.n_cubes);
  for (int e = threadIdx.x; e < L::CPB * L::N3; e += WG) {
    int s, i, j, k;
    cell_of<NL>(e, s, i, j, k);
    const int c = cube[s];
    if (c < 0) continue;
    tile[s * L::TILE + ti<NL>(i, j, k)] = a.x[(size_t)c * L::N3 + (e - s * L::N3)];
  }
  fill_halo<NL, RULE_P, T>(tile, sm, cube, FaceGet<NL, T>{a.xf}, BcZero<T>{});
  __syncthreads();
  for (int e = threadIdx.x; e < L::CPB * NC3; e += WG) {
    const int s = e / NC3;
    const int cc = e - s * NC3;
    const int c = cube[s];
    if (c < 0) continue;
    const int I = cc % NC, J = (cc / NC) % NC, K = cc / (NC * NC);
    const CubeMeta& m = sm[s];
    const T h = T(m.h * a.g.hscale);
    const T ih2 = T(1) / (h * h);
    T acc = T(0);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = 2 * I + (q & 1), j = 2 * J + ((q >> 1) & 1), k = 2 * K + (q >> 2);
      T nb, dg;
      stencil_p<NL, T>(tile + s * L::TILE, m, i, j, k, nb, dg);
      const T x = tile[s * L::TILE + ti<NL>(i, j, k)];
      acc += a.b[(size_t)c * L::N3 + (k * NL + j) * NL + i] - (nb - dg * x) * ih2;
    }
    a.bc[(size_t)c * NC3 + cc] = acc * T(0.125);
  }
}

// p = z + beta p (or p = z); q = A p; partial <p, q>_V.
template <int NL, typename T>
__global__ __launch_bounds__(256) void k_apply(ApplyArgs<T> a) {
  using L = Lv<NL>;
  __shared__ CubeMeta sm[L::CPB];
  __shared__ int cube[L::CPB];
  __shared__ T tile[L::CPB * L::TILE];
  __shared__ double red[8];
  load_meta<NL>(sm, cube, a.g.meta, a.g.launch, a.g.n_cubes);
  const T beta = a.first ? T(0) : T(a.sc->beta);
  for (int e = threadIdx.x; e < L::CPB * L::N3; e += WG) {
    int s, i, j, k;
    cell_of<NL>(e, s, i, j, k);
    const int c = cube[s];
    if (c < 0) continue;
    const size_t g = (size_t)c * L::N3 + (e - s * L::N3);
    tile[s * L::TILE + ti<NL>(i, j, k)] = a.first ? a.z[g] : a.z[g] + beta * a.p[g];
  }
  if (a.first)
    fill_halo<NL, RULE_P, T>(tile, sm, cube, FaceGet<NL, T>{a.zf}, BcZero<T>{});
  else
    fill_halo<NL, RULE_P, T>(tile, sm, cube, FaceGetAxpy<NL, T>{a.zf, a.pf_in, beta}, BcZero<T>{});
  __syncthreads();
  double pq = 0.0;
  for (int e = threadIdx.x; e < L::CPB * L::N3; e += WG) {
    int s, i, j, k;
    cell_of<NL>(e, s, i, j, k);
    const int c = cube[s];
    if (c < 0) continue;
    const CubeMeta& m = sm[s];
    const size_t g = (size_t)c * L::N3 + (e - s * L::N3);
    const T h = T(m.h * a.g.hscale);
    T nb, dg;
    stencil_p<NL, T>(tile + s * L::TILE, m, i, j, k, nb, dg);
    const T pv = tile[s * L::TILE + ti<NL>(i, j, k)];
    const T qv = (nb - dg * pv) / (h * h);
    a.p[g] = pv;
    a.q[g] = qv;
    pq += m.vol * double(pv) * double(qv);
  }
  export_faces<NL, T, T>(a.pf_out, tile, cube);
  const double t = block_sum(pq, red);
  if (threadIdx.x == 0) a.part[blockIdx.x] = t;
}

// x += alpha p; r -= alpha q; partial <r, r>_V.  One workgroup per cube.
template <typename T>
__global__ __launch_bounds__(256) void k_update(UpdateArgs<T> a) {
  __shared__ double red[8];
  const int c = blockIdx.x;
  const T al = T(a.sc->alpha);
  double rr = 0.0;
  const size_t base = (size_t)c * a.n3;
  for (int e = threadIdx.x; e < a.n3; e += WG) {
    const size_t g = base + e;
    a.x[g] += al * a.p[g];
    const T rv = a.r[g] - al * a.q[g];
    a.r[g] = rv;
    rr += double(rv) * double(rv);
  }
  const double t = block_sum(rr, red);
  if (threadIdx.x == 0) a.part[c] = t * a.meta[c].vol;
}

// r = b - A p (FP64), stored as TO scaled by rscale; partial <r,r>_V and <b,b>_V.
// With b == nullptr it computes r = A p instead (operator apply).
template <int NL, typename TO>
__global__ __launch_bounds__(256) void k_resid64(Resid64Args<TO> a) {
  using L = Lv<NL>;
  __shared__ CubeMeta sm[L::CPB];
  __shared__ int cube[L::CPB];
  __shared__ double tile[L::CPB * L::TILE];
  __shared__ double red[8];
  load_meta<NL>(sm, cube, a.g.meta, a.g.launch, a.g.n_cubes);
  for (int e = threadIdx.x; e < L::CPB * L::N3; e += WG) {
    int s, i, j, k;
    cell_of<NL>(e, s, i, j, k);
    const int c = cube[s];
    if (c < 0) continue;
    tile[s * L::TILE + ti<NL>(i, j, k)] = a.p ? a.p[(size_t)c * L::N3 + (e - s * L::N3)] : 0.0;
  }
  if (a.p)
    fill_halo<NL, RULE_P, double>(tile, sm, cube, FaceGet<NL, double>{a.pf}, BcZero<double>{});
  else
    zero_halo<NL, double>(tile, cube);
  __syncthreads();
  double rr = 0.0, bb = 0.0;
  for (int e = threadIdx.x; e < L::CPB * L::N3; e += WG) {
    int s, i, j, k;
    cell_of<NL>(e, s, i, j, k);
    const int c = cube[s];
    if (c < 0) continue;
    const CubeMeta& m = sm[s];
    const size_t g = (size_t)c * L::N3 + (e - s * L::N3);
    const double h = m.h * a.g.hscale;
    double nb, dg;
    stencil_p<NL, double>(tile + s * L::TILE, m, i, j, k, nb, dg);
    const double ap = (nb - dg * tile[s * L::TILE + ti<NL>(i, j, k)]) / (h * h);
    double r;
    if (a.b) {
      const double bv = a.b[g];
      r = bv - ap;
      bb += m.vol * bv * bv;
    } else {
      r = ap;
    }
    rr += m.vol * r * r;
    a.r[g] = TO(r * a.rscale);
  }
  if (a.part_rr) {
    const double t0 = block_sum(rr, red);
    __syncthreads();
    const double t1 = block_sum(bb, red);
    if (threadIdx.x == 0) {
      a.part_rr[blockIdx.x] = t0;
      if (a.part_bb) a.part_bb[blockIdx.x] = t1;
    }
  }
}

// p += d (refinement update) and export the faces of p.
template <int NL, typename T>
__global__ __launch_bounds__(256) void k_ir(IrArgs<T> a) {
  using L = Lv<NL>;
  __shared__ CubeMeta sm[L::CPB];
  __shared__ int cube[L::CPB];
  __shared__ double tile[L::CPB * L::TILE];
  load_meta<NL>(sm, cube, a.g.meta, a.g.launch, a.g.n_cubes);
  for (int e = threadIdx.x; e < L::CPB * L::N3; e += WG) {
    int s, i, j, k;
    cell_of<NL>(e, s, i, j, k);
    const int c = cube[s];
    if (c < 0) continue;
    const size_t g = (size_t)c * L::N3 + (e - s * L::N3);
    const double v = (a.d ? a.p[g] + a.dscale * double(a.d[g]) : a.p[g]);
    if (a.d) a.p[g] = v;
    tile[s * L::TILE + ti<NL>(i, j, k)] = v;
  }
  __syncthreads();
  export_faces<NL, double, double>(a.pf_out, tile, cube);
}

// Face export of a field (or of the face-normal components of a vector field).
template <int NL, typename T, typename TO>
__global__ __launch_bounds__(256) void k_export(ExportArgs<T, TO> a) {
  using L = Lv<NL>;
  __shared__ CubeMeta sm[L::CPB];
  __shared__ int cube[L::CPB];
  __shared__ T tile[L::CPB * L::TILE];
  load_meta<NL>(sm, cube, a.g.meta, a.g.launch, a.g.n_cubes);
  const int ncomp = a.comp_faces ? 3 : 1;
  for (int d = 0; d < ncomp; ++d) {
    const T* src = a.comp_faces ? a.x3[d] : a.x;
    for (int e = threadIdx.x; e < L::CPB * L::N3; e += WG) {
      int s, i, j, k;
      cell_of<NL>(e, s, i, j, k);
      const int c = cube[s];
      if (c < 0) continue;
      tile[s * L::TILE + ti<NL>(i, j, k)] = src[(size_t)c * L::N3 + (e - s * L::N3)];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < L::CPB * 6 * L::N2; e += WG) {
      const int s = e / (6 * L::N2);
      const int r = e - s * 6 * L::N2;
      const int f = r / L::N2, t = r - f * L::N2;
      if (cube[s] < 0 || (a.comp_faces && (f >> 1) != d)) continue;
      int i, j, k;
      face_cell<NL>(f, t % NL, t / NL, i, j, k);
      a.xf[(size_t)cube[s] * 6 * L::N2 + r] = TO(tile[s * L::TILE + ti<NL>(i, j, k)]);
    }
    __syncthreads();
  }
}

// Sum of per-workgroup partials in a fixed order, then the scalar recurrences.
__global__ __launch_bounds__(1024) void k_finalize(FinalizeArgs a) {
  __shared__ double red[16];
  double s0 = 0.0, s1 = 0.0;
  for (int e = threadIdx.x; e < a.n; e += 1024) {
    s0 += a.p0[e];
    if (a.p1) s1 += a.p1[e];
  }
  const double t0 = block_sum(s0, red);
  __syncthreads();
  const double t1 = block_sum(s1, red);
  if (threadIdx.x != 0) return;
  Scalars* sc = a.sc;
  switch (a.op) {
    case OP_BB:
      sc->bb = t1;
      sc->rr = t0;
      sc->rr0 = t0;
      break;
    case OP_RR0:
      sc->rr = t0;
      sc->rr0 = t0;
      break;
    case OP_ZRZQ:
      sc->zr = t0;
      sc->zq = t1;
      sc->beta = (a.first || sc->pq == 0.0) ? 0.0 : -t1 / sc->pq;
      break;
    case OP_PQ:
      sc->pq = t0;
      sc->alpha = (t0 != 0.0) ? sc->zr / t0 : 0.0;
      break;
    case OP_RR:
      sc->rr = t0;
      break;
    case OP_GU:
      sc->gU = t0;
      break;
  }
}

// Conjugate gradients on the one-cell-per-cube level (the cube graph), one workgroup.
// Solves (-V A) x = -V b, symmetric positive definite (V = relative cube volume), from
// x = 0 for at most `iters` iterations; writes x and its (trivial) face buffer.
__device__ __forceinline__ double coarse_Ax(const CubeMeta& m, const double* x, double xc, double ih2) {
  double acc = 0.0;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int kd = m.kind[f];
    double raw = 0.0;
    if (kd == FK_SAME || kd == FK_COARSER)
      raw = x[m.nbr[f][0]];
    else if (kd == FK_FINER)
      raw = 0.25 * (x[m.nbr[f][0]] + x[m.nbr[f][1]] + x[m.nbr[f][2]] + x[m.nbr[f][3]]);
    acc += RuleTab<RULE_P>::nbeff(kd) * raw - RuleTab<RULE_P>::own(kd) * xc;
  }
  return acc * ih2;
}

__device__ __forceinline__ double block_sum_all(double v, double* sh) {
  // sum over the workgroup, broadcast to every lane
  const double t = block_sum(v, sh);
  __syncthreads();
  if (threadIdx.x == 0) sh[0] = t;
  __syncthreads();
  const double r = sh[0];
  __syncthreads();
  return r;
}

template <typename T>
__global__ __launch_bounds__(1024) void k_coarse(CoarseArgs<T> a) {
  __shared__ double red[16];
  const int nc = a.n_cubes;
  double* xv = a.w;
  double* rv = a.w + nc;
  double* pv = a.w + 2 * (size_t)nc;
  double* qv = a.w + 3 * (size_t)nc;
  double rr = 0.0;
  for (int c = threadIdx.x; c < nc; c += 1024) {
    const double r = -a.meta[c].vol * double(a.b[c]);
    xv[c] = 0.0;
    rv[c] = r;
    pv[c] = r;
    rr += r * r;
  }
  rr = block_sum_all(rr, red);
  for (int it = 0; it < a.iters && rr > 0.0; ++it) {
    double pq = 0.0;
    for (int c = threadIdx.x; c < nc; c += 1024) {
      const CubeMeta& m = a.meta[c];
      const double h = m.h * a.hscale;
      const double q = -m.vol * coarse_Ax(m, pv, pv[c], 1.0 / (h * h));
      qv[c] = q;
      pq += pv[c] * q;
    }
    pq = block_sum_all(pq, red);
    if (!(pq > 0.0)) break;
    const double al = rr / pq;
    double rn = 0.0;
    for (int c = threadIdx.x; c < nc; c += 1024) {
      xv[c] += al * pv[c];
      const double r = rv[c] - al * qv[c];
      rv[c] = r;
      rn += r * r;
    }
    rn = block_sum_all(rn, red);
    const double be = rn / rr;
    rr = rn;
    for (int c = threadIdx.x; c < nc; c += 1024) pv[c] = rv[c] + be * pv[c];
    __syncthreads();
  }
  for (int c = threadIdx.x; c < nc; c += 1024) {
    const T v = T(xv[c]);
    a.x[c] = v;
#pragma unroll
    for (int f = 0; f < 6; ++f) a.xf[(size_t)c * 6 + f] = v;
  }
}

// ------------------------------------------------------------------------------------------
// Multigrid on the cube graph (one unknown per cube), one workgroup: multicolour
// Gauss-Seidel on every graph level, volume-weighted restriction, piecewise-constant
// prolongation, CG on the last (smallest) level.  Runs `cycles` V-cycles from x = 0.
// ------------------------------------------------------------------------------------------
// sum_w val[w][i] * x[col[w][i]] (column-major ELL: the loads of all w are independent)
template <typename T>
__device__ __forceinline__ T g_offdiag(const GLevel<T>& L, const T* x, int i) {
  T acc = T(0);
  for (int w = 0; w < L.W; ++w) {
    const size_t o = size_t(w) * L.n + i;
    acc += L.val[o] * x[L.col[o]];
  }
  return acc;
}

// Width-6 rows (every lattice level): four nodes per lane per pass, all their coupling loads
// issued before any of them is used.
template <typename T, bool RESID>
__device__ __forceinline__ void g_pass6(const GLevel<T>& L, int lo, int hi) {
  constexpr int U = 4;
  for (int base = lo + threadIdx.x; base < hi; base += U * 1024) {
    int col[U][6];
    T val[U][6], bb[U], dg[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = base + u * 1024;
      const int ii = i < hi ? i : lo;
#pragma unroll
      for (int w = 0; w < 6; ++w) {
        col[u][w] = L.col[size_t(w) * L.n + ii];
        val[u][w] = L.val[size_t(w) * L.n + ii];
      }
      bb[u] = L.b[ii];
      dg[u] = L.diag[ii];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = base + u * 1024;
      if (i >= hi) continue;
      T acc = T(0);
#pragma unroll
      for (int w = 0; w < 6; ++w) acc += val[u][w] * L.x[col[u][w]];
      if (RESID)
        L.r[i] = bb[u] - dg[u] * L.x[i] - acc;
      else
        L.x[i] = (bb[u] - acc) / dg[u];
    }
  }
}

template <typename T>
__device__ void g_smooth(const GLevel<T>& L, int sweeps, bool forward) {
  for (int s = 0; s < sweeps; ++s)
    for (int cc = 0; cc < L.ncol; ++cc) {
      const int c = forward ? cc : L.ncol - 1 - cc;
      const int o1 = L.color_off[c + 1];
      if (L.W == 6) {
        g_pass6<T, false>(L, L.color_off[c], o1);
      } else {
        for (int i = L.color_off[c] + threadIdx.x; i < o1; i += blockDim.x)
          L.x[i] = (L.b[i] - g_offdiag(L, L.x, i)) / L.diag[i];
      }
      __syncthreads();
    }
}

template <typename T>
__device__ void g_residual(const GLevel<T>& L) {
  if (L.W == 6) {
    g_pass6<T, true>(L, 0, L.n);
  } else {
    for (int i = threadIdx.x; i < L.n; i += blockDim.x)
      L.r[i] = L.b[i] - L.diag[i] * L.x[i] - g_offdiag(L, L.x, i);
  }
  __syncthreads();
}

template <typename T>
__device__ void g_bottom(const GLevel<T>& L, int iters, double* w, double* red) {
  // CG on the symmetric positive definite (-V A) x = -V b (V = relative node volume).
  double* xv = w;
  double* rv = w + L.n;
  double* pv = w + 2 * L.n;
  double* qv = w + 3 * L.n;
  double rr = 0.0;
  for (int i = threadIdx.x; i < L.n; i += blockDim.x) {
    const double r = -double(L.vol[i]) * double(L.b[i]);
    xv[i] = 0.0;
    rv[i] = r;
    pv[i] = r;
    rr += r * r;
  }
  rr = block_sum_all(rr, red);
  const double stop = 1e-20 * rr;
  for (int it = 0; it < iters && rr > stop; ++it) {
    double pq = 0.0;
    for (int i = threadIdx.x; i < L.n; i += blockDim.x) {
      double acc = double(L.diag[i]) * pv[i];
      for (int w = 0; w < L.W; ++w) {
        const size_t o = size_t(w) * L.n + i;
        acc += double(L.val[o]) * pv[L.col[o]];
      }
      acc *= -double(L.vol[i]);
      qv[i] = acc;
      pq += pv[i] * acc;
    }
    pq = block_sum_all(pq, red);
    if (!(pq > 0.0)) break;
    const double al = rr / pq;
    double rn = 0.0;
    for (int i = threadIdx.x; i < L.n; i += blockDim.x) {
      xv[i] += al * pv[i];
      rv[i] -= al * qv[i];
      rn += rv[i] * rv[i];
    }
    rn = block_sum_all(rn, red);
    const double be = rn / rr;
    rr = rn;
    for (int i = threadIdx.x; i < L.n; i += blockDim.x) pv[i] = rv[i] + be * pv[i];
    __syncthreads();
  }
  for (int i = threadIdx.x; i < L.n; i += blockDim.x) L.x[i] = T(xv[i]);
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(1024) void k_coarse_mg(CoarseMGArgs<T> a) {
  extern __shared__ __align__(16) unsigned char gsm[];
  __shared__ double red[16];
  __shared__ GLevel<T> lv[kMaxGraphLevels];
  if (threadIdx.x < a.nlev) {
    GLevel<T> L = a.lev[threadIdx.x];
    if (L.lds_x >= 0) L.x = reinterpret_cast<T*>(gsm + L.lds_x);
    if (L.lds_b >= 0) L.b = reinterpret_cast<T*>(gsm + L.lds_b);
    if (L.lds_r >= 0) L.r = reinterpret_cast<T*>(gsm + L.lds_r);
    lv[threadIdx.x] = L;
  }
  __syncthreads();
  const int G = a.nlev;
  for (int c = threadIdx.x; c < lv[0].n; c += blockDim.x) {
    const int i = a.perm0[c];
    lv[0].b[i] = a.b_in[c];
    lv[0].x[i] = T(0);
  }
  __syncthreads();
  for (int cy = 0; cy < a.cycles; ++cy) {
    for (int g = 0; g + 1 < G; ++g) {
      g_smooth(lv[g], a.pre, true);
      g_residual(lv[g]);
      const GLevel<T>& C = lv[g + 1];
      const T* r = lv[g].r;
      for (int J = threadIdx.x; J < C.n; J += blockDim.x) {
        T acc = T(0);
        for (int w = 0; w < C.CW; ++w) {
          const size_t o = size_t(w) * C.n + J;
          const int ch = C.child[o];
          if (ch >= 0) acc += C.child_w[o] * r[ch];
        }
        C.b[J] = acc;
        C.x[J] = T(0);
      }
      __syncthreads();
    }
    g_bottom(lv[G - 1], a.bottom_iters, a.w, red);
    for (int g = G - 2; g >= 0; --g) {
      const GLevel<T>& F = lv[g];
      const T* xc = lv[g + 1].x;
      for (int i = threadIdx.x; i < F.n; i += blockDim.x) F.x[i] += xc[F.parent[i]];
      __syncthreads();
      g_smooth(F, a.post, false);
    }
  }
  for (int c = threadIdx.x; c < lv[0].n; c += blockDim.x) {
    const T v = lv[0].x[a.perm0[c]];
    a.x_out[c] = v;
#pragma unroll
    for (int f = 0; f < 6; ++f) a.xf_out[(size_t)c * 6 + f] = v;
  }
}

__global__ __launch_bounds__(256) void k_scale(ScaleArgs a) {
  const int c = blockIdx.x;
  const double w = a.power > 0 ? a.meta[c].vol : 1.0 / a.meta[c].vol;
  const size_t base = (size_t)c * a.n3;
  for (int e = threadIdx.x; e < a.n3; e += WG) a.y[base + e] = a.x[base + e] * w;
}

}  // namespace

// ------------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------------
#define BCM_DISPATCH_NL(NLV, CALL)                 \
  switch (NLV) {                                   \
    case 16: { constexpr int NLC = 16; CALL; } break; \
    case 8: { constexpr int NLC = 8; CALL; } break;   \
    case 4: { constexpr int NLC = 4; CALL; } break;   \
    case 2: { constexpr int NLC = 2; CALL; } break;   \
    default: return hipErrorInvalidValue;          \
  }

static inline int n_wg(int NL, int n_cubes) {
  const int cpb = cubes_per_wg(NL);
  return (n_cubes + cpb - 1) / cpb;
}

template <typename T>
hipError_t launch_smooth(int NL, const SmoothArgs<T>& a, hipStream_t s) {
  if (NL == 16) return launch16_smooth<T>(a, s);
  BCM_DISPATCH_NL(NL, hipLaunchKernelGGL((k_smooth<NLC, T>), dim3(n_wg(NLC, a.g.n_cubes)), dim3(WG), 0, s, a));
  return hipGetLastError();
}
template <typename T>
hipError_t launch_restrict(int NL, const RestrictArgs<T>& a, hipStream_t s) {
  if (NL == 16) return launch16_restrict<T>(a, s);
  BCM_DISPATCH_NL(NL, hipLaunchKernelGGL((k_restrict<NLC, T>), dim3(n_wg(NLC, a.g.n_cubes)), dim3(WG), 0, s, a));
  return hipGetLastError();
}
template <typename T>
hipError_t launch_apply(int NL, const ApplyArgs<T>& a, hipStream_t s) {
  if (NL == 16) return launch16_apply<T>(a, s);
  BCM_DISPATCH_NL(NL, hipLaunchKernelGGL((k_apply<NLC, T>), dim3(n_wg(NLC, a.g.n_cubes)), dim3(WG), 0, s, a));
  return hipGetLastError();
}
template <typename T>
hipError_t launch_update(const UpdateArgs<T>& a, hipStream_t s) {
  hipLaunchKernelGGL((k_update<T>), dim3(a.n_cubes), dim3(WG), 0, s, a);
  return hipGetLastError();
}
template <typename TO>
hipError_t launch_resid64(int NL, const Resid64Args<TO>& a, hipStream_t s) {
  if (NL == 16) return launch16_resid64<TO>(a, s);
  BCM_DISPATCH_NL(NL, hipLaunchKernelGGL((k_resid64<NLC, TO>), dim3(n_wg(NLC, a.g.n_cubes)), dim3(WG), 0, s, a));
  return hipGetLastError();
}
template <typename T>
hipError_t launch_ir(int NL, const IrArgs<T>& a, hipStream_t s) {
  BCM_DISPATCH_NL(NL, hipLaunchKernelGGL((k_ir<NLC, T>), dim3(n_wg(NLC, a.g.n_cubes)), dim3(WG), 0, s, a));
  return hipGetLastError();
}
template <typename T, typename TO>
hipError_t launch_export(int NL, const ExportArgs<T, TO>& a, hipStream_t s) {
  BCM_DISPATCH_NL(NL, hipLaunchKernelGGL((k_export<NLC, T, TO>), dim3(n_wg(NLC, a.g.n_cubes)), dim3(WG), 0, s, a));
  return hipGetLastError();
}
hipError_t launch_finalize(const FinalizeArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, s, a);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_coarse(const CoarseArgs<T>& a, hipStream_t s) {
  hipLaunchKernelGGL((k_coarse<T>), dim3(1), dim3(1024), 0, s, a);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_coarse_mg(const CoarseMGArgs<T>& a, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_coarse_mg<T>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kGraphLdsBudget);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL((k_coarse_mg<T>), dim3(1), dim3(1024), a.lds_bytes, s, a);
  return hipGetLastError();
}
template hipError_t launch_coarse_mg<float>(const CoarseMGArgs<float>&, hipStream_t);
template hipError_t launch_coarse_mg<double>(const CoarseMGArgs<double>&, hipStream_t);

hipError_t launch_scale(const ScaleArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(a.n_cubes), dim3(WG), 0, s, a);
  return hipGetLastError();
}

#define BCM_INST_T(T)                                                              \
  template hipError_t launch_smooth<T>(int, const SmoothArgs<T>&, hipStream_t);     \
  template hipError_t launch_restrict<T>(int, const RestrictArgs<T>&, hipStream_t); \
  template hipError_t launch_apply<T>(int, const ApplyArgs<T>&, hipStream_t);       \
  template hipError_t launch_update<T>(const UpdateArgs<T>&, hipStream_t);          \
  template hipError_t launch_resid64<T>(int, const Resid64Args<T>&, hipStream_t);   \
  template hipError_t launch_ir<T>(int, const IrArgs<T>&, hipStream_t);             \
  template hipError_t launch_coarse<T>(const CoarseArgs<T>&, hipStream_t);          \
  template hipError_t launch_export<T, T>(int, const ExportArgs<T, T>&, hipStream_t);
BCM_INST_T(float)
BCM_INST_T(double)
template hipError_t launch_export<double, float>(int, const ExportArgs<double, float>&, hipStream_t);

}  // namespace bcm
