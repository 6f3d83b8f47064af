// Krylov, reduction and coarse-level kernels of the pressure Poisson solve (Sec. 3): the
// vector update with its fused norm, face export, the deterministic reduction of partial
// sums, the conjugate-gradient solve on the one-cell-per-cube level (Sec. 7: at most 10
// iterations) and multigrid on the cube graph that replaces it by default.  The stencil
// kernels of the per-cube levels are in kernels_col.hip.
//
// All sums are accumulated in FP64 with a fixed reduction order: each workgroup writes one
// partial, k_finalize sums them.
#include "kernels.hpp"
#include "tile.hpp"

namespace bcm {

namespace {

// x += alpha p; r -= alpha q; partial <r, r>_V.  One workgroup per cube.  SEL splits the two
// updates (1: r and <r, r> only, 2: x only; 0: both), so that the x update can run beside the
// next V-cycle; 3: <r - alpha q, r - alpha q>_V only, r left as it is (a convergence probe).
template <typename T, int SEL>
__global__ __launch_bounds__(256) void k_update(UpdateArgs<T> a) {
  __shared__ double red[8];
  const int c = blockIdx.x;
  const T al = T(a.sc->alpha);
  double rr = 0.0;
  const size_t base = (size_t)c * a.n3;
  constexpr bool do_x = SEL == 0 || SEL == 2, do_r = SEL != 2;
  for (int e = threadIdx.x; e < a.n3; e += WG) {
    const size_t g = base + e;
    if (do_x) st_nt(a.x + g, (a.x_zero ? T(0) : ld_nt(a.x + g)) + al * ld_nt(a.p + g));
    if (do_r) {
      const T rv = ld_nt(a.r + g) - al * ld_nt(a.q + g);
      if (SEL != 3) st_nt(a.r + g, rv);
      rr += double(rv) * double(rv);
    }
  }
  if (!do_r) return;
  const double t = block_sum(rr, red);
  if (threadIdx.x == 0) a.part[c] = t * a.meta[c].vol;
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
      a.xf[(size_t)cube[s] * L::FACE + r] = TO(tile[s * L::TILE + ti<NL>(i, j, k)]);
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
    case OP_ZRZQ: {
      const double zr_old = sc->zr;
      sc->zr = t0;
      sc->zq = t1;
      if (a.first)
        sc->beta = 0.0;
      else if (a.p1)  // flexible CG: -<z, q_old> / <p_old, q_old>
        sc->beta = sc->pq == 0.0 ? 0.0 : -t1 / sc->pq;
      else            // standard preconditioned CG: <z, r> / <z_old, r_old>
        sc->beta = zr_old == 0.0 ? 0.0 : t0 / zr_old;
      break;
    }
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
    case OP_VUU:
      sc->vuu = t0;
      break;
    case OP_B0:
      sc->bb = t0;
      break;
  }
  if (a.mirror) {
    a.mirror->sc = *sc;
    __threadfence_system();
    __hip_atomic_store(&a.mirror->seq, a.seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
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
    for (int f = 0; f < 6; ++f) a.xf[(size_t)c * face_stride(1) + f] = v;
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

// Width-6 rows (every lattice level): two nodes per lane per pass, all their coupling loads
// issued before any of them is used.
template <typename T, bool RESID>
__device__ __forceinline__ void g_pass6(const GLevel<T>& L, int lo, int hi) {
  constexpr int U = 2;
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

// Packed rows held in registers: lane t owns nodes t + 1024 k (k < K) of a level with at most
// 1024 K nodes, so that its sweeps and residual read the rows once per kernel, not per pass
// (the passes of one workgroup are bound by how fast its CU brings rows in: 56 bytes per node
// in FP32 as columns and values, 16 as packed columns and the diagonal).  Padding slots hold
// the node's own index and are skipped.
template <typename T, int K>
struct GRows {
  uint32_t pc[K][3];
  T dg[K];
  __device__ __forceinline__ void load(const GLevel<T>& L) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = threadIdx.x + 1024 * k;
      const int ii = i < L.n ? i : 0;
#pragma unroll
      for (int q = 0; q < 3; ++q) pc[k][q] = L.pcol[size_t(q) * L.n + ii];
      dg[k] = L.diag[ii];
    }
  }
  // nodes [lo, hi) of one colour (RESID false) or all nodes (RESID true), four at a time; a
  // colour does not couple with itself, so the loads of a group may come before its stores.
  // x, b and r are the level's arrays in LDS, passed as pointers derived from the kernel's
  // shared array so that the compiler emits LDS instructions rather than generic ones.
  template <bool RESID>
  __device__ __forceinline__ void pass(T* x, const T* b, T* r, T uval, int lo, int hi) const {
#pragma unroll
    for (int k0 = 0; k0 < K; k0 += 4) {
      constexpr int M = K < 4 ? K : 4;
      T acc[M];
#pragma unroll
      for (int m = 0; m < M; ++m) {
        const int k = k0 + m, i = threadIdx.x + 1024 * k;
        acc[m] = T(0);
        if (k >= K || i < lo || i >= hi) continue;
        // opaque copies: keeps the compiler from unpacking all the columns once, outside
        // the sweep loops, into 8 times as many registers
        uint32_t p[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          p[q] = pc[k][q];
          asm volatile("" : "+v"(p[q]));
        }
#pragma unroll
        for (int w = 0; w < 6; ++w) {
          const int c = int(w & 1 ? p[w >> 1] >> 16 : p[w >> 1] & 0xffffu);
          if (c != i) acc[m] += uval * x[c];
        }
        if (RESID) acc[m] = b[i] - dg[k] * x[i] - acc[m];
        else acc[m] = (b[i] - acc[m]) / dg[k];
      }
#pragma unroll
      for (int m = 0; m < M; ++m) {
        const int k = k0 + m, i = threadIdx.x + 1024 * k;
        if (k >= K || i < lo || i >= hi) continue;
        if (RESID) r[i] = acc[m];
        else x[i] = acc[m];
      }
    }
  }
  __device__ __forceinline__ void smooth(const GLevel<T>& L, T* x, const T* b, int sweeps,
                                         bool forward) const {
    for (int s = 0; s < sweeps; ++s)
      for (int cc = 0; cc < L.ncol; ++cc) {
        const int c = forward ? cc : L.ncol - 1 - cc;
        pass<false>(x, b, nullptr, L.uval, L.color_off[c], L.color_off[c + 1]);
        __syncthreads();
      }
  }
  __device__ __forceinline__ void residual(const GLevel<T>& L, T* x, const T* b, T* r) const {
    pass<true>(x, b, r, L.uval, 0, L.n);
    __syncthreads();
  }
};

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

// b = volume-weighted restriction of the finer level's residual r; x = 0.  With at most 8
// children (every merge here is 2x2x2 or a subset) all loads of a node are issued before use.
template <typename T>
__device__ __forceinline__ void g_restrict(const GLevel<T>& C, const T* r, T* cb, T* cx) {
  for (int J = threadIdx.x; J < C.n; J += blockDim.x) {
    T acc = T(0);
    if (C.CW <= 8) {
      int ch[8];
      T wt[8], rv[8];
#pragma unroll
      for (int w = 0; w < 8; ++w) {
        ch[w] = w < C.CW ? C.child[size_t(w) * C.n + J] : -1;
        wt[w] = w < C.CW ? C.child_w[size_t(w) * C.n + J] : T(0);
      }
#pragma unroll
      for (int w = 0; w < 8; ++w) rv[w] = r[ch[w] >= 0 ? ch[w] : 0];
#pragma unroll
      for (int w = 0; w < 8; ++w)
        if (ch[w] >= 0) acc += wt[w] * rv[w];
    } else {
      for (int w = 0; w < C.CW; ++w) {
        const size_t o = size_t(w) * C.n + J;
        const int ch = C.child[o];
        if (ch >= 0) acc += C.child_w[o] * r[ch];
      }
    }
    cb[J] = acc;
    cx[J] = T(0);
  }
  __syncthreads();
}

// Direct solve of the (small) last level with its inverse precomputed on the host.
template <typename T>
__device__ __forceinline__ void g_direct(int n, const T* inv_t, const T* b, T* x) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    T acc = T(0);
    for (int j = 0; j < n; ++j) acc += inv_t[j * n + i] * b[j];
    x[i] = acc;
  }
  __syncthreads();
}

// x of level g += x of its parent (piecewise-constant prolongation).
template <typename T>
__device__ __forceinline__ void g_prolong(const GLevel<T>& F, T* x, const T* xc) {
  for (int i = threadIdx.x; i < F.n; i += blockDim.x) x[i] += xc[F.parent[i]];
  __syncthreads();
}

// The vector update x += alpha p of the workgroups after the first of k_coarse_mg: 16-byte
// non-temporal accesses, the same arithmetic as k_update.
template <typename T>
__device__ __forceinline__ void coarse_side_update(const CoarseMGArgs<T>& a) {
  typedef T V __attribute__((ext_vector_type(16 / sizeof(T))));
  constexpr int W = 16 / sizeof(T);
  const T al = T(*a.xu_alpha);
  const size_t nv = a.xu_n / W;
  const size_t first = size_t(blockIdx.x - 1) * blockDim.x + threadIdx.x;
  const size_t stride = size_t(gridDim.x - 1) * blockDim.x;
  V* xv = reinterpret_cast<V*>(a.xu_x);
  const V* pv = reinterpret_cast<const V*>(a.xu_p);
  for (size_t e = first; e < nv; e += stride) {
    const V p = __builtin_nontemporal_load(pv + e);
    const V x = a.xu_zero ? V(T(0)) : __builtin_nontemporal_load(xv + e);
    __builtin_nontemporal_store(x + al * p, xv + e);
  }
  for (size_t e = nv * W + first; e < a.xu_n; e += stride)
    a.xu_x[e] = (a.xu_zero ? T(0) : a.xu_x[e]) + al * a.xu_p[e];
}

template <typename T>
__global__ __launch_bounds__(1024) void k_coarse_mg(CoarseMGArgs<T> a) {
  if (blockIdx.x > 0) {  // the side update (only launched with xu_n > 0)
    coarse_side_update(a);
    return;
  }
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
  const int G = a.nlev, S = a.start;
  const T* binv = a.binv;
  if (binv && a.lds_inv >= 0) {
    T* sb = reinterpret_cast<T*>(gsm + a.lds_inv);
    const int nn = lv[G - 1].n * lv[G - 1].n;
    for (int e = threadIdx.x; e < nn; e += blockDim.x) sb[e] = binv[e];
    binv = sb;
  }
  // Arrays kept in LDS are addressed through pointers derived from gsm here (not the
  // generic ones stored in lv), so that the compiler emits LDS instructions for them.
  auto lds = [&](int off) { return reinterpret_cast<T*>(gsm + off); };
  auto in_lds = [&](int g) { return lv[g].lds_x >= 0 && lv[g].lds_b >= 0 && lv[g].lds_r >= 0; };
  auto gather = [&](T* b0, T* x0) {
    for (int c = threadIdx.x; c < lv[0].n; c += blockDim.x) {
      const int i = a.perm0[c];
      b0[i] = a.b_in[c];
      x0[i] = T(0);
    }
  };
  if (S == 0) {
    if (lv[0].lds_b >= 0 && lv[0].lds_x >= 0)
      gather(lds(lv[0].lds_b), lds(lv[0].lds_x));
    else
      gather(lv[0].b, lv[0].x);
  } else {
    const GLevel<T>& L = a.lev[S];  // global buffers of the first level solved here
    for (int i = threadIdx.x; i < L.n; i += blockDim.x) {
      if (lv[S].b != L.b) lv[S].b[i] = L.b[i];
      lv[S].x[i] = T(0);
    }
  }
  // rows of the first levels in registers when they are packed and small enough (one level
  // in FP64, three in FP32) and their arrays live in LDS
  constexpr int K0 = sizeof(T) == 4 ? 8 : 4;
  GRows<T, K0> R0;
  GRows<T, 1> R1, R2;
  const bool c0 = S + 1 < G && lv[S].pcol && lv[S].n <= K0 * 1024 && in_lds(S);
  const bool c1 = sizeof(T) == 4 && S + 2 < G && lv[S + 1].pcol && lv[S + 1].n <= 1024 && in_lds(S + 1);
  const bool c2 = sizeof(T) == 4 && S + 3 < G && lv[S + 2].pcol && lv[S + 2].n <= 1024 && in_lds(S + 2);
  if (c0) R0.load(lv[S]);
  if (c1) R1.load(lv[S + 1]);
  if (c2) R2.load(lv[S + 2]);
  __syncthreads();
  for (int cy = 0; cy < (S == 0 ? a.cycles : 1); ++cy) {
    for (int g = S; g + 1 < G; ++g) {
      const GLevel<T>& L = lv[g];
      if (g == S && c0) {
        R0.smooth(L, lds(L.lds_x), lds(L.lds_b), a.pre, true);
        R0.residual(L, lds(L.lds_x), lds(L.lds_b), lds(L.lds_r));
      } else if (g == S + 1 && c1) {
        R1.smooth(L, lds(L.lds_x), lds(L.lds_b), a.pre, true);
        R1.residual(L, lds(L.lds_x), lds(L.lds_b), lds(L.lds_r));
      } else if (g == S + 2 && c2) {
        R2.smooth(L, lds(L.lds_x), lds(L.lds_b), a.pre, true);
        R2.residual(L, lds(L.lds_x), lds(L.lds_b), lds(L.lds_r));
      } else {
        g_smooth(L, a.pre, true);
        g_residual(L);
      }
      const GLevel<T>& C = lv[g + 1];
      if (L.lds_r >= 0 && C.lds_b >= 0 && C.lds_x >= 0)
        g_restrict(C, lds(L.lds_r), lds(C.lds_b), lds(C.lds_x));
      else
        g_restrict(C, L.r, C.b, C.x);
    }
    const GLevel<T>& B = lv[G - 1];
    if (binv) {
      if (a.lds_inv >= 0 && B.lds_b >= 0 && B.lds_x >= 0)
        g_direct(B.n, lds(a.lds_inv), lds(B.lds_b), lds(B.lds_x));
      else
        g_direct(B.n, binv, B.b, B.x);
    } else {
      g_bottom(B, a.bottom_iters, a.w, red);
    }
    for (int g = G - 2; g >= S; --g) {
      const GLevel<T>& F = lv[g];
      const GLevel<T>& C = lv[g + 1];
      if (F.lds_x >= 0 && C.lds_x >= 0)
        g_prolong(F, lds(F.lds_x), lds(C.lds_x));
      else
        g_prolong(F, F.x, C.x);
      if (g == S && c0)
        R0.smooth(F, lds(F.lds_x), lds(F.lds_b), a.post, false);
      else if (g == S + 1 && c1)
        R1.smooth(F, lds(F.lds_x), lds(F.lds_b), a.post, false);
      else if (g == S + 2 && c2)
        R2.smooth(F, lds(F.lds_x), lds(F.lds_b), a.post, false);
      else
        g_smooth(F, a.post, false);
    }
  }
  auto scatter = [&](const T* x0) {
    for (int c = threadIdx.x; c < lv[0].n; c += blockDim.x) {
      const T v = x0[a.perm0[c]];
      a.x_out[c] = v;
#pragma unroll
      for (int f = 0; f < 6; ++f) a.xf_out[(size_t)c * face_stride(1) + f] = v;
    }
  };
  if (S == 0) {
    if (lv[0].lds_x >= 0)
      scatter(lds(lv[0].lds_x));
    else
      scatter(lv[0].x);
  } else if (lv[S].x != a.lev[S].x) {
    for (int i = threadIdx.x; i < lv[S].n; i += blockDim.x) a.lev[S].x[i] = lv[S].x[i];
  }
}

// ---- multi-workgroup kernels of the large graph levels (one lane per node) ----

// Level 0 from the one-cell-per-cube right-hand side: b = b_in (permuted), x = 0.
template <typename T>
__global__ __launch_bounds__(256) void k_g_gather(GStepArgs<T> a) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= a.n_cubes) return;
  const GLevel<T>& L = a.lev[0];
  const int i = a.perm0[c];
  L.b[i] = a.b_in[c];
  L.x[i] = T(0);
}

// sum_w val[w][i] * x[col[w][i]] with every load of the row issued before use (W <= 16).
template <typename T>
__device__ __forceinline__ T g_row(const GLevel<T>& L, int i) {
  if (L.W > 16) return g_offdiag(L, L.x, i);
  int col[16];
  T val[16], xv[16];
#pragma unroll
  for (int w = 0; w < 16; ++w) {
    col[w] = w < L.W ? L.col[size_t(w) * L.n + i] : i;
    val[w] = w < L.W ? L.val[size_t(w) * L.n + i] : T(0);
  }
#pragma unroll
  for (int w = 0; w < 16; ++w) xv[w] = w < L.W ? L.x[col[w]] : T(0);
  T acc = T(0);
#pragma unroll
  for (int w = 0; w < 16; ++w) acc += val[w] * xv[w];
  return acc;
}

// One colour of a Gauss-Seidel sweep on level g: nodes [lo, hi) do not couple.
template <typename T>
__global__ __launch_bounds__(256) void k_g_smooth(GStepArgs<T> a) {
  const int i = a.lo + blockIdx.x * 256 + threadIdx.x;
  if (i >= a.hi) return;
  const GLevel<T>& L = a.lev[a.g];
  L.x[i] = (L.b[i] - g_row(L, i)) / L.diag[i];
}

// Residual of level g (one lane per node), kept in r for the restriction.
template <typename T>
__global__ __launch_bounds__(256) void k_g_resid(GStepArgs<T> a) {
  const GLevel<T>& F = a.lev[a.g];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= F.n) return;
  F.r[i] = F.b[i] - F.diag[i] * F.x[i] - g_row(F, i);
}

// Residual of level g restricted to level g+1 (volume weights, every child load issued before
// use), x of level g+1 set to zero.
template <typename T>
__global__ __launch_bounds__(256) void k_g_restrict(GStepArgs<T> a) {
  const GLevel<T>& F = a.lev[a.g];
  const GLevel<T>& C = a.lev[a.g + 1];
  const int J = blockIdx.x * 256 + threadIdx.x;
  if (J >= C.n) return;
  T acc = T(0);
  if (C.CW <= 8) {
    int ch[8];
    T w[8], r[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const size_t o = size_t(k) * C.n + J;
      ch[k] = k < C.CW ? C.child[o] : -1;
      w[k] = k < C.CW ? C.child_w[o] : T(0);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) r[k] = ch[k] >= 0 ? F.r[ch[k]] : T(0);
#pragma unroll
    for (int k = 0; k < 8; ++k) acc += w[k] * r[k];
  } else {
    for (int k = 0; k < C.CW; ++k) {
      const size_t o = size_t(k) * C.n + J;
      const int ch = C.child[o];
      if (ch >= 0) acc += C.child_w[o] * F.r[ch];
    }
  }
  C.b[J] = acc;
  C.x[J] = T(0);
}

// x of level g += x of its parent on level g+1 (piecewise-constant prolongation).
template <typename T>
__global__ __launch_bounds__(256) void k_g_prolong(GStepArgs<T> a) {
  const GLevel<T>& F = a.lev[a.g];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= F.n) return;
  F.x[i] += a.lev[a.g + 1].x[F.parent[i]];
}

// Level-0 solution back to cube order, with its (trivial) face buffer.
template <typename T>
__global__ __launch_bounds__(256) void k_g_scatter(GStepArgs<T> a) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= a.n_cubes) return;
  const T v = a.lev[0].x[a.perm0[c]];
  a.x_out[c] = v;
#pragma unroll
  for (int f = 0; f < 6; ++f) a.xf_out[(size_t)c * face_stride(1) + f] = v;
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
  return launchc_smooth<T>(NL, a, s);
}
template <typename T>
hipError_t launch_apply(int NL, const ApplyArgs<T>& a, hipStream_t s) {
  return launchc_apply<T>(NL, a, s);
}
template <typename T>
hipError_t launch_update(const UpdateArgs<T>& a, hipStream_t s) {
  if (a.part_sel == 1)
    hipLaunchKernelGGL((k_update<T, 1>), dim3(a.n_cubes), dim3(WG), 0, s, a);
  else if (a.part_sel == 2)
    hipLaunchKernelGGL((k_update<T, 2>), dim3(a.n_cubes), dim3(WG), 0, s, a);
  else if (a.part_sel == 3)
    hipLaunchKernelGGL((k_update<T, 3>), dim3(a.n_cubes), dim3(WG), 0, s, a);
  else
    hipLaunchKernelGGL((k_update<T, 0>), dim3(a.n_cubes), dim3(WG), 0, s, a);
  return hipGetLastError();
}
template <typename TO>
hipError_t launch_resid64(int NL, const Resid64Args<TO>& a, hipStream_t s) {
  return launchc_resid64<TO>(NL, a, s);
}
template <typename T>
hipError_t launch_ir(int NL, const IrArgs<T>& a, hipStream_t s) {
  return launchc_ir<T>(NL, a, s);
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
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kGraphLdsTotal);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int grid = a.xu_n > 0 ? 1 + (a.xu_wgs > 1 ? a.xu_wgs : 1) : 1;
  hipLaunchKernelGGL((k_coarse_mg<T>), dim3(grid), dim3(1024), a.lds_bytes, s, a);
  return hipGetLastError();
}
template hipError_t launch_coarse_mg<float>(const CoarseMGArgs<float>&, hipStream_t);
template hipError_t launch_coarse_mg<double>(const CoarseMGArgs<double>&, hipStream_t);

template <typename T>
hipError_t launch_g_step(int kind, int n, const GStepArgs<T>& a, hipStream_t s) {
  const dim3 grid((n + 255) / 256), block(256);
  if (n <= 0) return hipSuccess;
  switch (kind) {
    case G_GATHER: hipLaunchKernelGGL((k_g_gather<T>), grid, block, 0, s, a); break;
    case G_SMOOTH: hipLaunchKernelGGL((k_g_smooth<T>), grid, block, 0, s, a); break;
    case G_RESID: hipLaunchKernelGGL((k_g_resid<T>), grid, block, 0, s, a); break;
    case G_RESTRICT: hipLaunchKernelGGL((k_g_restrict<T>), grid, block, 0, s, a); break;
    case G_PROLONG: hipLaunchKernelGGL((k_g_prolong<T>), grid, block, 0, s, a); break;
    case G_SCATTER: hipLaunchKernelGGL((k_g_scatter<T>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template hipError_t launch_g_step<float>(int, int, const GStepArgs<float>&, hipStream_t);
template hipError_t launch_g_step<double>(int, int, const GStepArgs<double>&, hipStream_t);

hipError_t launch_scale(const ScaleArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(a.n_cubes), dim3(WG), 0, s, a);
  return hipGetLastError();
}

#define BCM_INST_T(T)                                                              \
  template hipError_t launch_smooth<T>(int, const SmoothArgs<T>&, hipStream_t);     \
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
