// Finest-level (16^3 cells per cube) stencil kernels: the HBM-bound part of the Poisson solve.
//
// Layout per workgroup (256 lanes): lane t owns the column (i = t & 15, j = t >> 4) of a
// cube, k = 0..15 held in registers.  Only the i/j neighbours go through LDS: a tile of 16
// planes of 18 x 18 (the cube's plane plus its x/y halo ring); the z neighbours are the
// lane's own registers, with the z halo of the column in two registers.  Every global
// access is a full 1 KB plane (coalesced) or a 1 KB face slab.
//
// The solver kernels are persistent: a workgroup walks the Z-ordered launch table with stride
// gridDim.x (a multiple of 8, so each workgroup stays on the XCD that owns its stretch of the
// curve) and, while it computes one cube, the loads of its next cube are in flight.  The
// prefetch does integer work only: the halo addresses are computed branch-free from the face
// relations and the loads land in raw registers that are combined when the cube is staged,
// because any arithmetic on a loaded value makes the in-order load counter wait for every
// load issued before it (the prefetched columns included).
#include <algorithm>

#include "kernels.hpp"
#include "tile.hpp"

namespace bcm {

namespace {

constexpr int P16 = 18 * 18;  // plane stride of the LDS tile

__device__ __forceinline__ int tix16(int i, int j, int k) { return k * P16 + (j + 1) * 18 + (i + 1); }

// LDS position of the halo value lane t stages for face f (faces 0..3; 4,5 stay in registers).
__device__ __forceinline__ int halo16(int f, int t) {
  const int a = t & 15, b = t >> 4;  // (t1, t2) of face f
  switch (f) {
    case 0: return tix16(-1, a, b);
    case 1: return tix16(16, a, b);
    case 2: return tix16(a, -1, b);
    default: return tix16(a, 16, b);
  }
}

template <typename T>
__device__ __forceinline__ T face_get(const T* f, int c, int of, int t1, int t2) {
  return f[(size_t)c * 1536 + of * 256 + t2 * 16 + t1];
}

// Face-buffer offsets of the NQ neighbour values lane t needs on each face (NQ = 1 on
// single-level meshes, 4 where a face may be covered by four finer cubes).  Same-level and
// coarser faces repeat one address; domain-boundary faces point at the cube's own slab (a
// value that staging discards).  Offsets into a fine (16^3) face buffer and into the face
// buffer of the 8^3 level (for prolongated corrections).
template <int NQ>
struct Slots16 {
  int fine[6][NQ];
  int coarse[6][NQ];
  int kind[6];
};

template <int NQ>
__device__ __forceinline__ void slots16(const CubeMeta& m, int self, int t, Slots16<NQ>& S,
                                        bool coarse) {
  const int t1 = t & 15, t2 = t >> 4;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int kd = m.kind[f], of = f ^ 1;
    S.kind[f] = kd;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      int c = self, o = f, a = t1, b = t2;
      if (kd == FK_SAME) {
        c = m.nbr[f][0];
        o = of;
      } else if (kd == FK_COARSER) {
        const int qd = m.quad[f];
        c = m.nbr[f][0];
        o = of;
        a = (qd & 1) * 8 + (t1 >> 1);
        b = (qd >> 1) * 8 + (t2 >> 1);
      } else if (kd == FK_FINER) {
        const int F1 = 2 * t1 + (q & 1), F2 = 2 * t2 + (q >> 1);
        c = m.nbr[f][(F1 >> 4) + 2 * (F2 >> 4)];
        o = of;
        a = F1 & 15;
        b = F2 & 15;
      }
      S.fine[f][q] = c * 1536 + o * 256 + b * 16 + a;
      if (coarse) S.coarse[f][q] = c * 384 + o * 64 + (b >> 1) * 8 + (a >> 1);
    }
  }
}

// Scaled halo value of one face from its raw neighbour values (RULE_P).
template <typename T, int NQ>
__device__ __forceinline__ T halo_val(int kd, const T (&r)[NQ]) {
  T s = r[0];
  if (NQ == 4 && kd == FK_FINER) s = T(0.25) * (((r[0] + r[1]) + r[2]) + r[3]);
  // a select, not a zero scale: the dummy slab of a boundary face may hold anything
  return kd <= FK_FINER ? T(RuleTab<RULE_P>::nbeff(kd)) * s : T(0);
}

// Stage face values: faces 0..3 into the LDS ring at this lane's slot, 4/5 into registers.
template <typename T>
__device__ __forceinline__ void stage16(T* tile, const T (&hv)[6], int t, T& zlo, T& zhi) {
#pragma unroll
  for (int f = 0; f < 4; ++f) tile[halo16(f, t)] = hv[f];
  zlo = hv[4];
  zhi = hv[5];
}

// Diagonal (sum of own coefficients) of the lane's column: cells k = 0, 1..14, 15.
template <typename T>
__device__ __forceinline__ void diag16(const CubeMeta& m, int i, int j, T& d0, T& dm, T& d15) {
  T c = T(6);
  if (i == 0) c += T(RuleTab<RULE_P>::own(m.kind[0])) - T(1);
  if (i == 15) c += T(RuleTab<RULE_P>::own(m.kind[1])) - T(1);
  if (j == 0) c += T(RuleTab<RULE_P>::own(m.kind[2])) - T(1);
  if (j == 15) c += T(RuleTab<RULE_P>::own(m.kind[3])) - T(1);
  dm = c;
  d0 = c + T(RuleTab<RULE_P>::own(m.kind[4])) - T(1);
  d15 = c + T(RuleTab<RULE_P>::own(m.kind[5])) - T(1);
}

// Write the six face slabs of a cube from the lane's column.
template <typename T>
__device__ __forceinline__ void export16(T* xf, int c, const T (&x)[16], int i, int j) {
  T* base = xf + (size_t)c * 1536;
  if (i == 0)
#pragma unroll
    for (int k = 0; k < 16; ++k) base[0 * 256 + k * 16 + j] = x[k];
  if (i == 15)
#pragma unroll
    for (int k = 0; k < 16; ++k) base[1 * 256 + k * 16 + j] = x[k];
  if (j == 0)
#pragma unroll
    for (int k = 0; k < 16; ++k) base[2 * 256 + k * 16 + i] = x[k];
  if (j == 15)
#pragma unroll
    for (int k = 0; k < 16; ++k) base[3 * 256 + k * 16 + i] = x[k];
  base[4 * 256 + j * 16 + i] = x[0];
  base[5 * 256 + j * 16 + i] = x[15];
}

template <typename T>
__device__ __forceinline__ T nbsum16(const T* tile, const T (&x)[16], int k, int c, T zlo, T zhi) {
  const T zm = k > 0 ? x[k > 0 ? k - 1 : 0] : zlo;
  const T zp = k < 15 ? x[k < 15 ? k + 1 : 15] : zhi;
  return tile[c - 1] + tile[c + 1] + tile[c - 18] + tile[c + 18] + zm + zp;
}

// ------------------------------------------------------------------------------------------
// Smoother (see k_smooth): POST = prolongation + post-smoothing (+ fused dots), else
// pre-smoothing from a zero initial guess.
// ------------------------------------------------------------------------------------------
template <typename T, bool POST, int NQ>
__global__ __launch_bounds__(256) void k16_smooth(SmoothArgs<T> a) {
  __shared__ T tile[16 * P16];
  __shared__ double red[8];
  const int t = threadIdx.x, i = t & 15, j = t >> 4;
  const int n = a.g.n_cubes, G = gridDim.x;
  const bool dots = POST && a.part_zr != nullptr;
  int w = blockIdx.x;
  int c = w < n ? a.g.launch[w] : -1;
  T nx[16], nb[16], nxc[8], rf[6][NQ], rc[6][NQ];
  int kinds[6];
  auto fetch = [&](int cc) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const size_t g = (size_t)cc * 4096 + k * 256 + t;
      nb[k] = a.b[g];
      if (POST) nx[k] = a.x[g];
    }
    if (POST) {
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) nxc[kk] = a.xc[(size_t)cc * 512 + (kk * 8 + (j >> 1)) * 8 + (i >> 1)];
      Slots16<NQ> S;
      slots16<NQ>(a.g.meta[cc], cc, t, S, true);
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        kinds[f] = S.kind[f];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          rf[f][q] = a.xf_in[S.fine[f][q]];
          rc[f][q] = a.xcf[S.coarse[f][q]];
        }
      }
    }
  };
  if (c >= 0) fetch(c);
  double zr = 0.0, zq = 0.0;
  while (c >= 0) {
    T x[16], bv[16];
    T zlo = T(0), zhi = T(0);
    const CubeMeta& m = a.g.meta[c];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      x[k] = POST ? nx[k] + nxc[k >> 1] : T(0);
      bv[k] = nb[k];
      tile[tix16(i, j, k)] = x[k];
    }
    if (POST) {
      T hv[6];
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        T r[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) r[q] = rf[f][q] + rc[f][q];
        hv[f] = halo_val<T, NQ>(kinds[f], r);
      }
      stage16<T>(tile, hv, t, zlo, zhi);
    } else {
#pragma unroll
      for (int f = 0; f < 4; ++f) tile[halo16(f, t)] = T(0);
    }
    const T h = T(m.h);
    const T h2 = h * h;
    T d0, dm, d15;
    diag16<T>(m, i, j, d0, dm, d15);
    const T i0 = T(1) / d0, im = T(1) / dm, i15 = T(1) / d15;
    const double vol = m.vol;
    const int wn = w + G;
    const int cn = wn < n ? a.g.launch[wn] : -1;
    __syncthreads();
    if (cn >= 0) fetch(cn);
    // q of this cube for the fused <x, q> (loads overlap the sweeps)
    T q[16];
    if (dots && a.q_dot) {
#pragma unroll
      for (int k = 0; k < 16; ++k) q[k] = a.q_dot[(size_t)c * 4096 + k * 256 + t];
    }
    for (int sw = 0; sw < a.sweeps; ++sw) {
#pragma unroll
      for (int col = 0; col < 2; ++col) {
        const int colour = POST ? (col ^ 1) : col;  // pre: red first, post: black first
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          if (((i + j + k) & 1) != colour) continue;
          const int cc = tix16(i, j, k);
          const T s = nbsum16<T>(tile, x, k, cc, zlo, zhi);
          const T id = k == 0 ? i0 : (k == 15 ? i15 : im);
          x[k] = (s - h2 * bv[k]) * id;
          tile[cc] = x[k];
        }
        __syncthreads();
      }
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const size_t g = (size_t)c * 4096 + k * 256 + t;
      a.x[g] = x[k];
      if (dots) {
        zr += vol * double(x[k]) * double(bv[k]);
        if (a.q_dot) zq += vol * double(x[k]) * double(q[k]);
      }
    }
    export16<T>(a.xf_out, c, x, i, j);
    w = wn;
    c = cn;
  }
  if (dots) {
    const double t0 = block_sum(zr, red);
    __syncthreads();
    const double t1 = block_sum(zq, red);
    if (threadIdx.x == 0) {
      a.part_zr[blockIdx.x] = t0;
      if (a.part_zq) a.part_zq[blockIdx.x] = t1;
      for (int k = blockIdx.x + G; k < fine_grid(n); k += G) {
        a.part_zr[k] = 0.0;
        if (a.part_zq) a.part_zq[k] = 0.0;
      }
    }
  }
}

// Residual of x and restriction to 8^3 (mean of the 8 children).
template <typename T, int NQ>
__global__ __launch_bounds__(256) void k16_restrict(RestrictArgs<T> a) {
  __shared__ T tile[16 * P16];
  __shared__ T rsum[16 * 16 * 8];  // residual summed over k pairs, per (i, j, kk)
  const int t = threadIdx.x, i = t & 15, j = t >> 4;
  const int n = a.g.n_cubes, G = gridDim.x;
  int w = blockIdx.x;
  int c = w < n ? a.g.launch[w] : -1;
  T nx[16], nb[16], rf[6][NQ];
  int kinds[6];
  auto fetch = [&](int cc) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const size_t g = (size_t)cc * 4096 + k * 256 + t;
      nx[k] = a.x[g];
      nb[k] = a.b[g];
    }
    Slots16<NQ> S;
    slots16<NQ>(a.g.meta[cc], cc, t, S, false);
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      kinds[f] = S.kind[f];
#pragma unroll
      for (int q = 0; q < NQ; ++q) rf[f][q] = a.xf[S.fine[f][q]];
    }
  };
  if (c >= 0) fetch(c);
  while (c >= 0) {
    T x[16], bv[16], hv[6];
    T zlo, zhi;
    const CubeMeta& m = a.g.meta[c];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      x[k] = nx[k];
      bv[k] = nb[k];
      tile[tix16(i, j, k)] = x[k];
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) hv[f] = halo_val<T, NQ>(kinds[f], rf[f]);
    stage16<T>(tile, hv, t, zlo, zhi);
    const T h = T(m.h);
    const T ih2 = T(1) / (h * h);
    T d0, dm, d15;
    diag16<T>(m, i, j, d0, dm, d15);
    const int wn = w + G;
    const int cn = wn < n ? a.g.launch[wn] : -1;
    __syncthreads();
    if (cn >= 0) fetch(cn);
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      T acc = T(0);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int k = 2 * kk + q;
        const T d = k == 0 ? d0 : (k == 15 ? d15 : dm);
        const T s = nbsum16<T>(tile, x, k, tix16(i, j, k), zlo, zhi);
        acc += bv[k] - (s - d * x[k]) * ih2;
      }
      rsum[(kk * 16 + j) * 16 + i] = acc;
    }
    __syncthreads();
    // 512 coarse cells: lanes 0..255 take two each; sum the 2x2 (i, j) neighbours
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int e = t + 256 * r;
      const int I = e & 7, J = (e >> 3) & 7, K = e >> 6;
      const T s = rsum[(K * 16 + 2 * J) * 16 + 2 * I] + rsum[(K * 16 + 2 * J) * 16 + 2 * I + 1] +
                  rsum[(K * 16 + 2 * J + 1) * 16 + 2 * I] + rsum[(K * 16 + 2 * J + 1) * 16 + 2 * I + 1];
      a.bc[(size_t)c * 512 + e] = s * T(0.125);
    }
    __syncthreads();
    w = wn;
    c = cn;
  }
}

// p = z + beta p (or z); q = A p; partial <p, q>_V.
template <typename T, int NQ>
__global__ __launch_bounds__(256) void k16_apply(ApplyArgs<T> a) {
  __shared__ T tile[16 * P16];
  __shared__ double red[8];
  const int t = threadIdx.x, i = t & 15, j = t >> 4;
  const int n = a.g.n_cubes, G = gridDim.x;
  const T beta = a.first ? T(0) : T(a.sc->beta);
  int w = blockIdx.x;
  int c = w < n ? a.g.launch[w] : -1;
  T nz[16], np[16], rz[6][NQ], rp[6][NQ];
  int kinds[6];
  auto fetch = [&](int cc) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const size_t g = (size_t)cc * 4096 + k * 256 + t;
      nz[k] = a.z[g];
      np[k] = a.first ? T(0) : a.p[g];
    }
    Slots16<NQ> S;
    slots16<NQ>(a.g.meta[cc], cc, t, S, false);
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      kinds[f] = S.kind[f];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        rz[f][q] = a.zf[S.fine[f][q]];
        rp[f][q] = a.first ? T(0) : a.pf_in[S.fine[f][q]];
      }
    }
  };
  if (c >= 0) fetch(c);
  double pq = 0.0;
  while (c >= 0) {
    T x[16], hv[6];
    T zlo, zhi;
    const CubeMeta& m = a.g.meta[c];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      x[k] = nz[k] + beta * np[k];
      tile[tix16(i, j, k)] = x[k];
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      T r[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) r[q] = rz[f][q] + beta * rp[f][q];
      hv[f] = halo_val<T, NQ>(kinds[f], r);
    }
    stage16<T>(tile, hv, t, zlo, zhi);
    const T h = T(m.h);
    const T ih2 = T(1) / (h * h);
    T d0, dm, d15;
    diag16<T>(m, i, j, d0, dm, d15);
    const double vol = m.vol;
    const int wn = w + G;
    const int cn = wn < n ? a.g.launch[wn] : -1;
    __syncthreads();
    if (cn >= 0) fetch(cn);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const T d = k == 0 ? d0 : (k == 15 ? d15 : dm);
      const T s = nbsum16<T>(tile, x, k, tix16(i, j, k), zlo, zhi);
      const T qv = (s - d * x[k]) * ih2;
      const size_t g = (size_t)c * 4096 + k * 256 + t;
      a.p[g] = x[k];
      a.q[g] = qv;
      pq += vol * double(x[k]) * double(qv);
    }
    export16<T>(a.pf_out, c, x, i, j);
    __syncthreads();
    w = wn;
    c = cn;
  }
  const double tot = block_sum(pq, red);
  if (threadIdx.x == 0) {
    a.part[blockIdx.x] = tot;
    for (int k = blockIdx.x + G; k < fine_grid(n); k += G) a.part[k] = 0.0;
  }
}

// r = b - A p in FP64 (p may be nullptr = 0; b may be nullptr -> r = A p), stored as TO * rscale.
template <typename TO, int NQ>
__global__ __launch_bounds__(256) void k16_resid64(Resid64Args<TO> a) {
  __shared__ double tile[16 * P16];
  __shared__ double red[8];
  const int t = threadIdx.x, i = t & 15, j = t >> 4;
  const int n = a.g.n_cubes, G = gridDim.x;
  int w = blockIdx.x;
  int c = w < n ? a.g.launch[w] : -1;
  double np[16], nb[16], rf[6][NQ];
  int kinds[6];
  auto fetch = [&](int cc) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const size_t g = (size_t)cc * 4096 + k * 256 + t;
      np[k] = a.p ? a.p[g] : 0.0;
      nb[k] = a.b ? a.b[g] : 0.0;
    }
    Slots16<NQ> S;
    slots16<NQ>(a.g.meta[cc], cc, t, S, false);
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      kinds[f] = S.kind[f];
#pragma unroll
      for (int q = 0; q < NQ; ++q) rf[f][q] = a.p ? a.pf[S.fine[f][q]] : 0.0;
    }
  };
  if (c >= 0) fetch(c);
  double rr = 0.0, bb = 0.0;
  while (c >= 0) {
    double x[16], bv[16], hv[6];
    double zlo, zhi;
    const CubeMeta& m = a.g.meta[c];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      x[k] = np[k];
      bv[k] = nb[k];
      tile[tix16(i, j, k)] = x[k];
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) hv[f] = halo_val<double, NQ>(kinds[f], rf[f]);
    stage16<double>(tile, hv, t, zlo, zhi);
    const double h = m.h;
    const double ih2 = 1.0 / (h * h);
    double d0, dm, d15;
    diag16<double>(m, i, j, d0, dm, d15);
    const double vol = m.vol;
    const int wn = w + G;
    const int cn = wn < n ? a.g.launch[wn] : -1;
    __syncthreads();
    if (cn >= 0) fetch(cn);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const double d = k == 0 ? d0 : (k == 15 ? d15 : dm);
      const double s = nbsum16<double>(tile, x, k, tix16(i, j, k), zlo, zhi);
      const double ap = (s - d * x[k]) * ih2;
      double r;
      if (a.b) {
        r = bv[k] - ap;
        bb += vol * bv[k] * bv[k];
      } else {
        r = ap;
      }
      rr += vol * r * r;
      a.r[(size_t)c * 4096 + k * 256 + t] = TO(r * a.rscale);
    }
    __syncthreads();
    w = wn;
    c = cn;
  }
  if (a.part_rr) {
    const double t0 = block_sum(rr, red);
    __syncthreads();
    const double t1 = block_sum(bb, red);
    if (threadIdx.x == 0) {
      a.part_rr[blockIdx.x] = t0;
      if (a.part_bb) a.part_bb[blockIdx.x] = t1;
      for (int k = blockIdx.x + G; k < fine_grid(n); k += G) {
        a.part_rr[k] = 0.0;
        if (a.part_bb) a.part_bb[k] = 0.0;
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// Projection step on 16^3 cubes (see kernels_proj.hip for the general-level versions).
// ------------------------------------------------------------------------------------------

// u* = (1 - alpha) u~ + alpha u_s, and the face-normal component of u* on each face.
template <typename TF>
__global__ __launch_bounds__(256) void k16_force(ForceArgs<TF> a) {
  const int t = threadIdx.x, i = t & 15, j = t >> 4;
  const int n = a.g.n_cubes;
  for (int w = blockIdx.x; w < n; w += gridDim.x) {
    const int c = a.g.launch[w];
    TF al[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) al[k] = a.alpha ? a.alpha[(size_t)c * 4096 + k * 256 + t] : TF(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      TF v[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const size_t g = (size_t)c * 4096 + k * 256 + t;
        const TF ut = a.u[d][g];
        const TF us = a.us[d] ? a.us[d][g] : TF(a.usc[d]);
        v[k] = a.alpha ? (TF(1) - al[k]) * ut + al[k] * us : ut;
        a.ustar[d][g] = v[k];
      }
      TF* base = a.uf + (size_t)c * 1536;
      if (d == 0) {
        if (i == 0)
#pragma unroll
          for (int k = 0; k < 16; ++k) base[0 * 256 + k * 16 + j] = v[k];
        if (i == 15)
#pragma unroll
          for (int k = 0; k < 16; ++k) base[1 * 256 + k * 16 + j] = v[k];
      } else if (d == 1) {
        if (j == 0)
#pragma unroll
          for (int k = 0; k < 16; ++k) base[2 * 256 + k * 16 + i] = v[k];
        if (j == 15)
#pragma unroll
          for (int k = 0; k < 16; ++k) base[3 * 256 + k * 16 + i] = v[k];
      } else {
        base[4 * 256 + j * 16 + i] = v[0];
        base[5 * 256 + j * 16 + i] = v[15];
      }
    }
  }
}

// b = (rho/dt) div U*, U* = face-normal velocity (RULE_U interpolation at the cube faces).
template <typename TF>
__global__ __launch_bounds__(256) void k16_div(DivArgs<TF> a) {
  __shared__ TF tile[16 * P16];
  const int t = threadIdx.x, i = t & 15, j = t >> 4;
  const int n = a.g.n_cubes;
  const int t1 = t & 15, t2 = t >> 4;
  for (int w = blockIdx.x; w < n; w += gridDim.x) {
    const int c = a.g.launch[w];
    const CubeMeta& m = a.g.meta[c];
    const double ih = 1.0 / m.h;
    double acc[16];
    const auto gf = [&](int cc, int of, int aa, int bb) { return face_get(a.uf, cc, of, aa, bb); };
    // z component: neighbours along k are this lane's registers
    {
      TF v[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) v[k] = a.ustar[2][(size_t)c * 4096 + k * 256 + t];
      double lo, hi;  // face velocities on the -z and +z faces of the column
      {
        const int k4 = m.kind[4], k5 = m.kind[5];
        const double r4 = k4 <= FK_FINER ? RuleTab<RULE_U>::nbeff(k4) * double(nb_raw<16, TF>(m, 4, t1, t2, gf)) : 0.0;
        const double r5 = k5 <= FK_FINER ? RuleTab<RULE_U>::nbeff(k5) * double(nb_raw<16, TF>(m, 5, t1, t2, gf)) : 0.0;
        lo = 0.5 * (k4 == FK_INFLOW ? 2.0 * a.U_in : r4) + RuleTab<RULE_U>::own(k4) * double(v[0]);
        hi = 0.5 * (k5 == FK_INFLOW ? -2.0 * a.U_in : r5) + RuleTab<RULE_U>::own(k5) * double(v[15]);
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const double up = k < 15 ? 0.5 * (double(v[k]) + double(v[k < 15 ? k + 1 : 15])) : hi;
        const double um = k > 0 ? 0.5 * (double(v[k > 0 ? k - 1 : 0]) + double(v[k])) : lo;
        acc[k] = up - um;
      }
    }
    // x and y components through the LDS plane tile
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      TF v[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        v[k] = a.ustar[d][(size_t)c * 4096 + k * 256 + t];
        tile[tix16(i, j, k)] = v[k];
      }
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int f = 2 * d + s;
        const int kd = m.kind[f];
        TF hv = TF(0);
        if (kd <= FK_FINER) hv = TF(RuleTab<RULE_U>::nbeff(kd)) * nb_raw<16, TF>(m, f, t1, t2, gf);
        else if (kd == FK_INFLOW) hv = TF(2.0 * (s ? -a.U_in : a.U_in));
        tile[halo16(f, t)] = hv;
      }
      __syncthreads();
      const int st = d == 0 ? 1 : 18;
      const double own_m = (d == 0 ? i == 0 : j == 0) ? RuleTab<RULE_U>::own(m.kind[2 * d]) : 0.5;
      const double own_p = (d == 0 ? i == 15 : j == 15) ? RuleTab<RULE_U>::own(m.kind[2 * d + 1]) : 0.5;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int cc = tix16(i, j, k);
        const double up = 0.5 * double(tile[cc + st]) + own_p * double(v[k]);
        const double um = 0.5 * double(tile[cc - st]) + own_m * double(v[k]);
        acc[k] += up - um;
      }
      __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) a.b[(size_t)c * 4096 + k * 256 + t] = acc[k] * ih * a.inv_c;
  }
}

// u_new = u* - c G_c p (cell velocities only; the face-velocity output uses k_correct).
template <typename TF, int NQ>
__global__ __launch_bounds__(256) void k16_correct(CorrectArgs<TF> a) {
  __shared__ double tile[16 * P16];
  const int t = threadIdx.x, i = t & 15, j = t >> 4;
  const int n = a.g.n_cubes;
  for (int w = blockIdx.x; w < n; w += gridDim.x) {
    const int c = a.g.launch[w];
    const CubeMeta& m = a.g.meta[c];
    double p[16], hv[6], rf[6][NQ];
    double zlo, zhi;
    Slots16<NQ> S;
    slots16<NQ>(m, c, t, S, false);
#pragma unroll
    for (int f = 0; f < 6; ++f)
#pragma unroll
      for (int q = 0; q < NQ; ++q) rf[f][q] = a.pf[S.fine[f][q]];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      p[k] = a.p[(size_t)c * 4096 + k * 256 + t];
      tile[tix16(i, j, k)] = p[k];
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) hv[f] = halo_val<double, NQ>(S.kind[f], rf[f]);
    stage16<double>(tile, hv, t, zlo, zhi);
    __syncthreads();
    const double ch = a.c * 0.5 / m.h;
    const double ox_m = i == 0 ? RuleTab<RULE_P>::own(m.kind[0]) : 1.0;
    const double ox_p = i == 15 ? RuleTab<RULE_P>::own(m.kind[1]) : 1.0;
    const double oy_m = j == 0 ? RuleTab<RULE_P>::own(m.kind[2]) : 1.0;
    const double oy_p = j == 15 ? RuleTab<RULE_P>::own(m.kind[3]) : 1.0;
    const double oz_m = RuleTab<RULE_P>::own(m.kind[4]), oz_p = RuleTab<RULE_P>::own(m.kind[5]);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int cc = tix16(i, j, k);
      const size_t g = (size_t)c * 4096 + k * 256 + t;
      const double gx = (tile[cc + 1] - ox_p * p[k]) - (tile[cc - 1] - ox_m * p[k]);
      const double gy = (tile[cc + 18] - oy_p * p[k]) - (tile[cc - 18] - oy_m * p[k]);
      const double zp = k < 15 ? p[k < 15 ? k + 1 : 15] - p[k] : zhi - oz_p * p[k];
      const double zm = k > 0 ? p[k > 0 ? k - 1 : 0] - p[k] : zlo - oz_m * p[k];
      if (a.unew[0]) a.unew[0][g] = TF(double(a.ustar[0][g]) - ch * gx);
      if (a.unew[1]) a.unew[1][g] = TF(double(a.ustar[1][g]) - ch * gy);
      if (a.unew[2]) a.unew[2][g] = TF(double(a.ustar[2][g]) - ch * (zp - zm));
    }
    __syncthreads();
  }
}

}  // namespace

// Persistent grid of one kernel: every workgroup resident at once (CUs x occupancy), rounded
// down to a multiple of 8 so each workgroup keeps to one XCD's stretch of the launch table.
static int grid_for(const void* fn, int n_cubes) {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 256;
  }
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, 256, 0) != hipSuccess || per < 1) per = 1;
  int g = cus * per;
  if (g >= 8) g -= g % 8;
  return std::max(1, std::min(g, fine_grid(n_cubes)));
}

#define BCM_LAUNCH16(KERNEL, ARGS)                                                        \
  do {                                                                                    \
    const void* fn = reinterpret_cast<const void*>(&KERNEL);                              \
    hipLaunchKernelGGL((KERNEL), dim3(grid_for(fn, ARGS.g.n_cubes)), dim3(256), 0, s, ARGS); \
  } while (0)

template <typename T>
hipError_t launch16_smooth(const SmoothArgs<T>& a, hipStream_t s) {
  if (a.zero_init) {
    BCM_LAUNCH16((k16_smooth<T, false, 1>), a);
  } else if (a.g.multilevel) {
    BCM_LAUNCH16((k16_smooth<T, true, 4>), a);
  } else {
    BCM_LAUNCH16((k16_smooth<T, true, 1>), a);
  }
  return hipGetLastError();
}
template <typename T>
hipError_t launch16_restrict(const RestrictArgs<T>& a, hipStream_t s) {
  if (a.g.multilevel)
    BCM_LAUNCH16((k16_restrict<T, 4>), a);
  else
    BCM_LAUNCH16((k16_restrict<T, 1>), a);
  return hipGetLastError();
}
template <typename T>
hipError_t launch16_apply(const ApplyArgs<T>& a, hipStream_t s) {
  if (a.g.multilevel)
    BCM_LAUNCH16((k16_apply<T, 4>), a);
  else
    BCM_LAUNCH16((k16_apply<T, 1>), a);
  return hipGetLastError();
}
template <typename TO>
hipError_t launch16_resid64(const Resid64Args<TO>& a, hipStream_t s) {
  if (a.g.multilevel)
    BCM_LAUNCH16((k16_resid64<TO, 4>), a);
  else
    BCM_LAUNCH16((k16_resid64<TO, 1>), a);
  return hipGetLastError();
}
template <typename TF>
hipError_t launch16_force(const ForceArgs<TF>& a, hipStream_t s) {
  hipLaunchKernelGGL((k16_force<TF>), dim3(std::min(a.g.n_cubes, 2048)), dim3(256), 0, s, a);
  return hipGetLastError();
}
template <typename TF>
hipError_t launch16_div(const DivArgs<TF>& a, hipStream_t s) {
  hipLaunchKernelGGL((k16_div<TF>), dim3(std::min(a.g.n_cubes, 2048)), dim3(256), 0, s, a);
  return hipGetLastError();
}
template <typename TF>
hipError_t launch16_correct(const CorrectArgs<TF>& a, hipStream_t s) {
  if (a.g.multilevel)
    hipLaunchKernelGGL((k16_correct<TF, 4>), dim3(std::min(a.g.n_cubes, 2048)), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k16_correct<TF, 1>), dim3(std::min(a.g.n_cubes, 2048)), dim3(256), 0, s, a);
  return hipGetLastError();
}

#define BCM_INST16(T)                                                             \
  template hipError_t launch16_smooth<T>(const SmoothArgs<T>&, hipStream_t);      \
  template hipError_t launch16_restrict<T>(const RestrictArgs<T>&, hipStream_t);  \
  template hipError_t launch16_apply<T>(const ApplyArgs<T>&, hipStream_t);        \
  template hipError_t launch16_resid64<T>(const Resid64Args<T>&, hipStream_t);    \
  template hipError_t launch16_force<T>(const ForceArgs<T>&, hipStream_t);        \
  template hipError_t launch16_div<T>(const DivArgs<T>&, hipStream_t);            \
  template hipError_t launch16_correct<T>(const CorrectArgs<T>&, hipStream_t);
BCM_INST16(float)
BCM_INST16(double)

}  // namespace bcm
