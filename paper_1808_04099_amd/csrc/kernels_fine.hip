// Finest-level (16^3 cells per cube) stencil kernels: the HBM-bound part of the Poisson solve.
//
// Layout per workgroup (256 lanes): lane t owns the column (i = t & 15, j = t >> 4) of a
// cube, k = 0..15 held in registers.  Only the i/j neighbours go through LDS: a tile of 16
// planes of 18 x 18 (the cube's plane plus its x/y halo ring); the z neighbours are the
// lane's own registers, with the z halo of the column in two registers.  Every global
// access is a full 1 KB plane (coalesced) or a 1 KB face slab.
//
// The kernels are persistent: a workgroup walks the Z-ordered launch table with stride
// gridDim.x (a multiple of 8, so each workgroup stays on the XCD that owns its stretch of
// the curve) and, while it computes one cube, the loads of its next cube are in flight
// (registers, consumed at the top of the next iteration; barriers only wait for LDS).
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

// Raw neighbour values across the 6 faces at this lane's face position (t & 15, t >> 4),
// optionally plus the coarse correction of the neighbour (prolongation).
template <typename T>
__device__ __forceinline__ void load_halo16(T (&h)[6], const CubeMeta& m, const T* xf,
                                            const T* xcf, int t) {
  const int t1 = t & 15, t2 = t >> 4;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    if (xcf)
      h[f] = nb_raw<16, T>(m, f, t1, t2, [&](int c, int of, int a, int b) {
        T v = xf ? face_get(xf, c, of, a, b) : T(0);
        return v + xcf[(size_t)c * 6 * 64 + of * 64 + (b >> 1) * 8 + (a >> 1)];
      });
    else
      h[f] = nb_raw<16, T>(m, f, t1, t2, [&](int c, int of, int a, int b) { return face_get(xf, c, of, a, b); });
  }
}

// Stage the halo (already raw neighbour values) into LDS / z registers with the RULE_P scale.
template <typename T>
__device__ __forceinline__ void stage_halo16(T* tile, const T (&h)[6], const CubeMeta& m, int t,
                                             T& zlo, T& zhi) {
#pragma unroll
  for (int f = 0; f < 4; ++f) tile[halo16(f, t)] = T(RuleTab<RULE_P>::nbeff(m.kind[f])) * h[f];
  zlo = T(RuleTab<RULE_P>::nbeff(m.kind[4])) * h[4];
  zhi = T(RuleTab<RULE_P>::nbeff(m.kind[5])) * h[5];
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

// Write the six face slabs of a cube from the lane's column (x is the column, tile holds it).
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
template <typename T, bool POST>
__global__ __launch_bounds__(256) void k16_smooth(SmoothArgs<T> a) {
  __shared__ T tile[16 * P16];
  __shared__ double red[8];
  const int t = threadIdx.x, i = t & 15, j = t >> 4;
  const int n = a.g.n_cubes, G = gridDim.x;
  const bool dots = POST && a.part_zr != nullptr;
  int w = blockIdx.x;
  int c = w < n ? a.g.launch[w] : -1;
  T nx[16], nb[16], nxc[8], nh[6];
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
      load_halo16<T>(nh, a.g.meta[cc], a.xf_in, a.xcf, t);
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
      stage_halo16<T>(tile, nh, m, t, zlo, zhi);
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
    const int sweeps = a.sweeps;
    for (int sw = 0; sw < sweeps; ++sw) {
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
template <typename T>
__global__ __launch_bounds__(256) void k16_restrict(RestrictArgs<T> a) {
  __shared__ T tile[16 * P16];
  __shared__ T rsum[16 * 16 * 8];  // residual summed over k pairs, per (i, j, kk)
  const int t = threadIdx.x, i = t & 15, j = t >> 4;
  const int n = a.g.n_cubes, G = gridDim.x;
  int w = blockIdx.x;
  int c = w < n ? a.g.launch[w] : -1;
  T nx[16], nb[16], nh[6];
  auto fetch = [&](int cc) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const size_t g = (size_t)cc * 4096 + k * 256 + t;
      nx[k] = a.x[g];
      nb[k] = a.b[g];
    }
    load_halo16<T>(nh, a.g.meta[cc], a.xf, (const T*)nullptr, t);
  };
  if (c >= 0) fetch(c);
  while (c >= 0) {
    T x[16], bv[16];
    T zlo, zhi;
    const CubeMeta& m = a.g.meta[c];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      x[k] = nx[k];
      bv[k] = nb[k];
      tile[tix16(i, j, k)] = x[k];
    }
    stage_halo16<T>(tile, nh, m, t, zlo, zhi);
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
template <typename T>
__global__ __launch_bounds__(256) void k16_apply(ApplyArgs<T> a) {
  __shared__ T tile[16 * P16];
  __shared__ double red[8];
  const int t = threadIdx.x, i = t & 15, j = t >> 4;
  const int n = a.g.n_cubes, G = gridDim.x;
  const T beta = a.first ? T(0) : T(a.sc->beta);
  int w = blockIdx.x;
  int c = w < n ? a.g.launch[w] : -1;
  T nz[16], np[16], nh[6];
  auto fetch = [&](int cc) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const size_t g = (size_t)cc * 4096 + k * 256 + t;
      nz[k] = a.z[g];
      np[k] = a.first ? T(0) : a.p[g];
    }
    const int t1 = t & 15, t2 = t >> 4;
    const CubeMeta& mm = a.g.meta[cc];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      if (a.first)
        nh[f] = nb_raw<16, T>(mm, f, t1, t2, [&](int c2, int of, int aa, int bb) { return face_get(a.zf, c2, of, aa, bb); });
      else
        nh[f] = nb_raw<16, T>(mm, f, t1, t2, [&](int c2, int of, int aa, int bb) {
          return face_get(a.zf, c2, of, aa, bb) + beta * face_get(a.pf_in, c2, of, aa, bb);
        });
    }
  };
  if (c >= 0) fetch(c);
  double pq = 0.0;
  while (c >= 0) {
    T x[16];
    T zlo, zhi;
    const CubeMeta& m = a.g.meta[c];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      x[k] = nz[k] + beta * np[k];
      tile[tix16(i, j, k)] = x[k];
    }
    stage_halo16<T>(tile, nh, m, t, zlo, zhi);
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
template <typename TO>
__global__ __launch_bounds__(256) void k16_resid64(Resid64Args<TO> a) {
  __shared__ double tile[16 * P16];
  __shared__ double red[8];
  const int t = threadIdx.x, i = t & 15, j = t >> 4;
  const int n = a.g.n_cubes, G = gridDim.x;
  int w = blockIdx.x;
  int c = w < n ? a.g.launch[w] : -1;
  double np[16], nb[16], nh[6];
  auto fetch = [&](int cc) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const size_t g = (size_t)cc * 4096 + k * 256 + t;
      np[k] = a.p ? a.p[g] : 0.0;
      nb[k] = a.b ? a.b[g] : 0.0;
    }
    if (a.p) {
      load_halo16<double>(nh, a.g.meta[cc], a.pf, (const double*)nullptr, t);
    } else {
#pragma unroll
      for (int f = 0; f < 6; ++f) nh[f] = 0.0;
    }
  };
  if (c >= 0) fetch(c);
  double rr = 0.0, bb = 0.0;
  while (c >= 0) {
    double x[16], bv[16];
    double zlo, zhi;
    const CubeMeta& m = a.g.meta[c];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      x[k] = np[k];
      bv[k] = nb[k];
      tile[tix16(i, j, k)] = x[k];
    }
    stage_halo16<double>(tile, nh, m, t, zlo, zhi);
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

template <typename T>
hipError_t launch16_smooth(const SmoothArgs<T>& a, hipStream_t s) {
  if (a.zero_init) {
    const void* fn = reinterpret_cast<const void*>(&k16_smooth<T, false>);
    hipLaunchKernelGGL((k16_smooth<T, false>), dim3(grid_for(fn, a.g.n_cubes)), dim3(256), 0, s, a);
  } else {
    const void* fn = reinterpret_cast<const void*>(&k16_smooth<T, true>);
    hipLaunchKernelGGL((k16_smooth<T, true>), dim3(grid_for(fn, a.g.n_cubes)), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}
template <typename T>
hipError_t launch16_restrict(const RestrictArgs<T>& a, hipStream_t s) {
  const void* fn = reinterpret_cast<const void*>(&k16_restrict<T>);
  hipLaunchKernelGGL((k16_restrict<T>), dim3(grid_for(fn, a.g.n_cubes)), dim3(256), 0, s, a);
  return hipGetLastError();
}
template <typename T>
hipError_t launch16_apply(const ApplyArgs<T>& a, hipStream_t s) {
  const void* fn = reinterpret_cast<const void*>(&k16_apply<T>);
  hipLaunchKernelGGL((k16_apply<T>), dim3(grid_for(fn, a.g.n_cubes)), dim3(256), 0, s, a);
  return hipGetLastError();
}
template <typename TO>
hipError_t launch16_resid64(const Resid64Args<TO>& a, hipStream_t s) {
  const void* fn = reinterpret_cast<const void*>(&k16_resid64<TO>);
  hipLaunchKernelGGL((k16_resid64<TO>), dim3(grid_for(fn, a.g.n_cubes)), dim3(256), 0, s, a);
  return hipGetLastError();
}

#define BCM_INST16(T)                                                             \
  template hipError_t launch16_smooth<T>(const SmoothArgs<T>&, hipStream_t);      \
  template hipError_t launch16_restrict<T>(const RestrictArgs<T>&, hipStream_t);  \
  template hipError_t launch16_apply<T>(const ApplyArgs<T>&, hipStream_t);        \
  template hipError_t launch16_resid64<T>(const Resid64Args<T>&, hipStream_t);
BCM_INST16(float)
BCM_INST16(double)

}  // namespace bcm
