// Projection-step kernels (Sec. 3 of the paper) and their transposes.
//
//   k_force   immersed-body forcing in volume-fraction form: the constraint force
//             f = (rho/dt) alpha (u_s - u~) added over one step gives u* = (1-alpha) u~ + alpha u_s;
//             also exports the face-normal component of u* on each cube face.
//   k_div     Poisson right-hand side b = (rho/dt) div(U*), U* = face-normal velocity by linear
//             interpolation (inflow / slip / open boundary values, 2:1 interface weights).
//   k_correct velocity correction u^{n+1} = u* - (dt/rho) G_c p (G_c = mean of the two face
//             gradients per axis) and, optionally, face velocities U* - (dt/rho) G p.
//   k_adj_gp  transpose of the correction: g_p = -(dt/rho) G^T G_c^T g_u (+ incoming g_p).
//   k_adj_rhs transpose of the right-hand side and the forcing: g_u* = g_u + (rho/dt) W^T D^T lam,
//             g_u~ = (1 - alpha) g_u*, g_alpha = sum_d g_u*_d (u_s,d - u~_d), g_U_in.
// One workgroup per cube (or several small cubes), LDS tiles as in tile.hpp.
#include "kernels.hpp"
#include "tile.hpp"

namespace bcm {

namespace {

template <typename T>
struct BcInflow {  // face-normal velocity prescribed on inflow faces (stored / int_scale = 0.5)
  double U_in;
  __device__ T operator()(const CubeMeta& m, int f) const {
    if (m.kind[f] != FK_INFLOW) return T(0);
    return T(2.0 * ((f & 1) ? -U_in : U_in));
  }
};

template <int NL>
__device__ __forceinline__ int axis_stride(int d) {
  constexpr int T1 = NL + 2;
  return d == 0 ? 1 : d == 1 ? T1 : T1 * T1;
}

template <int NL>
__device__ __forceinline__ int axis_coord(int d, int i, int j, int k) {
  return d == 0 ? i : d == 1 ? j : k;
}

template <int NL, typename TF>
__global__ __launch_bounds__(256) void k_force(ForceArgs<TF> a) {
  using L = Lv<NL>;
  __shared__ CubeMeta sm[L::CPB];
  __shared__ int cube[L::CPB];
  __shared__ TF tile[L::CPB * L::TILE];
  load_meta<NL>(sm, cube, a.g.meta, a.g.launch, a.g.n_cubes);
  for (int d = 0; d < 3; ++d) {
    for (int e = threadIdx.x; e < L::CPB * L::N3; e += WG) {
      int s, i, j, k;
      cell_of<NL>(e, s, i, j, k);
      const int c = cube[s];
      if (c < 0) continue;
      const size_t g = (size_t)c * L::N3 + (e - s * L::N3);
      const TF ut = a.u[d][g];
      TF v = ut;
      if (a.alpha) {
        const TF al = a.alpha[g];
        const TF us = a.us[d] ? a.us[d][g] : TF(a.usc[d]);
        v = (TF(1) - al) * ut + al * us;
      }
      a.ustar[d][g] = v;
      tile[s * L::TILE + ti<NL>(i, j, k)] = v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < L::CPB * 2 * L::N2; e += WG) {
      const int s = e / (2 * L::N2);
      const int r = e - s * 2 * L::N2;
      const int f = 2 * d + r / L::N2, t = r % L::N2;
      if (cube[s] < 0) continue;
      int i, j, k;
      face_cell<NL>(f, t % NL, t / NL, i, j, k);
      a.uf[(size_t)cube[s] * L::FACE + f * L::N2 + t] = tile[s * L::TILE + ti<NL>(i, j, k)];
    }
    __syncthreads();
  }
}

template <int NL, typename TF>
__global__ __launch_bounds__(256) void k_div(DivArgs<TF> a) {
  using L = Lv<NL>;
  constexpr int R = (L::CPB * L::N3 + WG - 1) / WG;
  __shared__ CubeMeta sm[L::CPB];
  __shared__ int cube[L::CPB];
  __shared__ TF tile[L::CPB * L::TILE];
  __shared__ double red[8];
  load_meta<NL>(sm, cube, a.g.meta, a.g.launch, a.g.n_cubes);
  double acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.0;
  for (int d = 0; d < 3; ++d) {
    for (int e = threadIdx.x; e < L::CPB * L::N3; e += WG) {
      int s, i, j, k;
      cell_of<NL>(e, s, i, j, k);
      const int c = cube[s];
      if (c < 0) continue;
      tile[s * L::TILE + ti<NL>(i, j, k)] = a.ustar[d][(size_t)c * L::N3 + (e - s * L::N3)];
    }
    fill_halo<NL, RULE_U, TF>(tile, sm, cube, FaceGet<NL, TF>{a.uf}, BcInflow<TF>{a.U_in},
                              3 << (2 * d));
    __syncthreads();
    const int st = axis_stride<NL>(d);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int e = threadIdx.x + r * WG;
      if (e >= L::CPB * L::N3) continue;
      int s, i, j, k;
      cell_of<NL>(e, s, i, j, k);
      if (cube[s] < 0) continue;
      const CubeMeta& m = sm[s];
      const TF* t = tile + s * L::TILE;
      const int c = ti<NL>(i, j, k);
      const double u = t[c];
      const double up = 0.5 * double(t[c + st]) + side_own<NL, RULE_U>(m, 2 * d + 1, i, j, k) * u;
      const double um = 0.5 * double(t[c - st]) + side_own<NL, RULE_U>(m, 2 * d, i, j, k) * u;
      acc[r] += (up - um) / m.h;
    }
    __syncthreads();
  }
  double bb = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int e = threadIdx.x + r * WG;
    if (e >= L::CPB * L::N3) continue;
    int s, i, j, k;
    cell_of<NL>(e, s, i, j, k);
    const int c = cube[s];
    if (c < 0) continue;
    const double b = acc[r] * a.inv_c;
    a.b[(size_t)c * L::N3 + (e - s * L::N3)] = b;
    bb += sm[s].vol * b * b;
  }
  if (a.part_bb) {
    const double t = block_sum(bb, red);
    if (threadIdx.x == 0) a.part_bb[blockIdx.x] = t;
  }
}

template <int NL, typename TF>
__global__ __launch_bounds__(256) void k_correct(CorrectArgs<TF> a) {
  using L = Lv<NL>;
  __shared__ CubeMeta sm[L::CPB];
  __shared__ int cube[L::CPB];
  __shared__ double tp[L::CPB * L::TILE];
  __shared__ TF tu[L::CPB * L::TILE];
  load_meta<NL>(sm, cube, a.g.meta, a.g.launch, a.g.n_cubes);
  for (int e = threadIdx.x; e < L::CPB * L::N3; e += WG) {
    int s, i, j, k;
    cell_of<NL>(e, s, i, j, k);
    const int c = cube[s];
    if (c < 0) continue;
    tp[s * L::TILE + ti<NL>(i, j, k)] = a.p[(size_t)c * L::N3 + (e - s * L::N3)];
  }
  fill_halo<NL, RULE_P, double>(tp, sm, cube, FaceGet<NL, double>{a.pf}, BcZero<double>{});
  __syncthreads();
  for (int d = 0; d < 3; ++d) {
    const int st = axis_stride<NL>(d);
    for (int e = threadIdx.x; e < L::CPB * L::N3; e += WG) {
      int s, i, j, k;
      cell_of<NL>(e, s, i, j, k);
      const int cb = cube[s];
      if (cb < 0) continue;
      const CubeMeta& m = sm[s];
      const double* t = tp + s * L::TILE;
      const int c = ti<NL>(i, j, k);
      const double p = t[c];
      const double dp = (t[c + st] - side_own<NL, RULE_P>(m, 2 * d + 1, i, j, k) * p) / m.h;
      const double dm = (t[c - st] - side_own<NL, RULE_P>(m, 2 * d, i, j, k) * p) / m.h;
      const size_t g = (size_t)cb * L::N3 + (e - s * L::N3);
      if (a.unew[d]) a.unew[d][g] = TF(double(a.ustar[d][g]) - a.c * 0.5 * (dp - dm));
    }
    if (!a.face_u[d]) continue;
    // face velocities along axis d: U* by interpolation, minus c times the face gradient
    for (int e = threadIdx.x; e < L::CPB * L::N3; e += WG) {
      int s, i, j, k;
      cell_of<NL>(e, s, i, j, k);
      if (cube[s] < 0) continue;
      tu[s * L::TILE + ti<NL>(i, j, k)] = a.ustar[d][(size_t)cube[s] * L::N3 + (e - s * L::N3)];
    }
    fill_halo<NL, RULE_U, TF>(tu, sm, cube, FaceGet<NL, TF>{a.uf}, BcInflow<TF>{a.U_in},
                              3 << (2 * d));
    __syncthreads();
    constexpr int NF = (NL + 1) * NL * NL;
    for (int e = threadIdx.x; e < L::CPB * NF; e += WG) {
      const int s = e / NF;
      const int r = e - s * NF;
      if (cube[s] < 0) continue;
      const CubeMeta& m = sm[s];
      // decode (i, j, k) with NL + 1 entries along axis d
      const int ex = d == 0 ? NL + 1 : NL, ey = d == 1 ? NL + 1 : NL;
      const int i = r % ex, j = (r / ex) % ey, k = r / (ex * ey);
      const int l = axis_coord<NL>(d, i, j, k);  // face index along d: between cells l-1 and l
      const int ic = d == 0 ? (l == NL ? NL - 1 : i) : i;
      const int jc = d == 1 ? (l == NL ? NL - 1 : j) : j;
      const int kc = d == 2 ? (l == NL ? NL - 1 : k) : k;
      const double* t = tp + s * L::TILE;
      const TF* u = tu + s * L::TILE;
      double Us, grad;
      if (l == NL) {  // + face of the last cell
        const int c = ti<NL>(ic, jc, kc);
        const double p = t[c], uu = u[c];
        Us = 0.5 * double(u[c + st]) + side_own<NL, RULE_U>(m, 2 * d + 1, ic, jc, kc) * uu;
        grad = (t[c + st] - side_own<NL, RULE_P>(m, 2 * d + 1, ic, jc, kc) * p) / m.h;
      } else if (l == 0) {  // - face of the first cell
        const int c = ti<NL>(ic, jc, kc);
        const double p = t[c], uu = u[c];
        Us = 0.5 * double(u[c - st]) + side_own<NL, RULE_U>(m, 2 * d, ic, jc, kc) * uu;
        grad = -(t[c - st] - side_own<NL, RULE_P>(m, 2 * d, ic, jc, kc) * p) / m.h;
      } else {
        const int c = ti<NL>(ic, jc, kc);
        Us = 0.5 * (double(u[c]) + double(u[c - st]));
        grad = (t[c] - t[c - st]) / m.h;
      }
      a.face_u[d][(size_t)cube[s] * NF + r] = TF(Us - a.c * grad);
    }
    __syncthreads();
  }
}

template <int NL, typename TF>
__global__ __launch_bounds__(256) void k_adj_gp(AdjGpArgs<TF> a) {
  using L = Lv<NL>;
  constexpr int R = (L::CPB * L::N3 + WG - 1) / WG;
  __shared__ CubeMeta sm[L::CPB];
  __shared__ int cube[L::CPB];
  __shared__ TF tile[L::CPB * L::TILE];
  load_meta<NL>(sm, cube, a.g.meta, a.g.launch, a.g.n_cubes);
  double acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.0;
  for (int d = 0; d < 3; ++d) {
    for (int e = threadIdx.x; e < L::CPB * L::N3; e += WG) {
      int s, i, j, k;
      cell_of<NL>(e, s, i, j, k);
      const int c = cube[s];
      if (c < 0) continue;
      tile[s * L::TILE + ti<NL>(i, j, k)] = a.v[d][(size_t)c * L::N3 + (e - s * L::N3)];
    }
    fill_halo<NL, RULE_V, TF>(tile, sm, cube, FaceGet<NL, TF>{a.vf}, BcZero<TF>{}, 3 << (2 * d));
    __syncthreads();
    const int st = axis_stride<NL>(d);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int e = threadIdx.x + r * WG;
      if (e >= L::CPB * L::N3) continue;
      int s, i, j, k;
      cell_of<NL>(e, s, i, j, k);
      if (cube[s] < 0) continue;
      const CubeMeta& m = sm[s];
      const TF* t = tile + s * L::TILE;
      const int c = ti<NL>(i, j, k);
      const double v = t[c];
      const double tp = side_own<NL, RULE_V>(m, 2 * d + 1, i, j, k) * v + 0.5 * double(t[c + st]);
      const double tm = side_own<NL, RULE_V>(m, 2 * d, i, j, k) * v + 0.5 * double(t[c - st]);
      acc[r] += a.c * (tp - tm) / m.h;
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int e = threadIdx.x + r * WG;
    if (e >= L::CPB * L::N3) continue;
    int s, i, j, k;
    cell_of<NL>(e, s, i, j, k);
    const int c = cube[s];
    if (c < 0) continue;
    const size_t g = (size_t)c * L::N3 + (e - s * L::N3);
    const double gp = acc[r] + (a.gp_in ? a.gp_in[g] : 0.0);
    a.out[g] = gp / sm[s].vol;
  }
}

template <int NL, typename TF>
__global__ __launch_bounds__(256) void k_adj_rhs(AdjRhsArgs<TF> a) {
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
    tile[s * L::TILE + ti<NL>(i, j, k)] = a.lam[(size_t)c * L::N3 + (e - s * L::N3)];
  }
  fill_halo<NL, RULE_L, double>(tile, sm, cube, FaceGet<NL, double>{a.lamf}, BcZero<double>{});
  __syncthreads();
  double gU = 0.0;
  for (int e = threadIdx.x; e < L::CPB * L::N3; e += WG) {
    int s, i, j, k;
    cell_of<NL>(e, s, i, j, k);
    const int cb = cube[s];
    if (cb < 0) continue;
    const CubeMeta& m = sm[s];
    const double* t = tile + s * L::TILE;
    const int c = ti<NL>(i, j, k);
    const double lam = t[c];
    const size_t g = (size_t)cb * L::N3 + (e - s * L::N3);
    const double al = a.alpha ? double(a.alpha[g]) : 0.0;
    double ga = 0.0;
    for (int d = 0; d < 3; ++d) {
      const int st = axis_stride<NL>(d);
      const double tp = side_own<NL, RULE_L>(m, 2 * d + 1, i, j, k) * lam - 0.5 * t[c + st];
      const double tm = side_own<NL, RULE_L>(m, 2 * d, i, j, k) * lam - 0.5 * t[c - st];
      const double gs = double(a.gun[d][g]) + a.inv_c * (tp - tm) / m.h;
      if (a.alpha) {
        const double us = a.us[d] ? double(a.us[d][g]) : a.usc[d];
        ga += gs * (us - double(a.u[d][g]));
      }
      a.gu[d][g] = TF((1.0 - al) * gs);
      const int co = axis_coord<NL>(d, i, j, k);
      if (co == 0 && m.kind[2 * d] == FK_INFLOW) gU -= a.inv_c * lam / m.h;
      if (co == NL - 1 && m.kind[2 * d + 1] == FK_INFLOW) gU -= a.inv_c * lam / m.h;
    }
    if (a.alpha && a.galpha) a.galpha[g] = a.accumulate ? TF(double(a.galpha[g]) + ga) : TF(ga);
  }
  if (a.part_gU) {
    const double t = block_sum(gU, red);
    if (threadIdx.x == 0) a.part_gU[blockIdx.x] = t;
  }
}

// Kinetic-energy objective: per workgroup the FP64 sum of V_i |u_i|^2 over its cubes (V_i = h^3,
// h the cube's cell width), and the seed cotangent gscale V_i u_i.  Workgroup w takes cubes
// w, w + G, ... in index order, so the partials and their sum are reproducible.
template <typename TF>
__global__ __launch_bounds__(256) void k_kinetic(KineticArgs<TF> a) {
  __shared__ double red[8];
  double acc = 0.0;
  for (int c = blockIdx.x; c < a.n_cubes; c += gridDim.x) {
    const double h = a.meta[c].h;
    const double V = h * h * h;
    for (int e = threadIdx.x; e < a.n3; e += 256) {
      const size_t g = (size_t)c * a.n3 + e;
      double uu = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double v = double(a.u[d][g]);
        uu += v * v;
        if (a.gu[d]) a.gu[d][g] = TF(a.gscale * V * v);
      }
      acc += V * uu;
    }
  }
  if (a.part) {
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) a.part[blockIdx.x] = t;
  }
}

}  // namespace

#define BCM_DISPATCH_NL(NLV, CALL)                    \
  switch (NLV) {                                      \
    case 16: { constexpr int NLC = 16; CALL; } break; \
    case 8: { constexpr int NLC = 8; CALL; } break;   \
    case 4: { constexpr int NLC = 4; CALL; } break;   \
    case 2: { constexpr int NLC = 2; CALL; } break;   \
    default: return hipErrorInvalidValue;             \
  }

static inline int n_wg(int NL, int n_cubes) {
  const int cpb = cubes_per_wg(NL);
  return (n_cubes + cpb - 1) / cpb;
}

template <typename TF>
hipError_t launch_force(int NL, const ForceArgs<TF>& a, hipStream_t s) {
  if (NL == 16) return launch16_force<TF>(a, s);
  BCM_DISPATCH_NL(NL, hipLaunchKernelGGL((k_force<NLC, TF>), dim3(n_wg(NLC, a.g.n_cubes)), dim3(WG), 0, s, a));
  return hipGetLastError();
}
template <typename TF>
hipError_t launch_div(int NL, const DivArgs<TF>& a, hipStream_t s) {
  if (NL == 16 && !a.part_bb) return launch16_div<TF>(a, s);
  BCM_DISPATCH_NL(NL, hipLaunchKernelGGL((k_div<NLC, TF>), dim3(n_wg(NLC, a.g.n_cubes)), dim3(WG), 0, s, a));
  return hipGetLastError();
}
template <typename TF>
hipError_t launch_correct(int NL, const CorrectArgs<TF>& a, hipStream_t s) {
  if (NL == 16 && !a.face_u[0] && !a.face_u[1] && !a.face_u[2]) return launch16_correct<TF>(a, s);
  BCM_DISPATCH_NL(NL, hipLaunchKernelGGL((k_correct<NLC, TF>), dim3(n_wg(NLC, a.g.n_cubes)), dim3(WG), 0, s, a));
  return hipGetLastError();
}
template <typename TF>
hipError_t launch_adj_gp(int NL, const AdjGpArgs<TF>& a, hipStream_t s) {
  BCM_DISPATCH_NL(NL, hipLaunchKernelGGL((k_adj_gp<NLC, TF>), dim3(n_wg(NLC, a.g.n_cubes)), dim3(WG), 0, s, a));
  return hipGetLastError();
}
template <typename TF>
hipError_t launch_adj_rhs(int NL, const AdjRhsArgs<TF>& a, hipStream_t s) {
  BCM_DISPATCH_NL(NL, hipLaunchKernelGGL((k_adj_rhs<NLC, TF>), dim3(n_wg(NLC, a.g.n_cubes)), dim3(WG), 0, s, a));
  return hipGetLastError();
}

template <typename TF>
hipError_t launch_kinetic(const KineticArgs<TF>& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_kinetic<TF>), dim3(grid), dim3(WG), 0, s, a);
  return hipGetLastError();
}

#define BCM_INST_F(TF)                                                                \
  template hipError_t launch_force<TF>(int, const ForceArgs<TF>&, hipStream_t);       \
  template hipError_t launch_div<TF>(int, const DivArgs<TF>&, hipStream_t);           \
  template hipError_t launch_correct<TF>(int, const CorrectArgs<TF>&, hipStream_t);   \
  template hipError_t launch_adj_gp<TF>(int, const AdjGpArgs<TF>&, hipStream_t);      \
  template hipError_t launch_adj_rhs<TF>(int, const AdjRhsArgs<TF>&, hipStream_t);    \
  template hipError_t launch_kinetic<TF>(const KineticArgs<TF>&, int, hipStream_t);
BCM_INST_F(float)
BCM_INST_F(double)

}  // namespace bcm
