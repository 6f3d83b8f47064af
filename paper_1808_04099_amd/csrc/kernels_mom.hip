// Momentum sub-step (Sec. 3, Eq. (substep1)) on single-level meshes: H(v) = -A[v] + nu D[v]
// with QUICK convection in flux form (upwinded on the advecting velocity, frozen at u^n) and
// 7-point diffusion, for explicit Euler / Adams-Bashforth steps and the Jacobi iterations of
// the Crank-Nicolson system.
//
// QUICK reaches two cells upwind, so the halo is two layers deep.  The y and z layers of a
// neighbour are rows and planes of its cube (whole lines), read from the field itself, which
// no pass writes while it is read (the iteration alternates between two arrays).  The x
// layers (one value per row) go through a face buffer: per cube and component, faces f = 0, 1
// (-x, +x), layers L = 0 (boundary layer) and 1 (next inside), NL^2 values each as [t2][t1]
// (y, z).
// Producers export it (k_mom_export for a caller's field, the iteration kernels for their own
// output); consumers gather the neighbours' layers.  On a domain face
// the two ghost layers mirror the cube's own two boundary layers: Dirichlet value g gives
// 2 g - v, zero gradient gives v (inflow: every component Dirichlet, the normal one U_in into
// the domain; slip: normal component Dirichlet 0, tangential zero gradient; open: zero
// gradient).
//
// Layout per workgroup as the column kernels: lane t owns column (i, j) of cube slot s
// (CPB = 256 / NL^2 cubes per workgroup).  The cube is swept plane by plane: plane k of the
// three components goes through LDS with a two-cell x/y ring, the z neighbours k-2..k+2 are
// the lane's own column registers, and the x/y components of the advecting velocity of plane
// k go through LDS with a one-cell ring.  Arithmetic is FP64 whatever the field type.
#include "kernels.hpp"
#include "tile.hpp"

namespace bcm {

namespace {

template <int NL>
struct Mom {
  static constexpr int N2 = NL * NL, N3 = N2 * NL;
  static constexpr int CPB = NL >= 16 ? 1 : 256 / N2;
  static constexpr int W4 = NL + 4, P4 = W4 * W4;  // plane with a two-cell ring
  static constexpr int W2 = NL + 2, P2 = W2 * W2;  // plane with a one-cell ring
  static constexpr int FS = 4 * N2;                // face-buffer values per cube and component
  __device__ static int fidx(int f, int L, int t1, int t2) { return (f * 2 + L) * N2 + t2 * NL + t1; }
};

// Value across face f of a cube (kind kd) as an affine map of a source value: the
// neighbour's layer (kd == FK_SAME: scale 1, shift 0) or the cube's own mirrored layer on a
// domain face (Dirichlet g: -1, 2 g; zero gradient: 1, 0).
struct Affine {
  double scale, shift;
};
__device__ __forceinline__ Affine mom_rule(int kd, int f, int comp, double U_in) {
  const int d = f >> 1;
  if (kd == FK_INFLOW) return {-1.0, 2.0 * (comp == d ? ((f & 1) ? -U_in : U_in) : 0.0)};
  if (kd == FK_SLIP && comp == d) return {-1.0, 0.0};
  return {1.0, 0.0};  // a neighbour, an open face, or a tangential component on a slip wall
}

// Write the lane's share of the two-layer x faces of one component from its column x[0..NL-1].
template <int NL, typename TF>
__device__ __forceinline__ void mom_export_col(TF* mf, int c, const double (&x)[NL], int i, int j) {
  using M = Mom<NL>;
  TF* base = mf + (size_t)c * M::FS;
#pragma unroll
  for (int L = 0; L < 2; ++L) {
    if (i == L)
#pragma unroll
      for (int k = 0; k < NL; ++k) base[M::fidx(0, L, j, k)] = TF(x[k]);
    if (i == NL - 1 - L)
#pragma unroll
      for (int k = 0; k < NL; ++k) base[M::fidx(1, L, j, k)] = TF(x[k]);
  }
}

template <typename TF, int NL>
__global__ __launch_bounds__(256) void k_mom_export(MomExportArgs<TF> a) {
  using M = Mom<NL>;
  const int t = threadIdx.x, s = t / M::N2, l = t - s * M::N2, i = l % NL, j = l / NL;
  const int units = (a.n_cubes + M::CPB - 1) / M::CPB;
  for (int u = blockIdx.x; u < units; u += gridDim.x) {
    const int c = u * M::CPB + s;
    if (s >= M::CPB || c >= a.n_cubes) continue;
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
      double x[NL];
#pragma unroll
      for (int k = 0; k < NL; ++k) x[k] = double(a.x[comp][(size_t)c * M::N3 + k * M::N2 + l]);
      mom_export_col<NL, TF>(a.xf[comp], c, x, i, j);
    }
  }
}

// One pass of H over every cube (see MomArgs for the modes).
template <typename TF, int NL, int MODE>
__global__ __launch_bounds__(256, 2) void k_mom(MomArgs<TF> a) {
  using M = Mom<NL>;
  __shared__ double pv[M::CPB][3][M::P4];
  __shared__ double pa[M::CPB][2][M::P2];
  __shared__ double red[8];
  const int t = threadIdx.x, s = t / M::N2, l = t - s * M::N2, i = l % NL, j = l / NL;
  const int units = (a.n_cubes + M::CPB - 1) / M::CPB;
  double acc = 0.0;
  for (int u = blockIdx.x; u < units; u += gridDim.x) {
    const int c = u * M::CPB + s;
    const bool live = c < a.n_cubes;
    const int ce = live ? c : 0;
    const CubeMeta& m = a.meta[ce];
    const double ih = 1.0 / m.h, ih2 = ih * ih;
    const size_t cb = (size_t)ce * M::N3 + l;
    // Halo sources of this lane, each with the affine rule per component: the two layers
    // across the -z / +z faces at (i, j), element offsets into the fields (the neighbour's
    // planes NL-1, NL-2 / 0, 1; on a domain face the cube's own planes 0, 1 / NL-1, NL-2); and,
    // for the ring lanes (rows j = 0..3 of the slot, face f = j), the two layers across face f
    // at tangential position i, per plane k at ro + k * rs: for the x faces offsets into the
    // face buffers (rs = NL), for the y faces into the fields (the neighbour's rows NL-1, NL-2
    // / 0, 1, or the cube's own rows; rs = N2).
    size_t zo[2][2], ro[2] = {0, 0};
    Affine zr[2][4], rr[4];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int f = 4 + side, kd = m.kind[f];
      const bool nbr = kd == FK_SAME;
      const size_t cube = nbr ? (size_t)m.nbr[f][0] : (size_t)ce;
#pragma unroll
      for (int L = 0; L < 2; ++L) {
        // the layer L planes away from the shared face: the neighbour's far side, or this
        // cube's own near side mirrored
        const int plane = (side == 0) == nbr ? NL - 1 - L : L;
        zo[side][L] = cube * M::N3 + (size_t)plane * M::N2 + j * NL + i;
      }
#pragma unroll
      for (int comp = 0; comp < 3; ++comp) zr[side][comp] = nbr ? Affine{1.0, 0.0} : mom_rule(kd, f, comp, a.U_in);
    }
    const bool ring = j < 4;
    const int rf = j & 3, rd = rf >> 1, rside = rf & 1;
    const bool ry = rf >= 2;  // a y face: rows of the fields
    const size_t rs = ry ? M::N2 : NL;
    {
      const int kd = m.kind[rf];
      const bool nbr = kd == FK_SAME;
      const size_t cube = nbr ? (size_t)m.nbr[rf][0] : (size_t)ce;
      const int fs = nbr ? rf ^ 1 : rf;
#pragma unroll
      for (int L = 0; L < 2; ++L) {
        const int row = (rside == 0) == nbr ? NL - 1 - L : L;
        ro[L] = ry ? cube * M::N3 + (size_t)row * NL + i : cube * M::FS + M::fidx(fs, L, i, 0);
      }
#pragma unroll
      for (int comp = 0; comp < 3; ++comp) rr[comp] = nbr ? Affine{1.0, 0.0} : mom_rule(kd, rf, comp, a.U_in);
    }
    // z stencil windows of the lane's column, rotated plane by plane: v at k-2..k+2 (wv) and
    // a_z at k-1..k+1 (za); gh holds the two planes past the +z face
    double gh[3][2], wv[3][5], za[3];
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
#pragma unroll
      for (int L = 0; L < 2; ++L) {
        gh[comp][L] = zr[1][comp].scale * double(a.v[comp][zo[1][L]]) + zr[1][comp].shift;
        wv[comp][1 - L] = zr[0][comp].scale * double(a.v[comp][zo[0][L]]) + zr[0][comp].shift;
      }
      wv[comp][2] = double(a.v[comp][cb]);
      wv[comp][3] = double(a.v[comp][cb + M::N2]);
      wv[comp][4] = double(a.v[comp][cb + 2 * M::N2]);
    }
    const double azh = zr[1][2].scale * double(a.a[2][zo[1][0]]) + zr[1][2].shift;
    za[0] = zr[0][2].scale * double(a.a[2][zo[0][0]]) + zr[0][2].shift;
    za[1] = double(a.a[2][cb]);
    za[2] = double(a.a[2][cb + M::N2]);
    const int rpos0 = rside ? NL + 2 : 1, rpos1 = rside ? NL + 3 : 0;  // ring index along rd
    const int ridx0 = rd == 0 ? (i + 2) * M::W4 + rpos0 : rpos0 * M::W4 + i + 2;
    const int ridx1 = rd == 0 ? (i + 2) * M::W4 + rpos1 : rpos1 * M::W4 + i + 2;
    const int rp = rside ? NL + 1 : 0;
    const int ria = rd == 0 ? (i + 1) * M::W2 + rp : rp * M::W2 + i + 1;
    const Affine ra = rd == 0 ? rr[0] : rr[1];  // a select: a dynamic index would put rr in scratch
    // The outputs of plane k are stored at the top of plane k + 1, after that plane's loads
    // are issued: the vector-memory counter is in order, so a load issued after a store could
    // not be consumed before the store completes.
    double po[3] = {0.0, 0.0, 0.0}, ph[3] = {0.0, 0.0, 0.0};
    auto put = [&](int kp) __attribute__((always_inline)) {
      if (!live) return;
      const size_t gp = cb + (size_t)kp * M::N2;
#pragma unroll
      for (int comp = 0; comp < 3; ++comp) {
        const double o = po[comp];
        a.out[comp][gp] = TF(o);
        if (a.hout[comp]) a.hout[comp][gp] = TF(ph[comp]);
        if (a.outf[comp]) {  // two-layer x faces of the output, cell by cell
          TF* fb = a.outf[comp] + (size_t)c * M::FS;
#pragma unroll
          for (int L = 0; L < 2; ++L) {
            if (i == L) fb[M::fidx(0, L, j, kp)] = TF(o);
            if (i == NL - 1 - L) fb[M::fidx(1, L, j, kp)] = TF(o);
          }
        }
      }
    };
#pragma unroll 1
    for (int k = 0; k < NL; ++k) {
      const double axk = double(a.a[0][cb + k * M::N2]), ayk = double(a.a[1][cb + k * M::N2]);
      double qk[3];  // right-hand side (or previous H) of plane k
#pragma unroll
      for (int comp = 0; comp < 3; ++comp) {
        qk[comp] = 0.0;
        if (MODE == MOM_CN_ITER) qk[comp] = double(a.rhs[comp][cb + k * M::N2]);
        if (MODE == MOM_EXPLICIT && a.hprev[comp]) qk[comp] = double(a.hprev[comp][cb + k * M::N2]);
      }
      TF rgv[7];
      if (ring) {
        const size_t ko = (size_t)k * rs;
#pragma unroll
        for (int comp = 0; comp < 3; ++comp) {
          const TF* src = ry ? a.v[comp] : a.vf[comp];
          rgv[2 * comp] = src[ro[0] + ko];
          rgv[2 * comp + 1] = src[ro[1] + ko];
        }
        rgv[6] = (ry ? a.a[rd] : a.af[rd])[ro[0] + ko];
      }
      if (k > 0) put(k - 1);
      // plane k into LDS: interior, then the rings
#pragma unroll
      for (int comp = 0; comp < 3; ++comp) pv[s][comp][(j + 2) * M::W4 + i + 2] = wv[comp][2];
      pa[s][0][(j + 1) * M::W2 + i + 1] = axk;
      pa[s][1][(j + 1) * M::W2 + i + 1] = ayk;
      if (ring) {
#pragma unroll
        for (int comp = 0; comp < 3; ++comp) {
          pv[s][comp][ridx0] = rr[comp].scale * double(rgv[2 * comp]) + rr[comp].shift;
          pv[s][comp][ridx1] = rr[comp].scale * double(rgv[2 * comp + 1]) + rr[comp].shift;
        }
        pa[s][rd][ria] = ra.scale * double(rgv[6]) + ra.shift;
      }
      __syncthreads();
      const double Ux[2] = {0.5 * (pa[s][0][(j + 1) * M::W2 + i] + axk),
                            0.5 * (axk + pa[s][0][(j + 1) * M::W2 + i + 2])};
      const double Uy[2] = {0.5 * (pa[s][1][j * M::W2 + i + 1] + ayk),
                            0.5 * (ayk + pa[s][1][(j + 2) * M::W2 + i + 1])};
      const double Uz[2] = {0.5 * (za[0] + za[1]), 0.5 * (za[1] + za[2])};
      // interior Jacobi diagonal of H (Crank-Nicolson iterations): the coefficient of v(i)
      // in the two QUICK face values of each axis, and the diffusion's -6 nu / h^2
      double dg = 0.0;
      if (MODE == MOM_CN_ITER) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const double Um = d == 0 ? Ux[0] : d == 1 ? Uy[0] : Uz[0];
          const double Up = d == 0 ? Ux[1] : d == 1 ? Uy[1] : Uz[1];
          dg += (Up * (Up >= 0.0 ? 0.75 : 0.375) - Um * (Um >= 0.0 ? 0.375 : 0.75)) * ih;
        }
      }
      const size_t g = cb + k * M::N2;
#pragma unroll
      for (int comp = 0; comp < 3; ++comp) {
        double H = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          double w[5];
#pragma unroll
          for (int o = -2; o <= 2; ++o) {
            if (d == 0) w[o + 2] = pv[s][comp][(j + 2) * M::W4 + i + 2 + o];
            else if (d == 1) w[o + 2] = pv[s][comp][(j + 2 + o) * M::W4 + i + 2];
            else w[o + 2] = wv[comp][o + 2];
          }
          const double Um = d == 0 ? Ux[0] : d == 1 ? Uy[0] : Uz[0];
          const double Up = d == 0 ? Ux[1] : d == 1 ? Uy[1] : Uz[1];
          const double qp = Up >= 0.0 ? 0.75 * w[2] + 0.375 * w[3] - 0.125 * w[1]
                                      : 0.75 * w[3] + 0.375 * w[2] - 0.125 * w[4];
          const double qm = Um >= 0.0 ? 0.75 * w[1] + 0.375 * w[2] - 0.125 * w[0]
                                      : 0.75 * w[2] + 0.375 * w[1] - 0.125 * w[3];
          H += a.nu * ((w[3] - 2.0 * w[2] + w[1]) * ih2) - (Up * qp - Um * qm) * ih;
        }
        const double v0 = wv[comp][2];
        double o;
        if (MODE == MOM_EXPLICIT) {
          o = v0 + a.dt * (a.c1 * H + a.c2 * qk[comp]);
        } else if (MODE == MOM_CN_START) {
          const double rhs = v0 + 0.5 * a.dt * H;
          if (live) a.rhs[comp][g] = TF(rhs);
          acc += rhs * rhs;
          o = v0 + a.dt * H;  // Euler predictor as the first iterate
        } else {
          const double diag = fmax(1.0 + 0.5 * a.dt * (6.0 * a.nu * ih2 + dg), 0.5);
          const double r = qk[comp] + 0.5 * a.dt * H - v0;
          acc += r * r;
          o = v0 + r / diag;
        }
        po[comp] = o;
        ph[comp] = H;
      }
      __syncthreads();  // the next plane overwrites the LDS planes
      // rotate the z windows; the plane entering at k + 3 is the cube's, or a ghost plane
      const int kn = k + 3;
      const int kl = kn < NL ? kn : NL - 1;  // clamped: always an address inside the cube
#pragma unroll
      for (int comp = 0; comp < 3; ++comp) {
        const double nv = double(a.v[comp][cb + kl * M::N2]);
        wv[comp][0] = wv[comp][1];
        wv[comp][1] = wv[comp][2];
        wv[comp][2] = wv[comp][3];
        wv[comp][3] = wv[comp][4];
        wv[comp][4] = kn < NL ? nv : (kn == NL ? gh[comp][0] : gh[comp][1]);
      }
      const int ka = k + 2 < NL ? k + 2 : NL - 1;
      const double na = double(a.a[2][cb + ka * M::N2]);
      za[0] = za[1];
      za[1] = za[2];
      za[2] = k + 2 < NL ? na : azh;
    }
    put(NL - 1);
  }
  if (a.part) {
    const double tsum = block_sum(acc, red);
    if (threadIdx.x == 0) a.part[blockIdx.x] = tsum;
  }
}

}  // namespace

#define BCM_MOM_NL(NLV, CALL)                         \
  switch (NLV) {                                      \
    case 16: { constexpr int NLC = 16; CALL; } break; \
    case 8: { constexpr int NLC = 8; CALL; } break;   \
    case 4: { constexpr int NLC = 4; CALL; } break;   \
    default: return hipErrorInvalidValue;             \
  }

template <typename TF>
hipError_t launch_mom_export(int NL, const MomExportArgs<TF>& a, int grid, hipStream_t s) {
  BCM_MOM_NL(NL, hipLaunchKernelGGL((k_mom_export<TF, NLC>), dim3(grid), dim3(256), 0, s, a));
  return hipGetLastError();
}

template <typename TF>
hipError_t launch_mom(int NL, int mode, const MomArgs<TF>& a, int grid, hipStream_t s) {
  switch (mode) {
    case MOM_EXPLICIT:
      BCM_MOM_NL(NL, hipLaunchKernelGGL((k_mom<TF, NLC, MOM_EXPLICIT>), dim3(grid), dim3(256), 0, s, a));
      break;
    case MOM_CN_START:
      BCM_MOM_NL(NL, hipLaunchKernelGGL((k_mom<TF, NLC, MOM_CN_START>), dim3(grid), dim3(256), 0, s, a));
      break;
    case MOM_CN_ITER:
      BCM_MOM_NL(NL, hipLaunchKernelGGL((k_mom<TF, NLC, MOM_CN_ITER>), dim3(grid), dim3(256), 0, s, a));
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template hipError_t launch_mom_export<float>(int, const MomExportArgs<float>&, int, hipStream_t);
template hipError_t launch_mom_export<double>(int, const MomExportArgs<double>&, int, hipStream_t);
template hipError_t launch_mom<float>(int, int, const MomArgs<float>&, int, hipStream_t);
template hipError_t launch_mom<double>(int, int, const MomArgs<double>&, int, hipStream_t);

}  // namespace bcm
