// Lagrangian-particle immersed-boundary forcing (Sec. 2.3-2.4 and the forcing sub-step of
// Sec. 3): surface particles interpolate the intermediate velocity with the 3-point smoothed
// discrete delta function (Eq. (ddeltai)), take the constraint force F = (rho/dt)(U_s - U)
// and spread it back with the same weights (Eq. (ddeltap)): u* = u~ + (dt/rho) f.
//
// Thirty-two lanes (half a wavefront) per particle, lane e < 27 for cell e of the support: the
// gather is summed across the lanes and every lane spreads to its own cell.  The paper groups
// the particles into per-cube sets so that the cells around a particle follow from index
// arithmetic in its cube; here the lanes find the particle's cube themselves (dense per-level
// lattice tables, finest level first) and walk from it to the face neighbours, so the caller
// passes plain arrays.  The support is the 3 x 3 x 3 cells
// around the cell holding the particle, all of its cube's level; a particle outside the mesh,
// or whose support would leave that level's cubes or the domain, is skipped and counted.
// Spreading adds with atomics: contributions of particles that share a cell are summed in
// whatever order the lanes reach them (reproducible to rounding, not bit for bit).
#include "kernels.hpp"

namespace bcm {

namespace {

__device__ __forceinline__ double phi3(double r) {
  const double a = fabs(r);
  if (a <= 0.5) return 0.75 - a * a;
  if (a <= 1.5) return 0.5 * (2.25 - 3.0 * a + a * a);
  return 0.0;
}

// Cube of the mesh that holds point X (finest level first), its lattice position; -1 if none.
template <typename TF>
__device__ __forceinline__ int ib_locate(const IbArgs<TF>& a, const double (&X)[3], int (&pos)[3],
                                         int& lev) {
  for (int l = 0; l < a.n_levels; ++l) {
    const IbLevel& L = a.lev[l];
    int q[3];
    bool in = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double t = floor((X[d] - a.anchor[d]) / L.edge) - L.lo[d];  // NaN fails both tests
      in = in && t >= 0.0 && t < double(L.dims[d]);
      q[d] = in ? int(t) : 0;
    }
    if (!in) continue;
    const int c = a.table[L.offset + ((long long)q[2] * L.dims[1] + q[1]) * L.dims[0] + q[0]];
    if (c >= 0) {
#pragma unroll
      for (int d = 0; d < 3; ++d) pos[d] = q[d] + L.lo[d];
      lev = l;
      return c;
    }
  }
  return -1;
}

template <typename TF>
__global__ __launch_bounds__(256) void k_ib_force(IbArgs<TF> a) {
  const int e = threadIdx.x & 31;                                 // cell of the support
  const int p = (blockIdx.x * blockDim.x + threadIdx.x) >> 5;     // the same on 32 lanes
  if (p >= a.n_particles) return;
  const double X[3] = {a.X[3 * (size_t)p], a.X[3 * (size_t)p + 1], a.X[3 * (size_t)p + 2]};
  int pos[3], lev = 0;
  const int c0 = ib_locate(a, X, pos, lev);
  if (c0 < 0) {
    if (e == 0) atomicAdd(a.errors, 1u);
    return;
  }
  const int n = a.n;
  const double h = a.meta[c0].h;
  const double edge = a.lev[lev].edge;
  // cell holding X, relative to its cube, and the weights of the three cells per axis
  int cell[3];
  double w[3][3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double o = a.anchor[d] + pos[d] * edge;
    int ic = int(floor((X[d] - o) / h));
    ic = ic < 0 ? 0 : (ic > n - 1 ? n - 1 : ic);
    cell[d] = ic;
#pragma unroll
    for (int s = 0; s < 3; ++s) w[d][s] = phi3((o + (ic + s - 1 + 0.5) * h - X[d]) / h);
  }
  // cell e of the 27 (e = ex + 3 ey + 9 ez): its cube, reached from the particle's cube by
  // steps to face neighbours of the same level along x, then y, then z, and its offset there;
  // not found when a step meets a face without a same-level neighbour
  size_t g = 0;
  bool ok = true;
  double we = 0.0;
  if (e < 27) {
    const int dd[3] = {e % 3 - 1, (e / 3) % 3 - 1, e / 9 - 1};
    int c = c0, loc[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      loc[d] = cell[d] + dd[d];
      if (loc[d] < 0 || loc[d] >= n) {
        const CubeMeta& m = a.meta[c];
        const int f = 2 * d + (loc[d] >= n ? 1 : 0);
        ok = ok && m.kind[f] == FK_SAME;
        c = ok ? m.nbr[f][0] : c0;
        loc[d] = loc[d] < 0 ? loc[d] + n : loc[d] - n;
      }
    }
    g = (size_t)c * n * n * n + (loc[2] * n + loc[1]) * n + loc[0];
    we = w[0][e % 3] * w[1][(e / 3) % 3] * w[2][e / 9];
  }
  // gather: each lane's term, summed over the 32 lanes (every lane ends with the sums)
  double U[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) U[d] = e < 27 ? we * double(a.u[d][g]) : 0.0;
  int all = ok ? 1 : 0;
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) {
#pragma unroll
    for (int d = 0; d < 3; ++d) U[d] += __shfl_xor(U[d], o, 32);
    all = min(all, __shfl_xor(all, o, 32));
  }
  if (!all) {
    if (e == 0) atomicAdd(a.errors, 1u);
    return;
  }
  double F[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double us = a.Us ? a.Us[3 * (size_t)p + d] : a.usc[d];
    F[d] = a.rho_dt * (us - U[d]);
    if (e == 0 && a.Up) a.Up[3 * (size_t)p + d] = U[d];
    if (e == 0 && a.Fp) a.Fp[3 * (size_t)p + d] = F[d];
  }
  const double dV = a.dV ? a.dV[p] : h * h * h;
  const double scale = a.dt_rho * dV / (h * h * h);
  if (e < 27) {
#pragma unroll
    for (int d = 0; d < 3; ++d) atomicAdd(a.ustar[d] + g, TF(we * scale * F[d]));
  }
}

__global__ void k_zero_u32(unsigned int* p) { *p = 0u; }

}  // namespace

template <typename TF>
hipError_t launch_ib_force(const IbArgs<TF>& a, hipStream_t s) {
  if (a.n_particles <= 0) return hipSuccess;
  const long long lanes = 32ll * a.n_particles;
  if (lanes > 0x7FFFFFFFll) return hipErrorInvalidValue;  // lane indices are 32-bit
  hipLaunchKernelGGL((k_ib_force<TF>), dim3((unsigned)((lanes + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_zero_u32(unsigned int* p, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, p);
  return hipGetLastError();
}

template hipError_t launch_ib_force<float>(const IbArgs<float>&, hipStream_t);
template hipError_t launch_ib_force<double>(const IbArgs<double>&, hipStream_t);

}  // namespace bcm
