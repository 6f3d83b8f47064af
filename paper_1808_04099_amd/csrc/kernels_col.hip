// Column kernels of the per-cube multigrid levels (16^3, 8^3, 4^3, 2^3 cells per cube): the
// HBM-bound part of the Poisson solve, plus the 16^3 projection kernels.
//
// Layout per workgroup (256 lanes): lane t owns one column (i, j) of a cube, k = 0..NL-1 held
// in registers; a workgroup holds CPB = max(1, 256 / NL^2) cubes.  Only the i/j neighbours go
// through LDS: per cube a tile of NL planes of (NL+2) x (NL+2) (the plane plus its x/y halo
// ring; at 16^3 the pre-smoother and the paired post-smoother use layouts of their own that
// avoid LDS bank conflicts, described at kc_smooth); the z neighbours are the lane's own
// registers, with the z halo of the column in two registers.  Every global access is a full
// plane of a cube (coalesced) or a face slab.
//
// The solver kernels are persistent: a workgroup walks units of CPB cubes with stride
// gridDim.x (a multiple of 8, so each workgroup stays on the XCD that owns its stretch of the
// Z-ordered launch table) and, while it computes one unit, the loads of its next unit are in
// flight (except FP64 at 16^3, where the registers are worth more as occupancy).  The
// prefetch does integer work only: the halo addresses are computed branch-free from the face
// relations and the loads land in raw registers that are combined when the cube is staged,
// because any arithmetic on a loaded value makes the in-order load counter wait for every
// load issued before it (the prefetched columns included).
//
// Whole-field values are read and written with non-temporal hints (each is touched once per
// launch); face slabs and scalars use ordinary cached accesses.  The cube metadata and the
// launch table are read with scalar loads (ro_load, meta_ro): the vector-memory counter is in
// order, so a wait on a vector load of a face kind or a cube index would also wait for the
// prefetched columns and the previous cube's stores.
//
// Multi-level meshes (2:1 faces) use the ML variants: one halo value per face cell still, the
// finer side exporting 2x2 means of the faces that border a coarser cube (face_stride).
#include <algorithm>
#include <type_traits>

#include "kernels.hpp"
#include "tile.hpp"

namespace bcm {

namespace {

template <int NL, int WW = NL + 2, int PP = WW * WW>
struct Col {
  static constexpr int N2 = NL * NL, N3 = N2 * NL;
  static constexpr int CPB = NL >= 16 ? 1 : 256 / N2;  // cubes per workgroup
  // LDS tile of one cube: NL planes of pitch P, rows of pitch W (NL cells and the x halos)
  static constexpr int W = WW, P = PP, TS = NL * P;
  static constexpr int H = NL / 2, H2 = H * H, H3 = H2 * H;  // next coarser per-cube level
  static constexpr int F = face_stride(NL), FH = face_stride(H);  // face-buffer values per cube
  __device__ static int tix(int s, int i, int j, int k) { return s * TS + k * P + (j + 1) * W + (i + 1); }
  // LDS position of the halo cell of face f (0..3) at tangential position (t1, t2)
  __device__ static int halo(int s, int f, int t1, int t2) {
    switch (f) {
      case 0: return tix(s, -1, t1, t2);
      case 1: return tix(s, NL, t1, t2);
      case 2: return tix(s, t1, -1, t2);
      default: return tix(s, t1, NL, t2);
    }
  }
};

// Lane geometry: cube slot s of the workgroup and column (i, j) within that cube.
template <int NL>
struct LaneC {
  int s, l, i, j;
  __device__ explicit LaneC(int t) {
    s = t / Col<NL>::N2;
    l = t - s * Col<NL>::N2;
    i = l % NL;
    j = l / NL;
  }
};

// Cube of slot s of unit u (-1 past the end).  With several cubes per unit, the unit takes
// launch-table positions 8 apart, so that all of them come from the stretch of the table that
// belongs to the unit's XCD (unit u runs on XCD u mod 8 when the grid is a multiple of 8).
template <int NL>
__device__ __forceinline__ int unit_cube(const Geom& g, int u, int s) {
  constexpr int CPB = Col<NL>::CPB;
  const int p = CPB == 1 ? u : ((u >> 3) * CPB + s) * 8 + (u & 7);
  int c = p < g.n_cubes ? ro_load(g.launch, p) : -1;
  if (Col<NL>::N2 >= 64) c = __builtin_amdgcn_readfirstlane(c);  // one cube per wavefront
  return c;
}

// Face-buffer offsets of the neighbour value a lane needs on each face:
//   same level    -> the neighbour's boundary cell;
//   coarser (2:1) -> the coarse cell covering this cell's quadrant of the face;
//   finer (2:1)   -> the 2x2 mean that the finer neighbour exports for this cell;
//   domain boundary -> the cube's own slab (a value that staging discards).
// Offsets into the face buffer of this level and, for prolongated corrections, into that of
// the next coarser level (the four finer cells facing a cell lie in one cell of that level).
struct Slots {
  int fine[6];
  int coarse[6];
  int kind[6];
};

// ML = false: a single-level mesh (only same-level neighbours and domain boundaries).
template <int NL, bool ML, class MT>
__device__ __forceinline__ void slots(const MT& m, int self, int t1, int t2, Slots& S) {
  using C = Col<NL>;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int kd = kind_of(m, f), of = f ^ 1;
    S.kind[f] = kd;
    int fo = self * C::F + f * C::N2 + t2 * NL + t1;
    int co = self * C::FH + f * C::H2 + (t2 >> 1) * C::H + (t1 >> 1);
    if (kd == FK_SAME) {
      const int c = m.nbr[f][0];
      fo = c * C::F + of * C::N2 + t2 * NL + t1;
      co = c * C::FH + of * C::H2 + (t2 >> 1) * C::H + (t1 >> 1);
    } else if (ML && kd == FK_COARSER) {
      const int qd = quad_of(m, f), c = m.nbr[f][0];
      const int a = (qd & 1) * C::H + (t1 >> 1), b = (qd >> 1) * C::H + (t2 >> 1);
      fo = c * C::F + of * C::N2 + b * NL + a;
      co = c * C::FH + of * C::H2 + (b >> 1) * C::H + (a >> 1);
    } else if (ML && kd == FK_FINER) {
      const int u1 = t1 >= C::H, u2 = t2 >= C::H;
      const int c = m.nbr[f][u1 + 2 * u2];
      const int A = t1 - u1 * C::H, B = t2 - u2 * C::H;
      fo = c * C::F + 6 * C::N2 + of * C::H2 + B * C::H + A;
      co = c * C::FH + of * C::H2 + B * C::H + A;
    }
    S.fine[f] = fo;
    S.coarse[f] = co;
  }
}

// Scaled halo value of one face from its raw neighbour value (RULE_P).  A select, not a zero
// scale: the dummy slab of a boundary face may hold anything.
template <typename T>
__device__ __forceinline__ T halo_val(int kd, T r) {
  return kd <= FK_FINER ? T(RuleTab<RULE_P>::nbeff(kd)) * r : T(0);
}

// Stage face values: faces 0..3 into the LDS ring at this lane's slot, 4/5 into registers.
template <int NL, typename T, class CL = Col<NL>>
__device__ __forceinline__ void stage(T* tile, const T (&hv)[6], const LaneC<NL>& L, T& zlo, T& zhi) {
#pragma unroll
  for (int f = 0; f < 4; ++f) tile[CL::halo(L.s, f, L.i, L.j)] = hv[f];
  zlo = hv[4];
  zhi = hv[5];
}

// Diagonal (sum of own coefficients) of the lane's column: cells k = 0, 1..NL-2, NL-1.
template <int NL, typename T, class MT>
__device__ __forceinline__ void diag(const MT& m, int i, int j, T& d0, T& dm, T& dl) {
  T c = T(6);
  if (i == 0) c += T(RuleTab<RULE_P>::own(kind_of(m, 0))) - T(1);
  if (i == NL - 1) c += T(RuleTab<RULE_P>::own(kind_of(m, 1))) - T(1);
  if (j == 0) c += T(RuleTab<RULE_P>::own(kind_of(m, 2))) - T(1);
  if (j == NL - 1) c += T(RuleTab<RULE_P>::own(kind_of(m, 3))) - T(1);
  dm = c;
  d0 = c + T(RuleTab<RULE_P>::own(kind_of(m, 4))) - T(1);
  dl = c + T(RuleTab<RULE_P>::own(kind_of(m, 5))) - T(1);
}

// Write the six face slabs of a cube from the lane's column.
template <int NL, typename T>
__device__ __forceinline__ void export_col(T* xf, int c, const T (&x)[NL], int i, int j) {
  constexpr int N2 = Col<NL>::N2;
  T* base = xf + (size_t)c * Col<NL>::F;
  if (i == 0)
#pragma unroll
    for (int k = 0; k < NL; ++k) base[0 * N2 + k * NL + j] = x[k];
  if (i == NL - 1)
#pragma unroll
    for (int k = 0; k < NL; ++k) base[1 * N2 + k * NL + j] = x[k];
  if (j == 0)
#pragma unroll
    for (int k = 0; k < NL; ++k) base[2 * N2 + k * NL + i] = x[k];
  if (j == NL - 1)
#pragma unroll
    for (int k = 0; k < NL; ++k) base[3 * N2 + k * NL + i] = x[k];
  base[4 * N2 + j * NL + i] = x[0];
  base[5 * N2 + j * NL + i] = x[NL - 1];
}

// The same slabs written in two steps through LDS (16^3 and 8^3).  The lanes on an x or y
// face hold a face row along z in registers, which export_col stores one value per
// instruction (NL instructions per face, a few lanes each).  Here those lanes put the row into
// LDS with 16-byte writes (per cube slot, 4 faces of NL rows of NL + 4 words: 16-byte aligned,
// and the reads below hit distinct banks at 8^3, two lanes per bank at 16^3), and after a
// barrier every lane reads its entry of each of the four slabs and stores it, one coalesced
// line per wavefront.  The z slabs are stored directly (every lane holds one value of each).
template <int NL>
struct XStage {
  static constexpr int R = NL + 4;           // row pitch in words
  static constexpr int S = 4 * NL * R;       // words per cube slot
  static constexpr int TOTAL = Col<NL>::CPB * S;
};
// NZ: no z slabs (the consumer reads the z neighbours from the field itself); z0 / z1: store
// the -z / +z slab.
template <int NL, typename T, bool NZ = false>
__device__ __forceinline__ void export_xy_put(T* xs, T* xf, int c, const T (&x)[NL], const LaneC<NL>& L,
                                              bool z0 = true, bool z1 = true) {
  using X = XStage<NL>;
  constexpr int N2 = Col<NL>::N2;
  const int i = L.i, j = L.j;
  auto put = [&](int f, int t1) {
    T* row = xs + L.s * X::S + (f * NL + t1) * X::R;
#pragma unroll
    for (int k = 0; k < NL; k += 4) {
      if constexpr (sizeof(T) == 4) {
        *reinterpret_cast<float4*>(row + k) = make_float4(x[k], x[k + 1], x[k + 2], x[k + 3]);
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) row[k + q] = x[k + q];
      }
    }
  };
  if (i == 0) put(0, j);
  if (i == NL - 1) put(1, j);
  if (j == 0) put(2, i);
  if (j == NL - 1) put(3, i);
  if (NZ) return;
  T* base = xf + (size_t)c * Col<NL>::F;
  if (z0) base[4 * N2 + j * NL + i] = x[0];
  if (z1) base[5 * N2 + j * NL + i] = x[NL - 1];
}
// After a barrier that follows export_xy_put: lane l of a cube slot stores slab entry l
// (t2 = l / NL, t1 = l % NL) of faces 0..3.
template <int NL, typename T>
__device__ __forceinline__ void export_xy_flush(const T* xs, T* xf, int c, const LaneC<NL>& L) {
  using X = XStage<NL>;
  constexpr int N2 = Col<NL>::N2;
  T* base = xf + (size_t)c * Col<NL>::F;
  const int t1 = L.l % NL, t2 = L.l / NL;
#pragma unroll
  for (int f = 0; f < 4; ++f) base[f * N2 + L.l] = xs[L.s * X::S + (f * NL + t1) * X::R + t2];
}

// 2x2 means of the face slabs on faces that border a coarser cube (see face_stride), from the
// cube's values in the LDS tile; summed in the order (0,0), (1,0), (0,1), (1,1) of the two
// tangential axes.  Lanes of each cube slot with l < (NL/2)^2 compute one mean per face.
template <int NL, typename T, class MT, class C = Col<NL>>
__device__ __forceinline__ void export_avg(T* xf, int c, const T* tile, const MT& m,
                                           const LaneC<NL>& L) {
  if (L.l >= C::H2) return;
  const int A = L.l % C::H, B = L.l / C::H;
  T* base = xf + (size_t)c * C::F + 6 * C::N2;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    if (kind_of(m, f) != FK_COARSER) continue;
    const int lay = (f & 1) ? NL - 1 : 0, d = f >> 1;
    T v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int a = 2 * A + (q & 1), b = 2 * B + (q >> 1);
      const int i = d == 0 ? lay : a, j = d == 0 ? a : (d == 1 ? lay : b), k = d == 2 ? lay : b;
      v[q] = tile[C::tix(L.s, i, j, k)];
    }
    base[f * C::H2 + B * C::H + A] = T(0.25) * (((v[0] + v[1]) + v[2]) + v[3]);
  }
}

template <int NL, typename T, class CL = Col<NL>>
__device__ __forceinline__ T nbsum(const T* tile, const T (&x)[NL], int k, int c, T zlo, T zhi) {
  constexpr int W = CL::W;
  const T zm = k > 0 ? x[k > 0 ? k - 1 : 0] : zlo;
  const T zp = k < NL - 1 ? x[k < NL - 1 ? k + 1 : NL - 1] : zhi;
  return tile[c - 1] + tile[c + 1] + tile[c - W] + tile[c + W] + zm + zp;
}

// The same sum in the halo-free tile of the 16^3 pre-smoother: neighbours at zb[] + plane
// offset o, zero z halo.
template <int NL, typename T>
__device__ __forceinline__ T nbsum_z(const T* tile, const int (&zb)[4], int o, const T (&x)[NL], int k) {
  const T zm = k > 0 ? x[k > 0 ? k - 1 : 0] : T(0);
  const T zp = k < NL - 1 ? x[k < NL - 1 ? k + 1 : NL - 1] : T(0);
  return tile[zb[0] + o] + tile[zb[1] + o] + tile[zb[2] + o] + tile[zb[3] + o] + zm + zp;
}

// Zero the partial sums past the grid, up to the count the reduction reads.
__device__ __forceinline__ void zero_tail(double* part, int units) {
  for (int k = blockIdx.x + gridDim.x; k < fine_grid(units); k += gridDim.x) part[k] = 0.0;
}

// ------------------------------------------------------------------------------------------
// Trilinear prolongation on single-level meshes.  Each cube slot of the workgroup gets a
// padded tile of the next coarser level: its (NL/2)^3 cells plus one layer on every side
// (faces, edges and corners), taken from the cube's 27-neighbourhood (pack_nb27), so that a
// fine cell next to a cube face interpolates from the neighbouring cube's coarse cells just as
// it would inside one cube.  Along each axis a fine cell takes 3/4 of the coarse cell that
// holds it and 1/4 of the next coarse cell on its side.  The fine halo of the post-smoother
// is the neighbour's own value after its prolongation: the neighbour's face cell interpolates
// from coarse cells that all lie in this padded tile, so it is computed here the same way.
// ------------------------------------------------------------------------------------------
template <int NL>
struct Pro {
  static constexpr int H = NL / 2, W = H + 2, P3 = W * W * W;
  // padded coordinates 0..H+1 (0 and H+1 are the neighbours' layers)
  __device__ static int ix(int s, int I, int J, int K) { return s * P3 + (K * W + J) * W + I; }
  // padded coarse index of fine index f (0..NL-1) and of the coarse cell on its side
  __device__ static int own(int f) { return (f >> 1) + 1; }
  __device__ static int side(int f) { return (f >> 1) + 1 + ((f & 1) ? 1 : -1); }
};

// Coordinate in the source cube of a padded coordinate P along one axis, given the step taken
// (d: 0 = none, -1 / +1) and whether the step was clamped at a domain boundary.
template <int H>
__device__ __forceinline__ int nb_coord(int P, int d, bool clamped) {
  if (d == 0) return P - 1;
  if (d < 0) return clamped ? 0 : H - 1;
  return clamped ? H - 1 : 0;
}

// Fill the padded coarse tiles of unit u from the coarse field xc.
template <int NL, typename T>
__device__ __forceinline__ void fill_coarse(T* ct, const T* xc, const uint32_t* nb27, int n_cubes,
                                            int u) {
  using C = Col<NL>;
  using Q = Pro<NL>;
  for (int e = threadIdx.x; e < C::CPB * Q::P3; e += 256) {
    const int s2 = e / Q::P3, r = e - s2 * Q::P3;
    const int I = r % Q::W, J = (r / Q::W) % Q::W, K = r / (Q::W * Q::W);
    const int p = C::CPB == 1 ? u : ((u >> 3) * C::CPB + s2) * 8 + (u & 7);
    T v = T(0);
    if (p < n_cubes) {
      const int dx = I == 0 ? -1 : (I == Q::W - 1 ? 1 : 0);
      const int dy = J == 0 ? -1 : (J == Q::W - 1 ? 1 : 0);
      const int dz = K == 0 ? -1 : (K == Q::W - 1 ? 1 : 0);
      const uint32_t ent = nb27[(size_t)p * 27 + ((dz + 1) * 3 + (dy + 1)) * 3 + (dx + 1)];
      const int id = int(ent & 0xFFFFFFu), cl = int(ent >> 24) & 7;
      const int I2 = nb_coord<Q::H>(I, dx, cl & 1), J2 = nb_coord<Q::H>(J, dy, cl & 2),
                K2 = nb_coord<Q::H>(K, dz, cl & 4);
      v = xc[(size_t)id * C::H3 + (K2 * Q::H + J2) * Q::H + I2];
      if (ent & (1u << 27)) v = -v;
    }
    ct[e] = v;
  }
}

// Prefetched form of fill_coarse.  The 27 table entries of each cube slot of a unit go to
// LDS (one load per lane, issued one unit ahead), the tile elements of a unit are spread over
// the lanes, NE per lane, and their values land in raw registers that are signed when they
// are written to LDS: no load waits on a load issued in the same step.
template <int NL>
struct ProPF {
  static constexpr int NT = Col<NL>::CPB * Pro<NL>::P3;  // tile elements per unit
  static constexpr int NE = (NT + 255) / 256;             // per lane
  static constexpr int NN = Col<NL>::CPB * 27;            // table entries per unit
  static constexpr int NEE = (NN + 255) / 256;            // per lane
};

template <int NL>
__device__ __forceinline__ void coarse_ent(const uint32_t* nb27, int n_cubes, int u,
                                           uint32_t (&ent)[ProPF<NL>::NEE]) {
  using C = Col<NL>;
#pragma unroll
  for (int m = 0; m < ProPF<NL>::NEE; ++m) {
    const int d = threadIdx.x + 256 * m, s2 = d / 27;
    const int p = C::CPB == 1 ? u : ((u >> 3) * C::CPB + s2) * 8 + (u & 7);
    const bool ok = d < ProPF<NL>::NN && p < n_cubes;
    ent[m] = ok ? nb27[(size_t)(ok ? p : 0) * 27 + (d - s2 * 27)] : ~0u;
  }
}

template <int NL>
__device__ __forceinline__ void coarse_ent_put(uint32_t* cent, const uint32_t (&ent)[ProPF<NL>::NEE]) {
#pragma unroll
  for (int m = 0; m < ProPF<NL>::NEE; ++m) {
    const int d = threadIdx.x + 256 * m;
    if (d < ProPF<NL>::NN) cent[d] = ent[m];
  }
}

// Unit-independent description of tile element e: bits 0..9 its source offset within the
// source cube when no step is clamped, bits 10..14 its direction (0..26), bits 15..20 its
// cube slot.  Computed once per workgroup.
template <int NL>
__device__ __forceinline__ uint32_t coarse_desc(int e) {
  using Q = Pro<NL>;
  const int s2 = e / Q::P3, r = e - s2 * Q::P3;
  const int I = r % Q::W, J = (r / Q::W) % Q::W, K = r / (Q::W * Q::W);
  const int dx = I == 0 ? -1 : (I == Q::W - 1 ? 1 : 0);
  const int dy = J == 0 ? -1 : (J == Q::W - 1 ? 1 : 0);
  const int dz = K == 0 ? -1 : (K == Q::W - 1 ? 1 : 0);
  const int off = (nb_coord<Q::H>(K, dz, false) * Q::H + nb_coord<Q::H>(J, dy, false)) * Q::H +
                  nb_coord<Q::H>(I, dx, false);
  const int dir = ((dz + 1) * 3 + (dy + 1)) * 3 + (dx + 1);
  return uint32_t(off) | (uint32_t(dir) << 10) | (uint32_t(s2) << 15);
}

// Issue the value loads of one unit from its entries in LDS; sg gets bit m = negate, bit
// 16 + m = element present.  A clamped step moves the source coordinate from the far layer
// of the neighbour to the near layer of the cube itself: d (H - 1) cells along that axis.
template <int NL, typename T>
__device__ __forceinline__ void coarse_val(const T* xc, const uint32_t* cdesc, const uint32_t* cent,
                                           T (&cv)[ProPF<NL>::NE], uint32_t& sg) {
  using C = Col<NL>;
  using Q = Pro<NL>;
  sg = 0;
#pragma unroll
  for (int m = 0; m < ProPF<NL>::NE; ++m) {
    const int e = threadIdx.x + 256 * m;
    const bool in = e < ProPF<NL>::NT;
    const uint32_t ds = cdesc[in ? e : 0];
    const int dir = int(ds >> 10) & 31;
    const uint32_t en = in ? cent[int(ds >> 15) * 27 + dir] : ~0u;
    const bool ok = en != ~0u;
    const int cl = int(en >> 24) & 7;
    const int dx = dir % 3 - 1, dy = (dir / 3) % 3 - 1, dz = dir / 9 - 1;
    const int off = int(ds & 1023u) + ((cl & 1) ? dx * (Q::H - 1) : 0) +
                    ((cl & 2) ? dy * (Q::H - 1) * Q::H : 0) + ((cl & 4) ? dz * (Q::H - 1) * Q::H * Q::H : 0);
    const int id = ok ? int(en & 0xFFFFFFu) : 0;
    cv[m] = xc[(size_t)id * C::H3 + (ok ? off : 0)];
    sg |= (ok ? (1u << (16 + m)) : 0u) | ((ok && (en >> 27 & 1u)) ? (1u << m) : 0u);
  }
}

template <int NL, typename T>
__device__ __forceinline__ void coarse_put(T* ct, const T (&cv)[ProPF<NL>::NE], uint32_t sg) {
#pragma unroll
  for (int m = 0; m < ProPF<NL>::NE; ++m) {
    const int e = threadIdx.x + 256 * m;
    if (e < ProPF<NL>::NT) {
      const T v = (sg >> m & 1u) ? -cv[m] : cv[m];
      ct[e] = (sg >> (16 + m) & 1u) ? v : T(0);
    }
  }
}

// Trilinear value from the padded tile: (a0, a1), (b0, b1), (c0, c1) are the near and far
// coarse cells along x, y and z.
template <int NL, typename T>
__device__ __forceinline__ T tri8(const T* ct, int s, int a0, int a1, int b0, int b1, int c0, int c1) {
  using Q = Pro<NL>;
  auto row = [&](int b, int c) { return T(0.75) * ct[Q::ix(s, a0, b, c)] + T(0.25) * ct[Q::ix(s, a1, b, c)]; };
  const T v0 = T(0.75) * row(b0, c0) + T(0.25) * row(b1, c0);
  const T v1 = T(0.75) * row(b0, c1) + T(0.25) * row(b1, c1);
  return T(0.75) * v0 + T(0.25) * v1;
}

// Prolongated correction of the lane's column (e[k]) and of its six halo cells (eh[f]): the
// x/y halos at tangential (t1, t2) = (i, j) as the stage() ring expects, the z halos of the
// column.
template <int NL, typename T>
__device__ __forceinline__ void tri_column(const T* ct, const LaneC<NL>& L, T (&e)[NL], T (&eh)[6]) {
  using Q = Pro<NL>;
  const int s = L.s, i = L.i, j = L.j;
  const int a0 = Q::own(i), a1 = Q::side(i), b0 = Q::own(j), b1 = Q::side(j);
  T v[Q::W];
#pragma unroll
  for (int K = 0; K < Q::W; ++K) {
    const T r0 = T(0.75) * ct[Q::ix(s, a0, b0, K)] + T(0.25) * ct[Q::ix(s, a1, b0, K)];
    const T r1 = T(0.75) * ct[Q::ix(s, a0, b1, K)] + T(0.25) * ct[Q::ix(s, a1, b1, K)];
    v[K] = T(0.75) * r0 + T(0.25) * r1;
  }
#pragma unroll
  for (int k = 0; k < NL; ++k) e[k] = T(0.75) * v[Q::own(k)] + T(0.25) * v[Q::side(k)];
  eh[4] = T(0.75) * v[0] + T(0.25) * v[1];
  eh[5] = T(0.75) * v[Q::W - 1] + T(0.25) * v[Q::W - 2];
  // x faces: (y, z) = (i, j); y faces: (x, z) = (i, j)
  eh[0] = tri8<NL, T>(ct, s, 0, 1, a0, a1, b0, b1);
  eh[1] = tri8<NL, T>(ct, s, Q::W - 1, Q::W - 2, a0, a1, b0, b1);
  eh[2] = tri8<NL, T>(ct, s, a0, a1, 0, 1, b0, b1);
  eh[3] = tri8<NL, T>(ct, s, a0, a1, Q::W - 1, Q::W - 2, b0, b1);
}

// ------------------------------------------------------------------------------------------
// Smoother (red-black Gauss-Seidel): POST = prolongation of the coarse correction + smoothing
// in black-red order (+ fused <x, b> and <x, q> on the finest level), else smoothing in
// red-black order from a zero initial guess.  TRI: trilinear prolongation (single-level
// meshes), else piecewise constant.
//
// The sweeps keep the column x (b in bv) in registers, the x/y neighbours in the LDS tile and
// the z halo in zlo / zhi, with one barrier per colour.  In a column the colour of cell k
// alternates, in phase with the lane's (i + j) parity; three forms of the same update order
// differ in how a lane reaches its cells of one colour:
//   masked:  every k, with the lanes of the other colour idle;
//   paired:  one cell of each pair (2n, 2n + 1), picked per lane by selects;
//   shifted: the column is copied into slots shifted by the parity (slot s = k + par + 1, the
//            z halo in slots par and NL + par + 1), so that one colour sits in the same slots
//            on every lane.
// In the shifted and paired forms a lane of parity 1 works one plane away from its neighbours
// of parity 0.  With (NL+2)-wide rows that puts lanes of a half-wavefront (the 32 lanes whose
// 32-bit LDS accesses are served together) on the same bank.  At 16^3:
//   * the pre-smoother of single-level meshes keeps a tile without halo (ZL): rows of NL cells,
//     planes of NL^2 cells followed by 64 zeros, a plane pitch that is a multiple of 64 words.
//     A lane on a cube face reads one of the zeros instead of its halo cell (the halo of a
//     pre-smoother is zero), picked so that its bank is one the other lanes leave free; every
//     access of the sweeps then hits distinct banks;
//   * the paired post-smoother keeps its halo ring in rows of 32 words and planes of 592
//     (16 mod 64 words), which puts the two parities on different banks.
// ------------------------------------------------------------------------------------------
// UPD (pre-smoother of level 0): the previous Krylov step's r update is fused in (upd_q).
template <typename T, int NL, bool POST, bool ML, bool TRI = false, bool UPD = false>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? (NL == 8 ? 4 : 3) : 2) void kc_smooth(SmoothArgs<T> a) {
  using C = Col<NL>;
  constexpr bool PF = sizeof(T) == 4 || NL < 16;
  // sweep form (same update order): shifted columns before restriction; in FP32 after the
  // trilinear prolongation or at 16^3 the paired form (fewer registers), else the masked form
  constexpr int SWEEP = !POST ? 2 : (sizeof(T) == 4 && (TRI || NL == 16) ? 1 : 0);
  // the halo-free tile of the 16^3 pre-smoother (plane pitch ZP words)
  constexpr bool ZL = !POST && NL == 16 && !ML;
  // the paired form at 16^3 (the FP32 trilinear post-smoother): rows of 32 words and planes
  // of 592, so that lanes one plane apart use other banks of each half-wavefront
  using CT = std::conditional_t<SWEEP == 1 && NL == 16, Col<NL, 32, 592>, Col<NL>>;
  constexpr int ZP = C::N2 + 64, TSL = ZL ? NL * ZP : CT::TS;
  // pre-smoother below the finest level: the finer level's face correction is applied here
  constexpr bool RFX = !POST && NL < 16;
  constexpr int NF = RFX ? 2 * NL : NL;  // the finer level
  __shared__ T tile[C::CPB * TSL];
  __shared__ T hsum[RFX ? C::CPB * 6 * C::N2 : 1];  // per cube and face: 2x2 sums of halo values
  __shared__ T ctile[TRI ? C::CPB * Pro<NL>::P3 : 1];
  __shared__ uint32_t cent[TRI && PF ? ProPF<NL>::NN : 1];
  __shared__ uint32_t cdesc[TRI && PF ? ProPF<NL>::NT : 1];
  __shared__ T rsum[POST ? 1 : C::CPB * C::H * C::N2];  // pre: residual summed over k pairs
  // the x and y slabs of the 16^3 smoothers and of the FP32 8^3 ones go out through LDS
  // (export_xy_put), stored after the next barrier: the restriction's
  // (pre-smoothers of single-level meshes), the one that ends the cube (multi-level meshes),
  // else the next unit's first (not the trilinear 8^3 post-smoother, which would spill)
  constexpr bool XS = ZL || NL == 16 || (NL == 8 && (ML || !POST) && sizeof(T) == 4);
  constexpr bool XPRE = XS && !POST && !ML;  // stored after the restriction's barrier
  // the 16^3 post-smoother of a single-level mesh feeds only apply, which reads the z
  // neighbours of z from z itself: no z slabs
  constexpr bool NZ = POST && !ML && NL == 16;
  // on a multi-level mesh its z slab is read across a face only by a finer neighbour (apply
  // reads a same-level neighbour from z itself, a coarser one's 2x2 means): stored only there
  constexpr bool MZ = POST && ML && NL == 16;
  __shared__ __align__(16) T xst[XS ? XStage<NL>::TOTAL : 1];
  __shared__ double red[8];
  const int t = threadIdx.x;
  const LaneC<NL> L(t);
  const int i = L.i, j = L.j;
  const int U = col_units(C::CPB, a.g.n_cubes), G = gridDim.x;
  const bool dots = POST && a.part_zr != nullptr;
  // ZL: the lane's cell in plane 0 and its x-, x+, y-, y+ neighbours there (a zero of the
  // plane's zero block on a cube face: bank 16 (j mod 4) + 15, 16 (j mod 4), 48 + i and i)
  const int zc = j * NL + i;
  const int zb[4] = {i > 0 ? zc - 1 : C::N2 + 16 * (j & 3) + 15, i < NL - 1 ? zc + 1 : C::N2 + 16 * (j & 3),
                     j > 0 ? zc - NL : C::N2 + 48 + i, j < NL - 1 ? zc + NL : C::N2 + i};
  if (ZL) {
    for (int e = t; e < NL * 64; e += 256) tile[(e >> 6) * ZP + C::N2 + (e & 63)] = T(0);
  }
  T nx[NL], nb[NL], nxc[C::H], rf[6], rc[6];
  int kinds[6];
  // face correction: raw finer-level halo values of the four finer cells (t1, t2) =
  // (2i + q % 2, 2j + q / 2) behind this column's position on each face
  T rr[RFX ? 24 : 1];
  int rk[RFX ? 6 : 1];
  const bool rfx = RFX && a.rfx != nullptr;
  // pre-smoother of level 0: the r update of the previous Krylov step, fused in
  constexpr bool upd = !POST && UPD;
  const T ual = upd ? T(a.upd_sc->alpha) : T(0);
  T nq[upd ? NL : 1];
  auto fetch = [&](int cc) {
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const size_t g = (size_t)cc * C::N3 + k * C::N2 + L.l;
      nb[k] = ld_nt(a.b + g);
      if (POST) nx[k] = ld_nt(a.x + g);
      if constexpr (upd) nq[k] = ld_nt(a.upd_q + g);
    }
    if constexpr (RFX) {
      if (rfx) {
        // the slot of (2i, 2j); the other three lie 1 and NF apart on a same-level face (or
        // the cube's own slab), 1 and NL apart among a finer neighbour's 2x2 means, and share
        // the coarser neighbour's value
        Slots S;
        slots<NF, ML>(meta_ro(a.g.meta, cc), cc, 2 * i, 2 * j, S);
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          const int kd = S.kind[f];
          const int d1 = ML && kd == FK_COARSER ? 0 : 1;
          const int d2 = ML && kd == FK_COARSER ? 0 : (ML && kd == FK_FINER ? NL : NF);
          const T* p = a.rfx + S.fine[f];
          rr[4 * f] = p[0];
          rr[4 * f + 1] = p[d1];
          rr[4 * f + 2] = p[d2];
          rr[4 * f + 3] = p[d1 + d2];
          rk[f] = kd;
        }
      }
    }
    if (POST) {
      if (!TRI) {
#pragma unroll
        for (int kk = 0; kk < C::H; ++kk)
          nxc[kk] = a.xc[(size_t)cc * C::H3 + (kk * C::H + (j >> 1)) * C::H + (i >> 1)];
      }
      Slots S;
      slots<NL, ML>(meta_ro(a.g.meta, cc), cc, i, j, S);
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        kinds[f] = S.kind[f];
        rf[f] = a.xf_in[S.fine[f]];
        if (!TRI) rc[f] = a.xcf[S.coarse[f]];
      }
    }
  };
  // trilinear prolongation with prefetch: entries one unit ahead of the values
  uint32_t entn[ProPF<NL>::NEE];
  T cvn[ProPF<NL>::NE];
  uint32_t sgn = 0;
  int u = blockIdx.x;
  int c = u < U ? unit_cube<NL>(a.g, u, L.s) : -1;
  int cx = -1;  // post-smoother: the cube whose x and y slabs wait in xst
  if (TRI && PF && u < U) {
    for (int e = t; e < ProPF<NL>::NT; e += 256) cdesc[e] = coarse_desc<NL>(e);
    coarse_ent<NL>(a.nb27, a.g.n_cubes, u, entn);
    coarse_ent_put<NL>(cent, entn);
    __syncthreads();
    coarse_val<NL, T>(a.xc, cdesc, cent, cvn, sgn);
    __syncthreads();
    if (u + G < U) coarse_ent<NL>(a.nb27, a.g.n_cubes, u + G, entn);
  }
  if (PF && u < U) fetch(c < 0 ? 0 : c);
  double zr = 0.0, zq = 0.0, rrs = 0.0;
  while (u < U) {
    const int ce = c < 0 ? 0 : c;
    if (!PF) fetch(ce);  // FP64 at 16^3: no prefetch (registers go to occupancy)
    T x[NL], bv[NL];
    T zlo = T(0), zhi = T(0);
    MetaRO& m = meta_ro(a.g.meta, ce);
    T eh[6];
    if (TRI) {
      if (PF) {
        coarse_put<NL, T>(ctile, cvn, sgn);
        if (u + G < U) coarse_ent_put<NL>(cent, entn);  // entries of the next unit
      } else
        fill_coarse<NL, T>(ctile, a.xc, a.nb27, a.g.n_cubes, u);
      __syncthreads();
      T e[NL];
      tri_column<NL, T>(ctile, L, e, eh);
#pragma unroll
      for (int k = 0; k < NL; ++k) x[k] = nx[k] + e[k];
    }
    if constexpr (upd) {
      // r -= alpha q (the arithmetic of k_update), stored back, and its norm
      MetaRO& mu = meta_ro(a.g.meta, ce);
      double rq = 0.0;
#pragma unroll
      for (int k = 0; k < NL; ++k) {
        nb[k] = nb[k] - ual * nq[k];
        rq += double(nb[k]) * double(nb[k]);
        if (c >= 0) st_nt(const_cast<T*>(a.b) + (size_t)c * C::N3 + k * C::N2 + L.l, nb[k]);
      }
      if (c >= 0) rrs += mu.vol * rq;
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      if (!TRI) x[k] = POST ? nx[k] + nxc[k >> 1] : T(0);
      bv[k] = nb[k];
      // (a pre-smoother's first pass writes its colour before anything reads the tile, and
      // the other colour is read only after its own first pass)
      if (POST || a.sweeps == 0) tile[ZL ? k * ZP + zc : CT::tix(L.s, i, j, k)] = x[k];
    }
    if (POST) {
      T hv[6];
#pragma unroll
      for (int f = 0; f < 6; ++f) hv[f] = halo_val<T>(kinds[f], rf[f] + (TRI ? eh[f] : rc[f]));
      stage<NL, T, CT>(tile, hv, L, zlo, zhi);
    } else if (!ZL) {
#pragma unroll
      for (int f = 0; f < 4; ++f) tile[CT::halo(L.s, f, i, j)] = T(0);
    }
    if constexpr (RFX) {
      if (rfx) {
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          const int kd = rk[f];
          hsum[(L.s * 6 + f) * C::N2 + j * NL + i] =
              (halo_val<T>(kd, rr[4 * f]) + halo_val<T>(kd, rr[4 * f + 1])) +
              (halo_val<T>(kd, rr[4 * f + 2]) + halo_val<T>(kd, rr[4 * f + 3]));
        }
      }
    }
    const T h = T(m.h * a.g.hscale);
    const T h2 = h * h;
    T d0, dm, dl;
    diag<NL, T>(m, i, j, d0, dm, dl);
    const T i0 = T(1) / d0, im = T(1) / dm, il = T(1) / dl;
    const double vol = m.vol;
    const int un = u + G;
    const int cn = un < U ? unit_cube<NL>(a.g, un, L.s) : -1;
    if (POST || RFX || a.sweeps == 0) __syncthreads();
    if (POST && XS && !ML && cx >= 0) export_xy_flush<NL, T>(xst, a.xf_out, cx, L);
    if constexpr (RFX) {
      // the finer level's restriction lacked the cross-cube terms of its residual: for each
      // face the cell lies on (x, y, then z), -(1/8) of the sum of its 2x2 finer halo values
      // over h_fine^2
      if (rfx) {
        const T hf = T(m.h * a.rfx_hscale);
        const T sc = T(0.125) / (hf * hf);
        const T* hs = hsum + L.s * 6 * C::N2;
#pragma unroll
        for (int k = 0; k < NL; ++k) {
          T corr = T(0);
          if (i == 0) corr += hs[0 * C::N2 + k * NL + j];
          if (i == NL - 1) corr += hs[1 * C::N2 + k * NL + j];
          if (j == 0) corr += hs[2 * C::N2 + k * NL + i];
          if (j == NL - 1) corr += hs[3 * C::N2 + k * NL + i];
          if (k == 0) corr += hs[4 * C::N2 + j * NL + i];
          if (k == NL - 1) corr += hs[5 * C::N2 + j * NL + i];
          bv[k] = bv[k] - corr * sc;
        }
      }
    }
    if (PF && un < U) {
      if (TRI) {
        coarse_val<NL, T>(a.xc, cdesc, cent, cvn, sgn);
        if (un + G < U) coarse_ent<NL>(a.nb27, a.g.n_cubes, un + G, entn);
      }
      fetch(cn < 0 ? 0 : cn);
    }
    // q of this cube for the fused <x, q> (loads overlap the sweeps)
    T q[NL];
    if (dots && a.q_dot) {
#pragma unroll
      for (int k = 0; k < NL; ++k) q[k] = ld_nt(a.q_dot + (size_t)ce * C::N3 + k * C::N2 + L.l);
    }
    if constexpr (SWEEP == 0) {
    for (int sw = 0; sw < a.sweeps; ++sw) {
  #pragma unroll
      for (int col = 0; col < 2; ++col) {
        const int colour = POST ? (col ^ 1) : col;
  #pragma unroll
        for (int k = 0; k < NL; ++k) {
          if (((i + j + k) & 1) != colour) continue;
          const int cc = CT::tix(L.s, i, j, k);
          const T sum = nbsum<NL, T, CT>(tile, x, k, cc, zlo, zhi);
          const T id = k == 0 ? i0 : (k == NL - 1 ? il : im);
          x[k] = (sum - h2 * bv[k]) * id;
          tile[cc] = x[k];
        }
        __syncthreads();
      }
    }
    } else if constexpr (SWEEP == 1) {
    const int par = (i + j) & 1;
    for (int sw = 0; sw < a.sweeps; ++sw) {
  #pragma unroll
      for (int col = 0; col < 2; ++col) {
        const int colour = POST ? (col ^ 1) : col;
        const bool odd = (colour ^ par) != 0;  // this lane updates k = 2n + 1, else k = 2n
  #pragma unroll
        for (int n = 0; n < NL / 2; ++n) {
          const int k0 = 2 * n, k1 = 2 * n + 1;
          const int cc = CT::tix(L.s, i, j, k0) + (odd ? CT::P : 0);
          const T zm = odd ? x[k0] : (k0 > 0 ? x[k0 > 0 ? k0 - 1 : 0] : zlo);
          const T zp = odd ? (k1 < NL - 1 ? x[k1 < NL - 1 ? k1 + 1 : 0] : zhi) : x[k1];
          const T sum = tile[cc - 1] + tile[cc + 1] + tile[cc - CT::W] + tile[cc + CT::W] + zm + zp;
          const T id = odd ? (k1 == NL - 1 ? il : im) : (k0 == 0 ? i0 : im);
          const T xn = (sum - h2 * (odd ? bv[k1] : bv[k0])) * id;
          x[k0] = odd ? x[k0] : xn;
          x[k1] = odd ? xn : x[k1];
          tile[cc] = xn;
        }
        __syncthreads();
      }
    }
    } else {
    const int par = (i + j) & 1;
    auto col_at = [&](int k) { return k == -1 ? zlo : (k == NL ? zhi : (k >= 0 && k < NL ? x[k >= 0 && k < NL ? k : 0] : T(0))); };
    auto b_at = [&](int k) { return k >= 0 && k < NL ? bv[k >= 0 && k < NL ? k : 0] : T(0); };
    T y[NL + 3], yb[NL + 3];
  #pragma unroll
    for (int sl = 0; sl < NL + 3; ++sl) {
      y[sl] = par ? col_at(sl - 2) : col_at(sl - 1);
      yb[sl] = par ? b_at(sl - 2) : b_at(sl - 1);
    }
    // LDS index of slot s: tb + s P (ZL: tz[0] + s ZP, the neighbours tz[1..4] + s ZP)
    const int tb = CT::tix(L.s, i, j, 0) - (1 + par) * CT::P;
    const int zs = (1 + par) * ZP;
    const int tz[5] = {zc - zs, zb[0] - zs, zb[1] - zs, zb[2] - zs, zb[3] - zs};
    // one colour pass (red-black order from the zero initial guess); RD = false in the
    // first pass, whose neighbours (the other colour and the halo) are still zero and are not
    // read: its sum is +0, as the sum of the zeros would be
    auto pass = [&](auto colour_c, auto rd_c) {
      constexpr int colour = decltype(colour_c)::value;
      constexpr bool RD = decltype(rd_c)::value;
  #pragma unroll
      for (int sl = 1; sl <= NL + 1; ++sl) {
        if ((sl & 1) != (colour ^ 1)) continue;  // the colour's slots (the same on every lane)
        // slot 1 is a cell only on par = 0 lanes, slot NL + 1 only on par = 1 lanes
        const bool valid = sl == 1 ? par == 0 : (sl == NL + 1 ? par == 1 : true);
        const int cc = ZL ? tz[0] + sl * ZP : tb + sl * CT::P;
        T sum = T(0);
        if constexpr (RD && ZL) {
          // a lane without a cell here reads the plane next to it (same banks), unused
          const int o = sl * ZP + (valid ? 0 : (sl == 1 ? ZP : -ZP));
          sum = tile[tz[1] + o] + tile[tz[2] + o] + tile[tz[3] + o] + tile[tz[4] + o] + y[sl - 1] + y[sl + 1];
        } else if constexpr (RD) {
          sum = tile[valid ? cc - 1 : 0] + tile[valid ? cc + 1 : 0] +
                tile[valid ? cc - CT::W : 0] + tile[valid ? cc + CT::W : 0] + y[sl - 1] + y[sl + 1];
        }
        // k = sl - 1 - par: the first cell sits at slot 1 or 2, the last at NL or NL + 1
        const T id = sl == 1 ? i0 : (sl == 2 ? (par ? i0 : im)
                                             : (sl == NL ? (par ? im : il) : (sl == NL + 1 ? il : im)));
        const T xn = (sum - h2 * yb[sl]) * id;
        if (sl == 1 || sl == NL + 1) {
          y[sl] = valid ? xn : y[sl];
          if (valid) tile[cc] = xn;
        } else {
          y[sl] = xn;
          tile[cc] = xn;
        }
      }
      __syncthreads();
    };
    static_assert(!POST, "the shifted form is the pre-smoother's");
    using C0 = std::integral_constant<int, 0>;
    using C1 = std::integral_constant<int, 1>;
    if (a.sweeps > 0) {
      pass(C0{}, std::false_type{});
      pass(C1{}, std::true_type{});
    }
    for (int sw = 1; sw < a.sweeps; ++sw) {
      pass(C0{}, std::true_type{});
      pass(C1{}, std::true_type{});
    }
  #pragma unroll
    for (int k = 0; k < NL; ++k) x[k] = par ? y[k + 2] : y[k + 1];
    }
    if (c >= 0) {
#pragma unroll
      for (int k = 0; k < NL; ++k) {
        st_nt(a.x + (size_t)c * C::N3 + k * C::N2 + L.l, x[k]);
        if (rfx) st_nt(a.b_fixed + (size_t)c * C::N3 + k * C::N2 + L.l, bv[k]);
        if (dots) {
          zr += vol * double(x[k]) * double(bv[k]);
          if (a.q_dot) zq += vol * double(x[k]) * double(q[k]);
        }
      }
      if constexpr (XS)
        export_xy_put<NL, T, NZ>(xst, a.xf_out, c, x, L, !MZ || kind_of(m, 4) == FK_FINER,
                                 !MZ || kind_of(m, 5) == FK_FINER);
      else
        export_col<NL, T>(a.xf_out, c, x, i, j);
      if (ML) export_avg<NL, T, MetaRO, CT>(a.xf_out, c, tile, m, L);
    }
    if (XPRE && !a.bc) __syncthreads();  // (a level without a coarser one)
    if (!POST && a.bc) {
      // residual with the halo the sweeps used (zero across cube faces), summed over the 2x2x2
      // children of each coarse cell; the face correction adds the cross-cube terms
      const T ih2 = T(1) / h2;
#pragma unroll
      for (int kk = 0; kk < C::H; ++kk) {
        T acc = T(0);
#pragma unroll
        for (int q2 = 0; q2 < 2; ++q2) {
          const int k = 2 * kk + q2;
          const T d = k == 0 ? d0 : (k == NL - 1 ? dl : dm);
          const T sum = ZL ? nbsum_z<NL, T>(tile, zb, k * ZP, x, k)
                           : nbsum<NL, T, CT>(tile, x, k, CT::tix(L.s, i, j, k), zlo, zhi);
          acc += bv[k] - (sum - d * x[k]) * ih2;
        }
        rsum[(L.s * C::H + kk) * C::N2 + L.l] = acc;
      }
      __syncthreads();
      for (int e = t; e < C::CPB * C::H3; e += 256) {
        const int s2 = e / C::H3, le = e - s2 * C::H3;
        const int I = le % C::H, J = (le / C::H) % C::H, K = le / C::H2;
        const int base = (s2 * C::H + K) * C::N2 + 2 * J * NL + 2 * I;
        const T sum = rsum[base] + rsum[base + 1] + rsum[base + NL] + rsum[base + NL + 1];
        const int c2 = unit_cube<NL>(a.g, u, s2);
        if (c2 >= 0) a.bc[(size_t)c2 * C::H3 + le] = sum * T(0.125);
      }
    }
    // (the next writes of xst come after the next cube's passes and their barriers)
    if (XPRE && c >= 0) export_xy_flush<NL, T>(xst, a.xf_out, c, L);
    if (ML) __syncthreads();  // the means read the tile the next cube overwrites
    if (ML && XS && c >= 0) export_xy_flush<NL, T>(xst, a.xf_out, c, L);
    if (POST && XS && !ML) cx = c;
    u = un;
    c = cn;
  }
  if (POST && XS && !ML) {
    __syncthreads();
    if (cx >= 0) export_xy_flush<NL, T>(xst, a.xf_out, cx, L);
  }
  if (dots) {
    const double t0 = block_sum(zr, red);
    __syncthreads();
    const double t1 = block_sum(zq, red);
    if (threadIdx.x == 0) {
      a.part_zr[blockIdx.x] = t0;
      zero_tail(a.part_zr, U);
      if (a.part_zq) {
        a.part_zq[blockIdx.x] = t1;
        zero_tail(a.part_zq, U);
      }
    }
  }
  if constexpr (upd) {
    const double t0 = block_sum(rrs, red);
    if (threadIdx.x == 0) {
      a.part_rr[blockIdx.x] = t0;
      zero_tail(a.part_rr, U);
    }
  }
}

// Completes the restriction fused into the pre-smoother of the last per-cube level (the
// pre-smoothers of the levels in between apply the same correction to their own right-hand
// side as they load it).  A coarse cell on a cube's boundary still lacks the cross-cube terms
// of its children's residuals, -(1/8) sum nbeff x_nb / h^2 over the children's faces that
// border a neighbour.  Lane (i, j) of each cube slot gathers
// the six halo values at tangential (t1, t2) = (i, j) (as the smoothers do), the 2x2 children
// of each coarse face cell are summed in LDS, and each coarse boundary cell adds the sums of
// its faces in the order x, y, z.
template <typename T, int NL, bool ML>
__global__ __launch_bounds__(256) void kc_rfix(RestrictFixArgs<T> a) {
  using C = Col<NL>;
  constexpr int NE = (C::CPB * C::H3 + 255) / 256;  // coarse cells per lane
  __shared__ T hv[C::CPB * 6 * C::N2];
  const LaneC<NL> L(threadIdx.x);
  const int U = col_units(C::CPB, a.g.n_cubes), G = gridDim.x;
  // per unit: the lane's six raw halo values and its coarse cells' current values, loaded one
  // unit ahead (raw registers, combined after the loads of the next unit are issued)
  T rf[6], bv[NE];
  int kinds[6], faces[NE];  // faces: bit f = the cell lies on face f of a cube present
  size_t at_g[NE];
  auto fetch = [&](int uu) {
    const int c = unit_cube<NL>(a.g, uu, L.s);
    Slots S;
    slots<NL, ML>(meta_ro(a.g.meta, c < 0 ? 0 : c), c < 0 ? 0 : c, L.i, L.j, S);
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      kinds[f] = c < 0 ? FK_OUTFLOW : S.kind[f];
      rf[f] = a.xf[S.fine[f]];
    }
#pragma unroll
    for (int n = 0; n < NE; ++n) {
      const int e = threadIdx.x + 256 * n;
      const int s2 = e / C::H3, le = e - s2 * C::H3;
      const int I = le % C::H, J = (le / C::H) % C::H, K = le / C::H2;
      const int c2 = e < C::CPB * C::H3 ? unit_cube<NL>(a.g, uu, s2) : -1;
      faces[n] = c2 < 0 ? 0
                        : (I == 0) | (I == C::H - 1) << 1 | (J == 0) << 2 | (J == C::H - 1) << 3 |
                              (K == 0) << 4 | (K == C::H - 1) << 5;
      at_g[n] = (size_t)(c2 < 0 ? 0 : c2) * C::H3 + le;
      bv[n] = a.bc[at_g[n]];
    }
  };
  int u = blockIdx.x;
  if (u < U) fetch(u);
  while (u < U) {
#pragma unroll
    for (int f = 0; f < 6; ++f) hv[(L.s * 6 + f) * C::N2 + L.l] = halo_val<T>(kinds[f], rf[f]);
    T cb[NE];
    int cf[NE];
    size_t cg[NE];
#pragma unroll
    for (int n = 0; n < NE; ++n) {
      cb[n] = bv[n];
      cf[n] = faces[n];
      cg[n] = at_g[n];
    }
    __syncthreads();
    if (u + G < U) fetch(u + G);
#pragma unroll
    for (int n = 0; n < NE; ++n) {
      const int e = threadIdx.x + 256 * n;
      if (e >= C::CPB * C::H3 || unit_cube<NL>(a.g, u, e / C::H3) < 0) continue;
      // every cell is written (interior ones unchanged), so that whole lines are stored
      const int s2 = e / C::H3, le = e - s2 * C::H3;
      const int I = le % C::H, J = (le / C::H) % C::H, K = le / C::H2;
      T corr = T(0);
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        if (!(cf[n] >> f & 1)) continue;
        const int T1 = f < 2 ? J : I, T2 = f < 4 ? K : J;  // coarse tangential position
        const T* h = hv + (s2 * 6 + f) * C::N2 + (2 * T2) * NL + 2 * T1;
        corr += (h[0] + h[1]) + (h[NL] + h[NL + 1]);
      }
      const T hh = T(meta_ro(a.g.meta, cg[n] / C::H3).h * a.g.hscale);
      a.bc[cg[n]] = cb[n] - corr * (T(0.125) / (hh * hh));
    }
    __syncthreads();  // hv is rewritten for the next unit
    u += G;
  }
}

// p = z + beta p (or z); q = A p; partial <p, q>_V.
template <typename T, int NL, bool ML>
__global__ __launch_bounds__(256) void kc_apply(ApplyArgs<T> a) {
  using C = Col<NL>;
  constexpr bool PF = sizeof(T) == 4 || NL < 16;
  __shared__ T tile[C::CPB * C::TS];
  // at 16^3: the x and y slabs of p go out through LDS (export_xy_put)
  constexpr bool XS = NL == 16;
  // at 16^3: the z neighbours of z of the same level are read from z (which this kernel does
  // not write; whole lines of the neighbours' end planes), so the post-smoother stores z slabs
  // only where a finer neighbour reads them
  constexpr bool ZD = XS;
  __shared__ __align__(16) T xst[XS ? XStage<NL>::TOTAL : 1];
  __shared__ double red[8];
  const int t = threadIdx.x;
  const LaneC<NL> L(t);
  const int i = L.i, j = L.j;
  const int U = col_units(C::CPB, a.g.n_cubes), G = gridDim.x;
  const T beta = a.first ? T(0) : T(a.sc->beta);
  T nz[NL], np[NL], rz[6], rp[6];
  int kinds[6];
  auto fetch = [&](int cc) {
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const size_t g = (size_t)cc * C::N3 + k * C::N2 + L.l;
      nz[k] = ld_nt(a.z + g);
      np[k] = a.first ? T(0) : ld_nt(a.p + g);
    }
    Slots S;
    slots<NL, ML>(meta_ro(a.g.meta, cc), cc, i, j, S);
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      kinds[f] = S.kind[f];
      rp[f] = a.first ? T(0) : a.pf_in[S.fine[f]];
      if (!ZD || f < 4 || (ML && S.kind[f] != FK_SAME)) {
        rz[f] = a.zf[S.fine[f]];
      } else {
        // the neighbour's cell next to the face at (i, j): (i, j, NL-1) below, (i, j, 0)
        // above; across a domain boundary a cell of this cube (the value is not used)
        MetaRO& mm = meta_ro(a.g.meta, cc);
        const int nb = S.kind[f] == FK_SAME ? mm.nbr[f][0] : cc;
        rz[f] = a.z[(size_t)nb * C::N3 + (f == 4 ? (NL - 1) * C::N2 : 0) + j * NL + i];
      }
    }
  };
  int u = blockIdx.x;
  int c = u < U ? unit_cube<NL>(a.g, u, L.s) : -1;
  if (PF && u < U) fetch(c < 0 ? 0 : c);
  double pq = 0.0;
  while (u < U) {
    const int ce = c < 0 ? 0 : c;
    if (!PF) fetch(ce);  // FP64 at 16^3: no prefetch (registers go to occupancy)
    T x[NL], hv[6];
    T zlo, zhi;
    MetaRO& m = meta_ro(a.g.meta, ce);
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      x[k] = nz[k] + beta * np[k];
      tile[C::tix(L.s, i, j, k)] = x[k];
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) hv[f] = halo_val<T>(kinds[f], rz[f] + beta * rp[f]);
    stage<NL, T>(tile, hv, L, zlo, zhi);
    const T h = T(m.h * a.g.hscale);
    const T ih2 = T(1) / (h * h);
    T d0, dm, dl;
    diag<NL, T>(m, i, j, d0, dm, dl);
    const double vol = m.vol;
    const int un = u + G;
    const int cn = un < U ? unit_cube<NL>(a.g, un, L.s) : -1;
    __syncthreads();
    if (PF && un < U) fetch(cn < 0 ? 0 : cn);
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const T d = k == 0 ? d0 : (k == NL - 1 ? dl : dm);
      const T sum = nbsum<NL, T>(tile, x, k, C::tix(L.s, i, j, k), zlo, zhi);
      const T qv = (sum - d * x[k]) * ih2;
      if (c >= 0) {
        const size_t g = (size_t)c * C::N3 + k * C::N2 + L.l;
        st_nt(a.p + g, x[k]);
        st_nt(a.q + g, qv);
        pq += vol * double(x[k]) * double(qv);
      }
    }
    if (c >= 0) {
      if constexpr (XS)
        export_xy_put<NL, T>(xst, a.pf_out, c, x, L);
      else
        export_col<NL, T>(a.pf_out, c, x, i, j);
      if (ML) export_avg<NL, T>(a.pf_out, c, tile, m, L);
    }
    __syncthreads();
    // (xst is written again after the next cube's first barrier)
    if (XS && c >= 0) export_xy_flush<NL, T>(xst, a.pf_out, c, L);
    u = un;
    c = cn;
  }
  const double tot = block_sum(pq, red);
  if (threadIdx.x == 0) {
    a.part[blockIdx.x] = tot;
    zero_tail(a.part, U);
  }
}

// r = b - A p in FP64 (p may be nullptr = 0; b may be nullptr -> r = A p), stored as TO * rscale.
template <typename TO, int NL, bool ML>
__global__ __launch_bounds__(256) void kc_resid64(Resid64Args<TO> a) {
  using C = Col<NL>;
  __shared__ double tile[C::CPB * C::TS];
  __shared__ double red[8];
  const int t = threadIdx.x;
  const LaneC<NL> L(t);
  const int i = L.i, j = L.j;
  const int U = col_units(C::CPB, a.g.n_cubes), G = gridDim.x;
  double np[NL], nb[NL], rf[6];
  int kinds[6];
  auto fetch = [&](int cc) {
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const size_t g = (size_t)cc * C::N3 + k * C::N2 + L.l;
      np[k] = a.p ? ld_nt(a.p + g) : 0.0;
      nb[k] = a.b ? ld_nt(a.b + g) : 0.0;
    }
    Slots S;
    slots<NL, ML>(meta_ro(a.g.meta, cc), cc, i, j, S);
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      kinds[f] = S.kind[f];
      rf[f] = a.p ? a.pf[S.fine[f]] : 0.0;
    }
  };
  int u = blockIdx.x;
  int c = u < U ? unit_cube<NL>(a.g, u, L.s) : -1;
  if (u < U) fetch(c < 0 ? 0 : c);
  double rr = 0.0, bb = 0.0;
  while (u < U) {
    const int ce = c < 0 ? 0 : c;
    double x[NL], bv[NL], hv[6];
    double zlo, zhi;
    MetaRO& m = meta_ro(a.g.meta, ce);
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      x[k] = np[k];
      bv[k] = nb[k];
      tile[C::tix(L.s, i, j, k)] = x[k];
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) hv[f] = halo_val<double>(kinds[f], rf[f]);
    stage<NL, double>(tile, hv, L, zlo, zhi);
    const double h = m.h * a.g.hscale;
    const double ih2 = 1.0 / (h * h);
    double d0, dm, dl;
    diag<NL, double>(m, i, j, d0, dm, dl);
    const double vol = m.vol;
    const int un = u + G;
    const int cn = un < U ? unit_cube<NL>(a.g, un, L.s) : -1;
    __syncthreads();
    if (un < U) fetch(cn < 0 ? 0 : cn);
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const double d = k == 0 ? d0 : (k == NL - 1 ? dl : dm);
      const double sum = nbsum<NL, double>(tile, x, k, C::tix(L.s, i, j, k), zlo, zhi);
      const double ap = (sum - d * x[k]) * ih2;
      const double r = a.b ? bv[k] - ap : ap;
      if (c >= 0) {
        if (a.b) bb += vol * bv[k] * bv[k];
        rr += vol * r * r;
        st_nt(a.r + (size_t)c * C::N3 + k * C::N2 + L.l, TO(r * a.rscale));
      }
    }
    __syncthreads();
    u = un;
    c = cn;
  }
  if (a.part_rr) {
    const double t0 = block_sum(rr, red);
    __syncthreads();
    const double t1 = block_sum(bb, red);
    if (threadIdx.x == 0) {
      a.part_rr[blockIdx.x] = t0;
      zero_tail(a.part_rr, U);
      if (a.part_bb) {
        a.part_bb[blockIdx.x] = t1;
        zero_tail(a.part_bb, U);
      }
    }
  }
}

// p += dscale d (when d is given) in FP64; export the faces of p (ML: and their 2x2 means,
// staged through LDS).
template <typename T, int NL, bool ML>
__global__ __launch_bounds__(256) void kc_ir(IrArgs<T> a) {
  using C = Col<NL>;
  __shared__ double tile[ML ? C::CPB * C::TS : 1];
  const LaneC<NL> L(threadIdx.x);
  const int U = col_units(C::CPB, a.g.n_cubes);
  for (int u = blockIdx.x; u < U; u += gridDim.x) {
    const int c = unit_cube<NL>(a.g, u, L.s);
    const int ce = c < 0 ? 0 : c;
    double p[NL];
    if (a.p_zero) {
#pragma unroll
      for (int k = 0; k < NL; ++k) p[k] = 0.0;
    } else {
#pragma unroll
      for (int k = 0; k < NL; ++k) p[k] = ld_nt(a.p + (size_t)ce * C::N3 + k * C::N2 + L.l);
    }
    if (a.d) {
      T d[NL];
      if (a.d_zero) {
#pragma unroll
        for (int k = 0; k < NL; ++k) d[k] = T(0);
      } else {
#pragma unroll
        for (int k = 0; k < NL; ++k) d[k] = ld_nt(a.d + (size_t)ce * C::N3 + k * C::N2 + L.l);
      }
      if (a.pdir) {  // the inner solve's last x update (the arithmetic of k_update)
        const T al = T(a.sc->alpha);
#pragma unroll
        for (int k = 0; k < NL; ++k) d[k] = d[k] + al * ld_nt(a.pdir + (size_t)ce * C::N3 + k * C::N2 + L.l);
      }
#pragma unroll
      for (int k = 0; k < NL; ++k) {
        p[k] += a.dscale * double(d[k]);
        if (c >= 0) st_nt(a.p + (size_t)c * C::N3 + k * C::N2 + L.l, p[k]);
      }
    }
    if (c >= 0) export_col<NL, double>(a.pf_out, c, p, L.i, L.j);
    if (ML) {
#pragma unroll
      for (int k = 0; k < NL; ++k) tile[C::tix(L.s, L.i, L.j, k)] = p[k];
      __syncthreads();
      if (c >= 0) export_avg<NL, double>(a.pf_out, c, tile, meta_ro(a.g.meta, c), L);
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------------------------------------
// Projection step on 16^3 cubes (kernels_proj.hip has the versions for every cube size).
// ------------------------------------------------------------------------------------------
constexpr int P16 = Col<16>::P;
__device__ __forceinline__ int tix16(int i, int j, int k) { return Col<16>::tix(0, i, j, k); }
__device__ __forceinline__ int halo16(int f, int t) { return Col<16>::halo(0, f, t & 15, t >> 4); }

template <typename T>
__device__ __forceinline__ T face_get(const T* f, int c, int of, int t1, int t2) {
  return f[(size_t)c * Col<16>::F + of * 256 + t2 * 16 + t1];
}

// u* = (1 - alpha) u~ + alpha u_s, and the face-normal component of u* on each face.  A pure
// stream: planes are processed four at a time so that few values are live per lane.
// With a.body set, only the cubes with some alpha != 0 (body cubes) are forced and stored; the
// kernel records the flag per cube, and for the other cubes, where u* = u~, it writes only the
// face slabs of u~ (u_x is read whole for its x faces, u_y two rows per plane, u_z two planes);
// the divergence and correction kernels then read u~ for them.
template <typename TF>
__global__ __launch_bounds__(256) void k16_force(ForceArgs<TF> a) {
  const int t = threadIdx.x, i = t & 15, j = t >> 4;
  const int n = a.g.n_cubes;
  for (int w = blockIdx.x; w < n; w += gridDim.x) {
    const int c = ro_load(a.g.launch, w);
    TF* base = a.uf + (size_t)c * Col<16>::F;
    if (a.body) {
      // alpha and the face sources of u~ are loaded together, before the decision; all three
      // comparisons wait only on loads issued before them
      const size_t g0 = (size_t)c * 4096 + t;
      const bool ry = j == 0 || j == 15;
      const TF* ap = a.alpha ? a.alpha : a.u[0];  // no alpha: loads that decide nothing
      const TF* yp = a.u[1] + (ry ? g0 : (size_t)c * 4096 + (t & 15));  // row j = 0 otherwise
      TF al[16], ux[16], uy[16], uz[2];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        al[k] = ld_nt(ap + g0 + k * 256);
        ux[k] = ld_nt(a.u[0] + g0 + k * 256);
        uy[k] = ld_nt(yp + k * 256);
      }
      uz[0] = ld_nt(a.u[2] + g0);
      uz[1] = ld_nt(a.u[2] + g0 + 15 * 256);
      bool nz = false;
#pragma unroll
      for (int k = 0; k < 16; ++k) nz |= al[k] != TF(0);
      nz = nz && a.alpha != nullptr;
      const bool any = __syncthreads_or(nz);
      if (t == 0) a.body[c] = any ? 1 : 0;
      if (!any) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          if (i == 0) base[0 * 256 + k * 16 + j] = ux[k];
          if (i == 15) base[1 * 256 + k * 16 + j] = ux[k];
          if (ry) base[(j ? 3 : 2) * 256 + k * 16 + i] = uy[k];
        }
        base[4 * 256 + j * 16 + i] = uz[0];
        base[5 * 256 + j * 16 + i] = uz[1];
        continue;
      }
    }
#pragma unroll 1
    for (int k0 = 0; k0 < 16; k0 += 4) {
      TF v[3][4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const size_t g = (size_t)c * 4096 + (k0 + kk) * 256 + t;
        const TF al = a.alpha ? ld_nt(a.alpha + g) : TF(0);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const TF ut = ld_nt(a.u[d] + g);
          const TF us = a.us[d] ? ld_nt(a.us[d] + g) : TF(a.usc[d]);
          v[d][kk] = a.alpha ? (TF(1) - al) * ut + al * us : ut;
        }
      }
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int k = k0 + kk;
        const size_t g = (size_t)c * 4096 + k * 256 + t;
#pragma unroll
        for (int d = 0; d < 3; ++d) st_nt(a.ustar[d] + g, v[d][kk]);
        if (i == 0) base[0 * 256 + k * 16 + j] = v[0][kk];
        if (i == 15) base[1 * 256 + k * 16 + j] = v[0][kk];
        if (j == 0) base[2 * 256 + k * 16 + i] = v[1][kk];
        if (j == 15) base[3 * 256 + k * 16 + i] = v[1][kk];
        if (k == 0) base[4 * 256 + j * 16 + i] = v[2][kk];
        if (k == 15) base[5 * 256 + j * 16 + i] = v[2][kk];
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
    const int c = ro_load(a.g.launch, w);
    MetaRO& m = meta_ro(a.g.meta, c);
    const double ih = 1.0 / m.h;
    const bool forced = !a.body || ro_byte(a.body, c) != 0;  // u* stored, else u* = u~
    const TF* src[3] = {forced ? a.ustar[0] : a.u[0], forced ? a.ustar[1] : a.u[1],
                        forced ? a.ustar[2] : a.u[2]};
    double acc[16];
    const auto gf = [&](int cc, int of, int aa, int bb) { return face_get(a.uf, cc, of, aa, bb); };
    // z component: neighbours along k are this lane's registers
    {
      TF v[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) v[k] = ld_nt(src[2] + (size_t)c * 4096 + k * 256 + t);
      double lo, hi;  // face velocities on the -z and +z faces of the column
      {
        const int k4 = kind_of(m, 4), k5 = kind_of(m, 5);
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
        v[k] = ld_nt(src[d] + (size_t)c * 4096 + k * 256 + t);
        tile[tix16(i, j, k)] = v[k];
      }
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int f = 2 * d + s;
        const int kd = kind_of(m, f);
        TF hv = TF(0);
        if (kd <= FK_FINER) hv = TF(RuleTab<RULE_U>::nbeff(kd)) * nb_raw<16, TF>(m, f, t1, t2, gf);
        else if (kd == FK_INFLOW) hv = TF(2.0 * (s ? -a.U_in : a.U_in));
        tile[halo16(f, t)] = hv;
      }
      __syncthreads();
      const int st = d == 0 ? 1 : 18;
      const double own_m = (d == 0 ? i == 0 : j == 0) ? RuleTab<RULE_U>::own(kind_of(m, 2 * d)) : 0.5;
      const double own_p = (d == 0 ? i == 15 : j == 15) ? RuleTab<RULE_U>::own(kind_of(m, 2 * d + 1)) : 0.5;
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
    for (int k = 0; k < 16; ++k) st_nt(a.b + (size_t)c * 4096 + k * 256 + t, acc[k] * ih * a.inv_c);
  }
}

// u_new = u* - c G_c p (cell velocities only; the face-velocity output uses k_correct).  The
// x/y neighbours of p go through LDS one plane at a time (two plane buffers used in turn);
// the halo ring of plane k comes from the lanes with j == k, which hold the x/y face values
// at z = k (tangential position (t1, t2) = (i, j) of faces 0..3).
template <typename TF, bool ML>
__global__ __launch_bounds__(256) void k16_correct(CorrectArgs<TF> a) {
  __shared__ double pl[2][P16];
  const int t = threadIdx.x, i = t & 15, j = t >> 4;
  const int n = a.g.n_cubes;
  for (int w = blockIdx.x; w < n; w += gridDim.x) {
    const int c = ro_load(a.g.launch, w);
    MetaRO& m = meta_ro(a.g.meta, c);
    double p[16], hv[6], rf[6];
    Slots S;
    slots<16, ML>(m, c, i, j, S);
#pragma unroll
    for (int f = 0; f < 6; ++f) rf[f] = a.pf[S.fine[f]];
#pragma unroll
    for (int k = 0; k < 16; ++k) p[k] = ld_nt(a.p + (size_t)c * 4096 + k * 256 + t);
#pragma unroll
    for (int f = 0; f < 6; ++f) hv[f] = halo_val<double>(S.kind[f], rf[f]);
    const double ch = a.c * 0.5 / m.h;
    const double ox_m = i == 0 ? RuleTab<RULE_P>::own(kind_of(m, 0)) : 1.0;
    const double ox_p = i == 15 ? RuleTab<RULE_P>::own(kind_of(m, 1)) : 1.0;
    const double oy_m = j == 0 ? RuleTab<RULE_P>::own(kind_of(m, 2)) : 1.0;
    const double oy_p = j == 15 ? RuleTab<RULE_P>::own(kind_of(m, 3)) : 1.0;
    const double oz_m = RuleTab<RULE_P>::own(kind_of(m, 4)), oz_p = RuleTab<RULE_P>::own(kind_of(m, 5));
    const int cc = (j + 1) * 18 + (i + 1);
    // u* of plane k + 1 is loaded while plane k is computed (the loads would otherwise start
    // only after each plane's barrier)
    const size_t g0 = (size_t)c * 4096 + t;
    const bool forced = !a.body || ro_byte(a.body, c) != 0;  // u* stored, else u* = u~
    const TF* src[3] = {forced ? a.ustar[0] : a.u[0], forced ? a.ustar[1] : a.u[1],
                        forced ? a.ustar[2] : a.u[2]};
    TF us[3], usn[3];
    // (loaded whether or not the component is written: a load under a branch makes the
    // following waits conservative)
#pragma unroll
    for (int d = 0; d < 3; ++d) usn[d] = ld_nt(src[d] + g0);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      double* b = pl[k & 1];
      b[cc] = p[k];
      if (j == k) {
        b[(i + 1) * 18 + 0] = hv[0];   // x = -1, y = i
        b[(i + 1) * 18 + 17] = hv[1];  // x = 16, y = i
        b[0 * 18 + (i + 1)] = hv[2];   // y = -1, x = i
        b[17 * 18 + (i + 1)] = hv[3];  // y = 16, x = i
      }
#pragma unroll
      for (int d = 0; d < 3; ++d) us[d] = usn[d];
      if (k < 15) {
#pragma unroll
        for (int d = 0; d < 3; ++d) usn[d] = ld_nt(src[d] + g0 + (k + 1) * 256);
      }
      __syncthreads();
      const size_t g = g0 + k * 256;
      const double gx = (b[cc + 1] - ox_p * p[k]) - (b[cc - 1] - ox_m * p[k]);
      const double gy = (b[cc + 18] - oy_p * p[k]) - (b[cc - 18] - oy_m * p[k]);
      const double zp = k < 15 ? p[k < 15 ? k + 1 : 15] - p[k] : hv[5] - oz_p * p[k];
      const double zm = k > 0 ? p[k > 0 ? k - 1 : 0] - p[k] : hv[4] - oz_m * p[k];
      if (a.unew[0]) st_nt(a.unew[0] + g, TF(double(us[0]) - ch * gx));
      if (a.unew[1]) st_nt(a.unew[1] + g, TF(double(us[1]) - ch * gy));
      if (a.unew[2]) st_nt(a.unew[2] + g, TF(double(us[2]) - ch * (zp - zm)));
    }
    __syncthreads();
  }
}

}  // namespace

// Persistent grid of one kernel: every workgroup resident at once (CUs x occupancy), rounded
// down to a multiple of 8 so each workgroup keeps to one XCD's stretch of the launch table.
static int grid_for(const void* fn, int units) {
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
  return std::max(1, std::min(g, fine_grid(units)));
}

template <class K, class A>
static hipError_t launch_col(K kernel, int cpb, const A& a, hipStream_t s) {
  const int units = col_units(cpb, a.g.n_cubes);
  hipLaunchKernelGGL(kernel, dim3(grid_for(reinterpret_cast<const void*>(kernel), units)), dim3(256),
                     0, s, a);
  return hipGetLastError();
}

#define BCM_COL_NL(NL, CALL)                            \
  switch (NL) {                                         \
    case 16: { constexpr int NLC = 16; CALL; } break;   \
    case 8: { constexpr int NLC = 8; CALL; } break;     \
    case 4: { constexpr int NLC = 4; CALL; } break;     \
    case 2: { constexpr int NLC = 2; CALL; } break;     \
    default: return hipErrorInvalidValue;               \
  }

template <typename T>
hipError_t launchc_smooth(int NL, const SmoothArgs<T>& a, hipStream_t s) {
  BCM_COL_NL(NL, {
    constexpr int cpb = Col<NLC>::CPB;
    if (a.g.multilevel) {
      if (a.zero_init && a.upd_q) return launch_col(kc_smooth<T, NLC, false, true, false, true>, cpb, a, s);
      if (a.zero_init) return launch_col(kc_smooth<T, NLC, false, true>, cpb, a, s);
      return launch_col(kc_smooth<T, NLC, true, true>, cpb, a, s);
    }
    if (a.zero_init && a.upd_q) return launch_col(kc_smooth<T, NLC, false, false, false, true>, cpb, a, s);
    if (a.zero_init) return launch_col(kc_smooth<T, NLC, false, false>, cpb, a, s);
    if (a.nb27) return launch_col(kc_smooth<T, NLC, true, false, true>, cpb, a, s);
    return launch_col(kc_smooth<T, NLC, true, false>, cpb, a, s);
  });
  return hipSuccess;
}
template <typename T>
hipError_t launchc_rfix(int NL, const RestrictFixArgs<T>& a, hipStream_t s) {
  BCM_COL_NL(NL, {
    if (a.g.multilevel) return launch_col(kc_rfix<T, NLC, true>, Col<NLC>::CPB, a, s);
    return launch_col(kc_rfix<T, NLC, false>, Col<NLC>::CPB, a, s);
  });
  return hipSuccess;
}
template <typename T>
hipError_t launchc_apply(int NL, const ApplyArgs<T>& a, hipStream_t s) {
  BCM_COL_NL(NL, {
    if (a.g.multilevel) return launch_col(kc_apply<T, NLC, true>, Col<NLC>::CPB, a, s);
    return launch_col(kc_apply<T, NLC, false>, Col<NLC>::CPB, a, s);
  });
  return hipSuccess;
}
template <typename TO>
hipError_t launchc_resid64(int NL, const Resid64Args<TO>& a, hipStream_t s) {
  BCM_COL_NL(NL, {
    if (a.g.multilevel) return launch_col(kc_resid64<TO, NLC, true>, Col<NLC>::CPB, a, s);
    return launch_col(kc_resid64<TO, NLC, false>, Col<NLC>::CPB, a, s);
  });
  return hipSuccess;
}
template <typename T>
hipError_t launchc_ir(int NL, const IrArgs<T>& a, hipStream_t s) {
  BCM_COL_NL(NL, {
    const int units = col_units(Col<NLC>::CPB, a.g.n_cubes);
    if (a.g.multilevel)
      hipLaunchKernelGGL((kc_ir<T, NLC, true>), dim3(std::min(units, 4096)), dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((kc_ir<T, NLC, false>), dim3(std::min(units, 4096)), dim3(256), 0, s, a);
    return hipGetLastError();
  });
  return hipSuccess;
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
    hipLaunchKernelGGL((k16_correct<TF, true>), dim3(std::min(a.g.n_cubes, 2048)), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k16_correct<TF, false>), dim3(std::min(a.g.n_cubes, 2048)), dim3(256), 0, s, a);
  return hipGetLastError();
}

#define BCM_INSTC(T)                                                                  \
  template hipError_t launchc_smooth<T>(int, const SmoothArgs<T>&, hipStream_t);      \
  template hipError_t launchc_rfix<T>(int, const RestrictFixArgs<T>&, hipStream_t);      \
  template hipError_t launchc_apply<T>(int, const ApplyArgs<T>&, hipStream_t);        \
  template hipError_t launchc_resid64<T>(int, const Resid64Args<T>&, hipStream_t);    \
  template hipError_t launchc_ir<T>(int, const IrArgs<T>&, hipStream_t);              \
  template hipError_t launch16_force<T>(const ForceArgs<T>&, hipStream_t);            \
  template hipError_t launch16_div<T>(const DivArgs<T>&, hipStream_t);                \
  template hipError_t launch16_correct<T>(const CorrectArgs<T>&, hipStream_t);
BCM_INSTC(float)
BCM_INSTC(double)

}  // namespace bcm
