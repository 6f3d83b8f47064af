// LDS tile machinery of the projection and adjoint kernels for every cube size and of the
// face export (device code), plus the operator rules and reductions that the column kernels
// of the solver (kernels_col.hip) share.
//
// A workgroup owns CPB cubes of NL^3 cells at one multigrid level.  Each cube is staged in
// LDS as an (NL+2)^3 tile: the cube's cells plus a one-cell halo on its six faces (no edges
// or corners: the 7-point stencil never reads them).  Halo values come from the face
// buffers of the neighbouring cubes: every field with a halo carries a buffer
// faces[cube][face][t2][t1] of the cube's own boundary layer (t1, t2 = tangential cell
// indices, first tangential axis fastest), written by the kernel that produced the field.
// (Behind the six slabs the buffer holds their 2x2 means, see face_stride; the tile kernels
// do not use them.)  The halo fill reads those contiguous 1-D slabs instead of strided
// columns of the neighbour's cube, and applies the face relation:
//   same level    -> the neighbour's boundary cell;
//   coarser (2:1) -> the coarse cell covering this fine cell's face quadrant;
//   finer (2:1)   -> the mean of the 2x2 fine cells covering this cell's face;
//   domain boundary -> nothing (the boundary enters through the per-side own coefficient).
// The raw neighbour value is scaled per relation by the rule of the operator being applied
// (RuleP, RuleU, RuleV, RuleL below) so that, after staging, every side of every cell reads
//   neighbour term = int_scale * tile[neighbour]   and   own term = own(side) * x_cell
// with own(side) = int_own inside the cube and the rule's table value on cube faces.
#pragma once

#include <hip/hip_runtime.h>

#include "bcm_internal.hpp"

namespace bcm {

constexpr int WG = 256;

// Streaming (non-temporal) global accesses for field values that a kernel reads or writes
// once: they bypass the cache retention that face slabs and scalars benefit from.
template <typename T>
__device__ __forceinline__ T ld_nt(const T* p) {
  return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ __forceinline__ void st_nt(T* p, T v) {
  __builtin_nontemporal_store(v, p);
}

// Tables that no kernel writes (cube metadata, the launch order) are read through the constant
// address space: with a wave-uniform index that is a scalar load, counted apart from the vector
// memory operations.  A vector load of the same value would make every wait on it (a branch on
// a face kind, a readfirstlane of a cube index) also wait for all loads and stores issued
// before it, the prefetched columns and the previous cube's stores included.
template <typename T>
__device__ __forceinline__ T ro_load(const T* p, size_t i) {
  return ((const __attribute__((address_space(4))) T*)(p))[i];
}
// A dword that may alias any other type (the byte fields below are read as whole dwords).
typedef uint32_t __attribute__((may_alias)) u32_alias;

// Byte i of a read-only byte table, from the dword that holds it (the table is padded to a
// multiple of 4 bytes).
__device__ __forceinline__ int ro_byte(const uint8_t* p, size_t i) {
  const uint32_t w = ((const __attribute__((address_space(4))) u32_alias*)(p))[i >> 2];
  return int((w >> (8 * (i & 3))) & 0xFFu);
}
// A cube's metadata in place, by reference through the constant address space (the helpers
// that read metadata take it as a template type, so LDS copies work as well).
using MetaRO = const __attribute__((address_space(4))) CubeMeta;
__device__ __forceinline__ MetaRO& meta_ro(const CubeMeta* p, size_t i) { return ((MetaRO*)p)[i]; }
// Face kind and quadrant of face f.  Through MetaRO each is taken from the dword that holds it
// (scalar loads fetch whole dwords; a byte access would be a vector load again).
__device__ __forceinline__ int meta_byte(MetaRO& m, int b) {
  const uint32_t w = ((const __attribute__((address_space(4))) u32_alias*)&m)[b >> 2];
  return int(int8_t(w >> (8 * (b & 3))));
}
__device__ __forceinline__ int kind_of(const CubeMeta& m, int f) { return m.kind[f]; }
__device__ __forceinline__ int kind_of(MetaRO& m, int f) { return meta_byte(m, offsetof(CubeMeta, kind) + f); }
__device__ __forceinline__ int quad_of(const CubeMeta& m, int f) { return m.quad[f]; }
__device__ __forceinline__ int quad_of(MetaRO& m, int f) { return meta_byte(m, offsetof(CubeMeta, quad) + f); }

template <int NL>
struct Lv {
  static constexpr int N = NL, N2 = NL * NL, N3 = NL * NL * NL;
  static constexpr int T = NL + 2, T2 = T * T, TILE = T * T * T;
  static constexpr int CPB = (N3 >= WG) ? 1 : WG / N3;  // cubes per workgroup
  static constexpr int FACE = face_stride(NL);          // face-buffer values per cube
};

template <int NL>
__device__ __forceinline__ int ti(int i, int j, int k) {
  constexpr int T = NL + 2;
  return ((k + 1) * T + (j + 1)) * T + (i + 1);
}

// Cell of face f (0..5 = -x,+x,-y,+y,-z,+z) at tangential position (t1, t2).
template <int NL>
__device__ __forceinline__ void face_cell(int f, int t1, int t2, int& i, int& j, int& k) {
  const int lay = (f & 1) ? NL - 1 : 0;
  const int d = f >> 1;
  i = d == 0 ? lay : t1;
  j = d == 1 ? lay : (d == 0 ? t1 : t2);
  k = d == 2 ? lay : t2;
}

template <int NL>
__device__ __forceinline__ int halo_idx(int f, int t1, int t2) {
  const int lay = (f & 1) ? NL : -1;
  const int d = f >> 1;
  if (d == 0) return ti<NL>(lay, t1, t2);
  if (d == 1) return ti<NL>(t1, lay, t2);
  return ti<NL>(t1, t2, lay);
}

// Raw neighbour value across face f of a cube at tangential cell (t1, t2).
// get(cube, face_of_that_cube, t1, t2) reads one value of that cube's face slab.
template <int NL, typename T, class Get, class MT>
__device__ __forceinline__ T nb_raw(const MT& m, int f, int t1, int t2, Get get) {
  const int of = f ^ 1;
  const int kd = kind_of(m, f);
  if (kd == FK_SAME) return get(m.nbr[f][0], of, t1, t2);
  if (kd == FK_COARSER) {
    const int q = quad_of(m, f);
    return get(m.nbr[f][0], of, (q & 1) * (NL / 2) + (t1 >> 1), (q >> 1) * (NL / 2) + (t2 >> 1));
  }
  if (kd == FK_FINER) {
    T s = T(0);
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int F1 = 2 * t1 + a, F2 = 2 * t2 + b;
        s += get(m.nbr[f][(F1 / NL) + 2 * (F2 / NL)], of, F1 % NL, F2 % NL);
      }
    return s * T(0.25);
  }
  return T(0);
}

// ---- operator rules (indexed by FaceKind: SAME, COARSER, FINER, OUTFLOW, INFLOW, SLIP) ----
// RuleP: 7-point Laplacian / face gradient of the pressure.  Side term = nb - own * x, so
//   (A x)_i = sum_sides (nb - own x_i) / h^2,  outward face derivative = (nb - own x_i) / h.
//   2:1 ghosts: fine side (2/3)(P - x) (centre distance 3h/2), coarse side (4/3)(mean - x).
// RuleU: face-normal velocity U = nb + own * u (linear interpolation to the face; inflow
//   faces carry the prescribed U_in, slip faces zero, open faces the boundary-cell value).
// RuleV: transpose of (cell gradient o face gradient): term = own * v + nb.
// RuleL: transpose of (face interpolation o divergence): term = own * lambda - nb.
enum Rule { RULE_P = 0, RULE_U = 1, RULE_V = 2, RULE_L = 3 };

template <int R>
struct RuleTab;
template <>
struct RuleTab<RULE_P> {
  static constexpr double int_scale = 1.0, int_own = 1.0;
  __device__ static double nbeff(int k) { return k == FK_SAME ? 1.0 : k == FK_COARSER ? 2.0 / 3.0 : k == FK_FINER ? 4.0 / 3.0 : 0.0; }
  __device__ static double own(int k) {
    return k == FK_SAME ? 1.0 : k == FK_COARSER ? 2.0 / 3.0 : k == FK_FINER ? 4.0 / 3.0 : k == FK_OUTFLOW ? 2.0 : 0.0;
  }
};
template <>
struct RuleTab<RULE_U> {
  static constexpr double int_scale = 0.5, int_own = 0.5;
  // halo stores neighbour contribution / int_scale
  __device__ static double nbeff(int k) { return k == FK_SAME ? 1.0 : k == FK_COARSER ? 2.0 / 3.0 : k == FK_FINER ? 4.0 / 3.0 : 0.0; }
  __device__ static double own(int k) {
    return k == FK_SAME ? 0.5 : k == FK_COARSER ? 2.0 / 3.0 : k == FK_FINER ? 1.0 / 3.0 : k == FK_OUTFLOW ? 1.0 : 0.0;
  }
};
template <>
struct RuleTab<RULE_V> {
  static constexpr double int_scale = 0.5, int_own = 0.5;
  __device__ static double nbeff(int k) { return k == FK_SAME ? 1.0 : k == FK_COARSER ? 1.0 / 6.0 : k == FK_FINER ? 16.0 / 3.0 : 0.0; }
  __device__ static double own(int k) {
    return k == FK_SAME ? 0.5 : k == FK_COARSER ? 1.0 / 3.0 : k == FK_FINER ? 2.0 / 3.0 : k == FK_OUTFLOW ? 1.0 : 0.0;
  }
};
template <>
struct RuleTab<RULE_L> {
  static constexpr double int_scale = 0.5, int_own = 0.5;
  __device__ static double nbeff(int k) { return k == FK_SAME ? 1.0 : k == FK_COARSER ? 1.0 / 6.0 : k == FK_FINER ? 16.0 / 3.0 : 0.0; }
  __device__ static double own(int k) {
    return k == FK_SAME ? 0.5 : k == FK_COARSER ? 2.0 / 3.0 : k == FK_FINER ? 1.0 / 3.0 : k == FK_OUTFLOW ? 1.0 : 0.0;
  }
};

// Stage the metadata of the workgroup's cubes in LDS.
template <int NL>
__device__ __forceinline__ void load_meta(CubeMeta* sm, int* cube, const CubeMeta* meta,
                                          const int32_t* launch, int n_cubes) {
  constexpr int CPB = Lv<NL>::CPB;
  const int base = blockIdx.x * CPB;
  for (int e = threadIdx.x; e < CPB * 32; e += blockDim.x) {
    const int s = e >> 5, w = e & 31;
    const int g = base + s;
    const int c = g < n_cubes ? launch[g] : -1;
    if (w == 0) cube[s] = c;
    reinterpret_cast<int32_t*>(&sm[s])[w] = c >= 0 ? reinterpret_cast<const int32_t*>(&meta[c])[w] : 0;
  }
  __syncthreads();
}

// Decompose a workgroup-local cell index into (slot, i, j, k).
template <int NL>
__device__ __forceinline__ void cell_of(int e, int& s, int& i, int& j, int& k) {
  constexpr int N3 = Lv<NL>::N3;
  s = e / N3;
  const int c = e - s * N3;
  i = c % NL;
  j = (c / NL) % NL;
  k = c / (NL * NL);
}

// Own coefficient of the side (face f) of cell (i,j,k) under rule R.
template <int NL, int R, class MT>
__device__ __forceinline__ double side_own(const MT& m, int f, int i, int j, int k) {
  const int d = f >> 1;
  const int c = d == 0 ? i : d == 1 ? j : k;
  const bool on = (f & 1) ? (c == NL - 1) : (c == 0);
  return on ? RuleTab<R>::own(kind_of(m, f)) : RuleTab<R>::int_own;
}

// Fill the six halo slabs of every cube of the workgroup under rule R.
// get(cube, face, t1, t2) returns a raw face value of a neighbour (see nb_raw);
// bcval(m, f) returns the value stored for a domain-boundary face (already / int_scale).
template <int NL, int R, typename T, class Get, class BcVal>
__device__ __forceinline__ void fill_halo(T* tile, const CubeMeta* sm, const int* cube, Get get,
                                          BcVal bcval, int fmask = 0x3F) {
  constexpr int CPB = Lv<NL>::CPB, N2 = Lv<NL>::N2, TILE = Lv<NL>::TILE;
  for (int e = threadIdx.x; e < CPB * 6 * N2; e += blockDim.x) {
    const int s = e / (6 * N2);
    const int r = e - s * 6 * N2;
    const int f = r / N2;
    const int t = r - f * N2;
    const int t1 = t % NL, t2 = t / NL;
    if (cube[s] < 0 || !((fmask >> f) & 1)) continue;
    const CubeMeta& m = sm[s];
    const int kd = m.kind[f];
    T v;
    if (kd <= FK_FINER)
      v = T(RuleTab<R>::nbeff(kd)) * nb_raw<NL, T>(m, f, t1, t2, get);
    else
      v = bcval(m, f);
    tile[s * TILE + halo_idx<NL>(f, t1, t2)] = v;
  }
}

// Deterministic workgroup sum (fixed shuffle tree, then waves in order); valid on thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < int(blockDim.x >> 6); ++w) t += sh[w];
  return t;
}

// ---- face getters and stencil helpers ----
template <int NL, typename T>
struct FaceGet {
  const T* f;
  __device__ T operator()(int c, int of, int t1, int t2) const {
    return f[(size_t)c * face_stride(NL) + of * NL * NL + t2 * NL + t1];
  }
};

template <typename T>
struct BcZero {
  __device__ T operator()(const CubeMeta&, int) const { return T(0); }
};

}  // namespace bcm
