// Per-cube lossy wavelet compression of an FP64 cell field (Sec. 6.4.1, Alg. "Compression
// algorithm"): each cube is transformed on its own (CDF 5/3 lifting along x, y and z, log2(n)
// levels, symmetric extension at the cube's faces, coarse half of each axis first), its
// coefficients quantised with one uniform step, and the codes packed in groups of 32 at the
// group's bit width (zigzag map for the sign).  The cubes' streams are concatenated behind a
// header that records where each one starts.  Stream layout (little-endian):
//   0 "BCMW" | 4 version 1 | 8 number of cubes | 12 n | 16 levels | 20 zero | 24 step (FP64)
//   32 cube offsets, (number of cubes + 1) x u64, relative to the data start
//   data: per cube the G = n^3/32 group widths (bytes, zero-padded to 4), then for each group
//   its w 32-bit words, code j at bits j w .. j w + w - 1.
//
// One workgroup per cube (grid-stride), the cube in LDS (FP64, 34 KB at n = 16 with its rows
// padded); lifting runs one line per lane.  The lifting scales by 1/2 and 1/4 (exact), the quantiser divides by the
// step (IEEE division) and rounds half to even, so the codes and bytes depend on no operation
// order that another implementation of the same steps could do differently.
#include "kernels.hpp"
#include "tile.hpp"

namespace bcm {

namespace {

// Forward lifting of one line of M values (M even) with stride st in LDS, in place, coarse
// half first.
template <int M>
__device__ __forceinline__ void lift_fwd(double* c, int base, int st) {
  constexpr int H = M / 2;
  double x[M], s[H], d[H];
#pragma unroll
  for (int q = 0; q < M; ++q) x[q] = c[base + q * st];
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const double right = 2 * i + 2 < M ? x[2 * i + 2 < M ? 2 * i + 2 : 0] : x[M - 2];
    d[i] = x[2 * i + 1] - (x[2 * i] + right) * 0.5;
  }
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const double left = i > 0 ? d[i > 0 ? i - 1 : 0] : d[0];
    s[i] = x[2 * i] + (left + d[i]) * 0.25;
  }
#pragma unroll
  for (int i = 0; i < H; ++i) {
    c[base + i * st] = s[i];
    c[base + (H + i) * st] = d[i];
  }
}

template <int M>
__device__ __forceinline__ void lift_inv(double* c, int base, int st) {
  constexpr int H = M / 2;
  double s[H], d[H], e[H];
#pragma unroll
  for (int i = 0; i < H; ++i) {
    s[i] = c[base + i * st];
    d[i] = c[base + (H + i) * st];
  }
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const double left = i > 0 ? d[i > 0 ? i - 1 : 0] : d[0];
    e[i] = s[i] - (left + d[i]) * 0.25;
  }
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const double right = i + 1 < H ? e[i + 1 < H ? i + 1 : 0] : e[H - 1];
    c[base + 2 * i * st] = e[i];
    c[base + (2 * i + 1) * st] = d[i] + (e[i] + right) * 0.5;
  }
}

// The cube in LDS with each x row padded by one value (row pitch NL + 1): lanes lifting x lines
// read values NL + 1 apart, not NL (a multiple of the bank count, every lane on one bank).
template <int NL>
struct Pad {
  static constexpr int R = NL + 1, P = NL * R, SIZE = NL * P;
  __device__ static int of(int e) { return e + e / NL; }  // element e = (k NL + j) NL + i
};

// One axis of one level over the M^3 corner block: lane t < M^2 takes one line.
template <int NL, int M, bool INV>
__device__ __forceinline__ void lift_axis(double* c, int axis) {
  using PD = Pad<NL>;
  for (int t = threadIdx.x; t < M * M; t += blockDim.x) {
    const int a = t % M, b = t / M;
    int base, st;
    if (axis == 0) {  // lines along i at (j, k) = (a, b)
      base = b * PD::P + a * PD::R;
      st = 1;
    } else if (axis == 1) {  // along j at (i, k)
      base = b * PD::P + a;
      st = PD::R;
    } else {  // along k at (i, j)
      base = b * PD::R + a;
      st = PD::P;
    }
    if (INV)
      lift_inv<M>(c, base, st);
    else
      lift_fwd<M>(c, base, st);
  }
  __syncthreads();
}

// Levels M = NL, NL/2, ..., 2: forward x, y, z per level going down; inverse z, y, x per level
// coming back up.
template <int NL, int M>
__device__ __forceinline__ void dwt_fwd(double* c) {
  lift_axis<NL, M, false>(c, 0);
  lift_axis<NL, M, false>(c, 1);
  lift_axis<NL, M, false>(c, 2);
  if constexpr (M > 2) dwt_fwd<NL, M / 2>(c);
}

template <int NL, int M>
__device__ __forceinline__ void dwt_inv(double* c) {
  if constexpr (M > 2) dwt_inv<NL, M / 2>(c);
  lift_axis<NL, M, true>(c, 2);
  lift_axis<NL, M, true>(c, 1);
  lift_axis<NL, M, true>(c, 0);
}

__device__ __forceinline__ int bit_length(uint32_t v) { return v ? 32 - __clz(v) : 0; }

// Pass 1: transform, quantise, zigzag codes; group widths and the cube's stream size.
template <int NL>
__global__ __launch_bounds__(256) void k_wc_encode(CodecArgs a) {
  constexpr int N3 = NL * NL * NL, G = N3 / 32;
  __shared__ double c[Pad<NL>::SIZE];
  __shared__ int wsum[8];
  // the next cube's values are loaded before this cube's codes are stored (a load issued after
  // a store would wait for it in the in-order memory counter)
  constexpr int PER = (N3 + 255) / 256;
  double nx[PER];
  auto fetch = [&](int cb) {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = r * 256 + threadIdx.x;
      nx[r] = e < N3 ? a.field[(size_t)cb * N3 + e] : 0.0;
    }
  };
  if (blockIdx.x < a.n_cubes) fetch(blockIdx.x);
  for (int cube = blockIdx.x; cube < a.n_cubes; cube += gridDim.x) {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = r * 256 + threadIdx.x;
      if (e < N3) c[Pad<NL>::of(e)] = nx[r];
    }
    __syncthreads();
    if (cube + gridDim.x < a.n_cubes) fetch(cube + gridDim.x);
    dwt_fwd<NL, NL>(c);
    int wacc = 0;
    for (int e0 = 0; e0 < N3; e0 += 256) {
      const int e = e0 + threadIdx.x;  // the 32 lanes of each half-wave form one group
      uint32_t z = 0;
      if (e < N3) {
        const double q = rint(c[Pad<NL>::of(e)] / a.step);
        if (!(fabs(q) < 1073741824.0)) {  // 2^30; also catches NaN
          atomicOr(a.flags, 1u);
        } else {
          const int qi = int(q);
          z = qi >= 0 ? uint32_t(qi) << 1 : (uint32_t(-qi) << 1) - 1u;
        }
        a.codes[(size_t)cube * N3 + e] = z;
      }
      int w = bit_length(z);
#pragma unroll
      for (int o = 16; o > 0; o >>= 1) w = max(w, __shfl_xor(w, o, 32));
      if (e < N3 && (e & 31) == 0) {
        a.widths[(size_t)cube * G + (e >> 5)] = uint8_t(w);
        wacc += w;
      }
    }
    // cube size in bytes: padded width table + 4 bytes per word
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wacc += __shfl_down(wacc, o, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = wacc;
    __syncthreads();
    if (threadIdx.x == 0) {
      int tot = 0;
      for (int w = 0; w < 4; ++w) tot += wsum[w];
      a.sizes[cube] = (unsigned long long)((G + 3) / 4 * 4) + 4ull * (unsigned long long)tot;
    }
    __syncthreads();
  }
}

// Header and cube offsets: one workgroup, exclusive scan of the cube sizes in chunks.
__global__ __launch_bounds__(1024) void k_wc_header(CodecArgs a) {
  __shared__ unsigned long long part[1024];
  __shared__ unsigned long long carry;
  unsigned char* h = static_cast<unsigned char*>(a.stream);
  if (threadIdx.x == 0) {
    const uint32_t head[6] = {0x574D4342u /* "BCMW" */, 1u, uint32_t(a.n_cubes), uint32_t(a.n),
                              uint32_t(a.levels), 0u};
    for (int i = 0; i < 6; ++i) reinterpret_cast<uint32_t*>(h)[i] = head[i];
    *reinterpret_cast<double*>(h + 24) = a.step;
    carry = 0;
  }
  __syncthreads();
  unsigned long long* offs = reinterpret_cast<unsigned long long*>(h + 32);
  for (int base = 0; base <= a.n_cubes; base += 1024) {
    const int e = base + threadIdx.x;
    const unsigned long long v = e < a.n_cubes ? a.sizes[e] : 0ull;
    part[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {  // inclusive Hillis-Steele scan
      const unsigned long long add = threadIdx.x >= o ? part[threadIdx.x - o] : 0ull;
      __syncthreads();
      part[threadIdx.x] += add;
      __syncthreads();
    }
    if (e <= a.n_cubes) offs[e] = carry + part[threadIdx.x] - v;  // exclusive
    __syncthreads();
    if (threadIdx.x == 0) carry += part[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.total[0] = carry;
}

// Pass 2: widths and packed words of every cube at its offset.
template <int NL>
__global__ __launch_bounds__(256) void k_wc_pack(CodecArgs a) {
  constexpr int N3 = NL * NL * NL, G = N3 / 32, GP = (G + 3) / 4 * 4;
  __shared__ int wpre[G + 1];
  __shared__ uint8_t wid[G];
  unsigned char* h = static_cast<unsigned char*>(a.stream);
  const unsigned long long* offs = reinterpret_cast<const unsigned long long*>(h + 32);
  unsigned char* data = h + 32 + 8 * (size_t)(a.n_cubes + 1);
  for (int cube = blockIdx.x; cube < a.n_cubes; cube += gridDim.x) {
    for (int g = threadIdx.x; g < G; g += 256) wid[g] = a.widths[(size_t)cube * G + g];
    __syncthreads();
    if (threadIdx.x == 0) {  // prefix of the widths (words before each group)
      int s = 0;
      for (int g = 0; g < G; ++g) {
        wpre[g] = s;
        s += wid[g];
      }
      wpre[G] = s;
    }
    __syncthreads();
    uint32_t* out = reinterpret_cast<uint32_t*>(data + offs[cube]);
    for (int t = threadIdx.x; t < GP / 4; t += 256) {  // width table, four bytes per word
      uint32_t v = 0;
      for (int b = 0; b < 4; ++b) {
        const int g = 4 * t + b;
        v |= uint32_t(g < G ? wid[g] : 0) << (8 * b);
      }
      out[t] = v;
    }
    uint32_t* words = out + GP / 4;
    const uint32_t* codes = a.codes + (size_t)cube * N3;
    for (int idx = threadIdx.x; idx < wpre[G]; idx += 256) {
      int lo = 0, hi = G - 1;  // group g with wpre[g] <= idx < wpre[g + 1]
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (wpre[mid] <= idx) lo = mid;
        else hi = mid - 1;
      }
      const int g = lo, w = wid[g], j = idx - wpre[g];
      const int b0 = 32 * j;  // the word's first bit within the group
      uint32_t v = 0;
      for (int i = b0 / w; i < 32 && i * w < b0 + 32; ++i) {
        const uint64_t z = codes[g * 32 + i];
        const int sh = i * w - b0;
        v |= uint32_t(sh >= 0 ? (z << sh) : (z >> (-sh)));
      }
      words[idx] = v;
    }
    __syncthreads();
  }
}

// Decode: unpack, dequantise, inverse transform.
template <int NL>
__global__ __launch_bounds__(256) void k_wc_decode(CodecArgs a) {
  constexpr int N3 = NL * NL * NL, G = N3 / 32, GP = (G + 3) / 4 * 4;
  __shared__ double c[Pad<NL>::SIZE];
  __shared__ int wpre[G + 1];
  __shared__ uint8_t wid[G];
  const unsigned char* h = static_cast<const unsigned char*>(a.stream_in);
  const unsigned long long* offs = reinterpret_cast<const unsigned long long*>(h + 32);
  const unsigned char* data = h + 32 + 8 * (size_t)(a.n_cubes + 1);
  for (int cube = blockIdx.x; cube < a.n_cubes; cube += gridDim.x) {
    const unsigned long long o0 = offs[cube], o1 = offs[cube + 1];
    const bool room = o1 >= o0 && o1 - o0 >= (unsigned long long)GP && o1 <= a.data_bytes;
    const uint32_t* in = reinterpret_cast<const uint32_t*>(data + (room ? o0 : 0));
    for (int g = threadIdx.x; g < G; g += 256) wid[g] = room ? uint8_t(in[g >> 2] >> (8 * (g & 3))) : 0;
    __syncthreads();
    if (threadIdx.x == 0) {
      int s = 0;
      bool ok = room;
      for (int g = 0; g < G; ++g) {
        ok = ok && wid[g] <= 32;
        wpre[g] = s;
        s += wid[g] <= 32 ? wid[g] : 0;
      }
      wpre[G] = s;
      if (!ok || o1 - o0 != (unsigned long long)GP + 4ull * s) {
        atomicOr(a.flags, 2u);
        wpre[G] = -1;  // this cube decodes to zeros
      }
    }
    __syncthreads();
    const bool valid = wpre[G] >= 0;
    const uint32_t* words = in + GP / 4;
    for (int e = threadIdx.x; e < N3; e += 256) {
      const int g = e >> 5, i = e & 31, w = valid ? int(wid[g]) : 0;
      uint64_t z = 0;
      if (w) {
        const int bit = i * w, wi = wpre[g] + (bit >> 5), sh = bit & 31;
        uint64_t two = words[wi];
        if (sh + w > 32) two |= uint64_t(words[wi + 1]) << 32;
        z = (two >> sh) & ((w == 32) ? 0xFFFFFFFFull : ((1ull << w) - 1));
      }
      const long long q = (z & 1) ? -(long long)((z + 1) >> 1) : (long long)(z >> 1);
      c[Pad<NL>::of(e)] = double(q) * a.step;
    }
    __syncthreads();
    dwt_inv<NL, NL>(c);
    for (int e = threadIdx.x; e < N3; e += 256) a.field_out[(size_t)cube * N3 + e] = c[Pad<NL>::of(e)];
    __syncthreads();
  }
}

}  // namespace

#define BCM_WC_NL(NLV, CALL)                          \
  switch (NLV) {                                      \
    case 16: { constexpr int NLC = 16; CALL; } break; \
    case 8: { constexpr int NLC = 8; CALL; } break;   \
    case 4: { constexpr int NLC = 4; CALL; } break;   \
    default: return hipErrorInvalidValue;             \
  }

hipError_t launch_wc_encode(int NL, const CodecArgs& a, int grid, hipStream_t s) {
  BCM_WC_NL(NL, hipLaunchKernelGGL((k_wc_encode<NLC>), dim3(grid), dim3(256), 0, s, a));
  return hipGetLastError();
}
hipError_t launch_wc_header(const CodecArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_wc_header, dim3(1), dim3(1024), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_wc_pack(int NL, const CodecArgs& a, int grid, hipStream_t s) {
  BCM_WC_NL(NL, hipLaunchKernelGGL((k_wc_pack<NLC>), dim3(grid), dim3(256), 0, s, a));
  return hipGetLastError();
}
hipError_t launch_wc_decode(int NL, const CodecArgs& a, int grid, hipStream_t s) {
  BCM_WC_NL(NL, hipLaunchKernelGGL((k_wc_decode<NLC>), dim3(grid), dim3(256), 0, s, a));
  return hipGetLastError();
}

}  // namespace bcm
