// Kernel argument blocks and host launchers of the building-cube library.
#pragma once

#include <hip/hip_runtime.h>

#include "bcm_internal.hpp"

namespace bcm {

// Values per cube in the face buffer of a level with NL cells per cube edge: the six face
// slabs (NL^2 values each, the cube's boundary layer) followed by their 2x2 means ((NL/2)^2
// values each).  The means are written only for faces that border a coarser cube: that
// cube's halo takes one value per cell, the mean of the four finer cells facing it.
__host__ __device__ constexpr int face_stride(int NL) { return 6 * NL * NL + 6 * (NL / 2) * (NL / 2); }

// Device-resident scalars of one Krylov solve (written by k_finalize, read by the kernels).
struct Scalars {
  double rr, rr0, bb, zr, zq, pq, alpha, beta, gU, vuu, spare[6];
};

// Host-visible copy of the scalars (pinned, coherent host memory): k_finalize writes the
// scalars, then the sequence number, so that the host can poll for them instead of waiting
// for the stream.
struct ScalarMirror {
  Scalars sc;
  uint32_t seq;
};

struct Geom {  // what every cube-tiled kernel needs
  const CubeMeta* meta;
  const int32_t* launch;
  int n_cubes;
  double hscale;  // cell width at this level = meta.h * hscale
  int multilevel; // the mesh has 2:1 faces (a face may need four neighbour values)
};

template <typename T>
struct SmoothArgs {
  Geom g;
  T* x;                 // iterate (in/out)
  const T* b;           // right-hand side
  const T* xf_in;       // faces of x before the launch (unused when zero_init)
  T* xf_out;            // faces of x after the launch
  const T* xc;          // coarse correction to add first (level NL/2) or nullptr
  const T* xcf;         // its faces
  const uint32_t* nb27; // per launch position, the 27-neighbourhood of the cube: trilinear
                        // prolongation of xc (single-level meshes); nullptr = piecewise constant
  int sweeps, black_first, zero_init;
  T* bc;                // pre-smoother: restricted residual with the cross-cube terms left out
                        // (completed by the face correction), or nullptr
  const T* rfx;         // pre-smoother below the finest level: faces of the finer level's
                        // pre-smoothed iterate; b then lacks its cross-cube terms, which the
                        // launch adds first and stores back into b_fixed (= b).  nullptr: b is
                        // complete
  T* b_fixed;
  double rfx_hscale;    // cell width of the finer level = meta.h * rfx_hscale
  const T* r_dot;       // fused <x, r_dot>_V and <x, q_dot>_V (level 0 of a Krylov step)
  const T* q_dot;
  double* part_zr;
  double* part_zq;
  // pre-smoother of level 0: the previous Krylov step's r -= alpha q applied to b (= r) as it
  // is loaded and stored back, with the partial sums of <r, r>_V (one per workgroup, zeros
  // up to fine_grid(units)); upd_q == nullptr: b is used as it is
  const T* upd_q;
  const Scalars* upd_sc;
  double* part_rr;
};

template <typename T>
struct RestrictFixArgs {
  Geom g;
  const T* xf;          // faces of the pre-smoothed iterate
  T* bc;                // restricted residual, level NL/2 (in/out)
};

template <typename T>
struct ApplyArgs {      // p = z + beta p (p = z on the first step); q = A p; <p, q>_V
  Geom g;
  const T* z;
  const T* zf;
  T* p;
  const T* pf_in;
  T* pf_out;
  T* q;
  const Scalars* sc;
  int first;
  double* part;
};

template <typename T>
struct UpdateArgs {     // x += alpha p; r -= alpha q; <r, r>_V
  const CubeMeta* meta;
  int n_cubes, n3;
  T* x;
  const T* p;
  T* r;
  const T* q;
  const Scalars* sc;
  double* part;
  int x_zero;           // x starts at zero (not read)
  int part_sel;         // 0: x and r; 1: r and <r, r> only; 2: x only; 3: <r', r'> of the
                        // updated r' only (r not written)
};

template <typename TO>
struct Resid64Args {    // r = b - A p in FP64 (or r = A p when b is nullptr); norms
  Geom g;
  const double* p;      // nullptr = zero
  const double* pf;
  const double* b;
  TO* r;
  double* part_rr;
  double* part_bb;
  double rscale;        // r is stored multiplied by rscale
};

template <typename T>
struct IrArgs {         // p += dscale * d (when d != nullptr); export faces of p
  Geom g;
  double* p;
  const T* d;
  double* pf_out;
  double dscale;
  int p_zero;           // p is zero and not read (p = dscale * d)
  // the inner solve's last x update, applied here (when pdir != nullptr): d + alpha pdir in
  // T precision, with d taken as zero (not read) when d_zero
  const T* pdir;
  const Scalars* sc;
  int d_zero;
};

template <typename T, typename TO>
struct ExportArgs {
  Geom g;
  const T* x;
  TO* xf;
  int comp_faces;       // 1: x is a 3-component field set, face f takes component f >> 1
  const T* x3[3];
};

struct FinalizeArgs {
  const double* p0;
  const double* p1;
  int n;
  Scalars* sc;
  int op;
  int first;
  ScalarMirror* mirror;  // nullptr: none
  uint32_t seq;          // written to mirror->seq after the scalars
};
enum { OP_BB = 0, OP_RR0 = 1, OP_ZRZQ = 2, OP_PQ = 3, OP_RR = 4, OP_GU = 5, OP_VUU = 6, OP_B0 = 7 };

template <typename T>
struct CoarseArgs {
  const CubeMeta* meta;
  int n_cubes;
  double hscale;
  const T* b;
  T* x;
  T* xf;
  double* w;            // 4 * n_cubes doubles
  int iters;
};

template <typename TF>
struct ForceArgs {      // u* = (1 - alpha) u~ + alpha u_s; export face-normal components
  Geom g;
  const TF* u[3];
  const TF* alpha;
  const TF* us[3];
  double usc[3];
  TF* ustar[3];
  TF* uf;
  uint8_t* body;        // 16^3 only: per cube 1 if forced (some alpha != 0), else u* = u~ and only
                        // its faces are written; nullptr = every cube forced and stored
};

template <typename TF>
struct DivArgs {        // b = (rho/dt) div(U*)
  Geom g;
  const TF* ustar[3];
  const TF* u[3];       // u~, read instead of u* in cubes whose body flag is 0
  const uint8_t* body;  // nullptr: u* everywhere
  const TF* uf;
  double U_in, inv_c;
  double* b;
  double* part_bb;
};

template <typename TF>
struct CorrectArgs {    // u_new = u* - c G_c p; optional face velocities U* - c G p
  Geom g;
  const double* p;
  const double* pf;
  const TF* ustar[3];
  const TF* u[3];       // u~, read instead of u* in cubes whose body flag is 0 (16^3 kernel)
  const uint8_t* body;  // nullptr: u* everywhere
  const TF* uf;
  double U_in, c;
  TF* unew[3];
  TF* face_u[3];
};

template <typename TF>
struct AdjGpArgs {      // out = ((c/h) sum_s sigma_s term_s(v) + g_p) / vol
  Geom g;
  const TF* v[3];
  const TF* vf;
  const double* gp_in;
  double c;
  double* out;
};

template <typename TF>
struct AdjRhsArgs {     // g_u* = g_u_new + (1/c) W^T D^T lambda; forcing transpose; g_U_in
  Geom g;
  const double* lam;
  const double* lamf;
  const TF* gun[3];
  const TF* u[3];
  const TF* alpha;
  const TF* us[3];
  double usc[3];
  double inv_c;
  TF* gu[3];
  TF* galpha;
  int accumulate;       // galpha += instead of =
  double* part_gU;
};

template <typename TF>
struct KineticArgs {    // sum_i V_i |u_i|^2 (partials per workgroup); g_u = gscale V u
  const CubeMeta* meta;
  int n_cubes, n3;
  const TF* u[3];
  TF* gu[3];            // nullptr: no seed
  double gscale;
  double* part;         // nullptr: no sum
};

// Momentum sub-step (kernels_mom.hip).  Two-layer face buffers: 12 n^2 values per cube and
// component.
enum { MOM_EXPLICIT = 0, MOM_CN_START = 1, MOM_CN_ITER = 2 };

template <typename TF>
struct MomExportArgs {
  int n_cubes;
  const TF* x[3];
  TF* xf[3];
};

template <typename TF>
struct MomArgs {
  // MOM_EXPLICIT  out = v + dt (c1 H(v) + c2 hprev)                 (v = a = u^n)
  // MOM_CN_START  rhs = v + dt/2 H(v); out = v + dt H(v); part: sum rhs^2   (v = a = u^n)
  // MOM_CN_ITER   r = rhs + dt/2 H(v) - v; out = v + r / diag; part: sum r^2 (v = iterate)
  // every mode: hout = H(v) (optional), outf = two-layer x faces of out (optional); vf / af:
  // the x faces of v / a (their y and z halos are read from v / a themselves)
  const CubeMeta* meta;
  int n_cubes;
  const TF* v[3];
  const TF* vf[3];
  const TF* a[3];
  const TF* af[3];
  const TF* hprev[3];
  TF* rhs[3];
  TF* out[3];
  TF* outf[3];
  TF* hout[3];
  double U_in, nu, dt, c1, c2;
  double* part;
};

// Lagrangian-particle forcing (kernels_ib.hip).  Point location: per refinement level present
// (finest first), a dense table over the bounding box of that level's cubes on its lattice,
// anchored at the minimum corner of the coarsest level's cubes; entry = cube index or -1.
struct IbLevel {
  int level;
  int lo[3], dims[3];     // lattice position of the table's first entry and its extent
  long long offset;       // first entry in the table array
  double edge;            // cube edge of the level
};
constexpr int kIbMaxLevels = 24;

template <typename TF>
struct IbArgs {
  const CubeMeta* meta;
  int n_cubes, n;
  const int32_t* table;
  IbLevel lev[kIbMaxLevels];
  int n_levels;
  double anchor[3];
  int n_particles;
  const double* X;        // [n_particles][3]
  const double* dV;       // [n_particles] or nullptr (h^3)
  const double* Us;       // [n_particles][3] or nullptr (usc)
  double usc[3];
  const TF* u[3];         // u~ (read)
  TF* ustar[3];           // u* (holds u~ on entry; the spread is added)
  double rho_dt, dt_rho;
  double* Up;             // [n_particles][3] or nullptr
  double* Fp;             // [n_particles][3] or nullptr
  unsigned int* errors;   // particles skipped (outside the mesh, or support leaving one level)
};

// Wavelet compression of an FP64 cell field (kernels_codec.hip).
struct CodecArgs {
  int n_cubes, n, levels;
  double step;
  const double* field;          // encode input
  uint32_t* codes;              // [n_cubes][n^3] zigzag codes (workspace)
  uint8_t* widths;              // [n_cubes][n^3 / 32] group bit widths (workspace)
  unsigned long long* sizes;    // [n_cubes] stream bytes of each cube (workspace)
  unsigned long long* total;    // data bytes of the whole stream (workspace)
  void* stream;                 // encode output
  const void* stream_in;        // decode input
  unsigned long long data_bytes;  // decode: bytes after the header and offsets
  double* field_out;            // decode output
  unsigned int* flags;          // bit 0: a code beyond 2^30; bit 1: a malformed cube stream
};
hipError_t launch_wc_encode(int NL, const CodecArgs& a, int grid, hipStream_t s);
hipError_t launch_wc_header(const CodecArgs& a, hipStream_t s);
hipError_t launch_wc_pack(int NL, const CodecArgs& a, int grid, hipStream_t s);
hipError_t launch_wc_decode(int NL, const CodecArgs& a, int grid, hipStream_t s);

struct ScaleArgs {      // y = x * (vol ^ power) per cube (power = +1 or -1)
  const CubeMeta* meta;
  int n_cubes, n3;
  const double* x;
  double* y;
  int power;
};

// Launchers (return hipError_t of the launch).
template <typename T> hipError_t launch_smooth(int NL, const SmoothArgs<T>& a, hipStream_t s);
template <typename T> hipError_t launch_apply(int NL, const ApplyArgs<T>& a, hipStream_t s);
template <typename T> hipError_t launch_update(const UpdateArgs<T>& a, hipStream_t s);
template <typename TO> hipError_t launch_resid64(int NL, const Resid64Args<TO>& a, hipStream_t s);
template <typename T> hipError_t launch_ir(int NL, const IrArgs<T>& a, hipStream_t s);
template <typename T, typename TO> hipError_t launch_export(int NL, const ExportArgs<T, TO>& a, hipStream_t s);
hipError_t launch_finalize(const FinalizeArgs& a, hipStream_t s);
template <typename T> hipError_t launch_coarse(const CoarseArgs<T>& a, hipStream_t s);
template <typename TF> hipError_t launch_force(int NL, const ForceArgs<TF>& a, hipStream_t s);
template <typename TF> hipError_t launch_div(int NL, const DivArgs<TF>& a, hipStream_t s);
template <typename TF> hipError_t launch_correct(int NL, const CorrectArgs<TF>& a, hipStream_t s);
template <typename TF> hipError_t launch_adj_gp(int NL, const AdjGpArgs<TF>& a, hipStream_t s);
template <typename TF> hipError_t launch_adj_rhs(int NL, const AdjRhsArgs<TF>& a, hipStream_t s);
hipError_t launch_scale(const ScaleArgs& a, hipStream_t s);
template <typename TF> hipError_t launch_kinetic(const KineticArgs<TF>& a, int grid, hipStream_t s);
template <typename TF> hipError_t launch_mom_export(int NL, const MomExportArgs<TF>& a, int grid, hipStream_t s);
template <typename TF> hipError_t launch_ib_force(const IbArgs<TF>& a, hipStream_t s);
hipError_t launch_zero_u32(unsigned int* p, hipStream_t s);
template <typename TF> hipError_t launch_mom(int NL, int mode, const MomArgs<TF>& a, int grid, hipStream_t s);
template <typename T> hipError_t launch_coarse_mg(const CoarseMGArgs<T>& a, hipStream_t s);
// Multi-workgroup steps on one large graph level; n = lanes (cubes, nodes of the range, nodes
// of the level for G_RESID, or nodes of the coarser level for G_RESTRICT).
enum { G_GATHER = 0, G_SMOOTH = 1, G_RESTRICT = 2, G_PROLONG = 3, G_SCATTER = 4, G_RESID = 5 };
template <typename T> hipError_t launch_g_step(int kind, int n, const GStepArgs<T>& a, hipStream_t s);

// Persistent column kernels of the per-cube levels (kernels_col.hip).  A workgroup handles
// units of col_cpb(NL) cubes; the grid never exceeds fine_grid(units) workgroups, and the
// kernels that reduce write fine_grid(units) partial sums (zeros past their own grid).
__host__ __device__ inline int fine_grid(int units) { return units < 4096 ? units : 4096; }
__host__ __device__ inline int col_cpb(int NL) { return NL >= 16 ? 1 : 256 / (NL * NL); }
__host__ __device__ inline int col_units(int cpb, int n_cubes) {
  return cpb == 1 ? n_cubes : 8 * ((n_cubes + 8 * cpb - 1) / (8 * cpb));
}
template <typename T> hipError_t launchc_smooth(int NL, const SmoothArgs<T>& a, hipStream_t s);
template <typename T> hipError_t launchc_rfix(int NL, const RestrictFixArgs<T>& a, hipStream_t s);
template <typename T> hipError_t launchc_apply(int NL, const ApplyArgs<T>& a, hipStream_t s);
template <typename TO> hipError_t launchc_resid64(int NL, const Resid64Args<TO>& a, hipStream_t s);
template <typename T> hipError_t launchc_ir(int NL, const IrArgs<T>& a, hipStream_t s);
template <typename TF> hipError_t launch16_force(const ForceArgs<TF>& a, hipStream_t s);
template <typename TF> hipError_t launch16_div(const DivArgs<TF>& a, hipStream_t s);
template <typename TF> hipError_t launch16_correct(const CorrectArgs<TF>& a, hipStream_t s);

// Number of partial sums a column kernel at level NL writes.
inline int partials_of(int NL, int n_cubes) { return fine_grid(col_units(col_cpb(NL), n_cubes)); }

// Cubes per workgroup of the LDS-tile kernels (tile.hpp).
inline int cubes_per_wg(int NL) {
  const int n3 = NL * NL * NL;
  return n3 >= 256 ? 1 : 256 / n3;
}

}  // namespace bcm
