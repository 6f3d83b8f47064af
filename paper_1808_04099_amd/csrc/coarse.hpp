// Cube-graph multigrid hierarchy (host description and device argument block).
#pragma once

#include <cstdint>
#include <vector>

namespace bcm {

struct HostMesh;

struct CoarseLevel {
  int n = 0;
  // construction (nodes in key order)
  std::vector<int32_t> row, col;      // off-diagonal couplings (CSR)
  std::vector<double> val, diag;      // A_ij and A_ii of the 7-point composite operator
  std::vector<double> vol;            // relative node volume
  std::vector<int32_t> order;         // nodes grouped by colour
  std::vector<int32_t> color_off;     // colour c = order[color_off[c] .. color_off[c+1])
  std::vector<int32_t> parent;        // node -> node of the next coarser level
  std::vector<int32_t> child_row, child;  // (this level) node -> children on the finer level
  std::vector<double> child_w;        // restriction weights (volume fractions, sum 1)
  // device form (nodes renumbered so that every colour is contiguous)
  int W = 0, CW = 0;                  // ELL widths of the couplings and of the child lists
  std::vector<int32_t> e_col;         // [W][n], padding: own index with value 0
  std::vector<double> e_val;          // [W][n]
  std::vector<double> e_diag, e_vol;  // [n]
  std::vector<int32_t> e_parent;      // [n] (empty on the last level)
  std::vector<int32_t> e_child;       // [CW][n] children on the finer level, -1 padding
  std::vector<double> e_child_w;      // [CW][n]
  std::vector<int32_t> perm;          // level 0: perm[cube] = device node index
  // W = 6 levels whose couplings all have one value uval: the columns packed two per word,
  // [3][n] (low half = even slot; padding = own index), else empty
  std::vector<uint32_t> e_pcol;
  double uval = 0.0;
};

// The last graph level is solved directly (dense inverse) when it has at most this many nodes.
constexpr int kBottomDirectMax = 64;

struct CoarseHierarchy {
  bool ok = false;
  std::vector<CoarseLevel> levels;    // levels[0] = the one-cell-per-cube graph
  std::vector<double> bottom_inv;     // [n][n] transposed inverse of the last level, or empty
};

bool build_coarse_hierarchy(const HostMesh& M, CoarseHierarchy& H, int max_levels);

// Device view of one graph level (pointers into the plan workspace).  x, b and r live in
// global memory unless lds_* >= 0, in which case the kernel points them into its LDS.
template <typename T>
struct GLevel {
  int n, ncol, W, CW;
  int color_off[9];         // up to 8 colours, contiguous node ranges
  int lds_x, lds_b, lds_r;  // byte offsets in the kernel's dynamic LDS, or -1
  const int32_t* col;       // [W][n]
  const T* val;             // [W][n]
  const T* diag;
  const T* vol;             // relative node volume (V A is symmetric)
  const int32_t* parent;    // to the next coarser level (nullptr on the last)
  const int32_t* child;     // [CW][n] from the next finer level (nullptr on level 0)
  const T* child_w;
  T* x;
  T* b;
  T* r;
  const uint32_t* pcol;     // [3][n] packed 16-bit columns (every coupling = uval), or nullptr
  T uval;
};

constexpr int kMaxGraphLevels = 12;

template <typename T>
struct CoarseMGArgs {
  const T* b_in;            // one-cell-per-cube right-hand side (cube order)
  T* x_out;                 // solution (cube order)
  T* xf_out;                // its face buffer (6 copies per cube)
  const GLevel<T>* lev;     // device array of levels
  const int32_t* perm0;     // cube -> level-0 node
  int nlev;
  int start;                // first level this workgroup solves: 0, or the first level below
                            // the ones smoothed by the multi-workgroup kernels (its b and x
                            // then come from and go to the levels' global buffers)
  int cycles, pre, post, bottom_iters;
  double* w;                // CG work space for the bottom level (4 * n_last doubles)
  const T* binv;            // transposed inverse of the bottom operator, or nullptr (CG)
  int lds_bytes;            // dynamic LDS the launch reserves for the lds_* placements
  int lds_inv;              // byte offset in that LDS where the kernel keeps binv, or -1
  // Optional vector update x += alpha p carried out by xu_wgs further workgroups of the
  // same launch, beside the coarse solve (xu_n = 0: none).
  T* xu_x;
  const T* xu_p;
  const double* xu_alpha;
  size_t xu_n;
  int xu_zero;              // x starts at zero (not read)
  int xu_wgs;
};

constexpr int kGraphLdsBudget = 128 * 1024;
// Dynamic LDS the single workgroup may reserve in all (the rest of 160 KB is its static LDS).
constexpr int kGraphLdsTotal = 156 * 1024;

// Argument block of the multi-workgroup graph kernels.
template <typename T>
struct GStepArgs {
  const GLevel<T>* lev;     // device array of levels (global buffers)
  int g;                    // level
  int lo, hi;               // node range (one colour) of a smoothing pass
  const T* b_in;            // gather: one-cell-per-cube right-hand side (cube order)
  T* x_out;                 // scatter: solution (cube order)
  T* xf_out;                // and its face buffer
  const int32_t* perm0;
  int n_cubes;
};

}  // namespace bcm
