// Cube-graph multigrid hierarchy (host description and device argument block).
#pragma once

#include <cstdint>
#include <vector>

namespace bcm {

struct HostMesh;

struct CoarseLevel {
  int n = 0;
  std::vector<int32_t> row, col;      // off-diagonal couplings (CSR)
  std::vector<double> val, diag;      // A_ij and A_ii of the 7-point composite operator
  std::vector<double> vol;            // relative node volume
  std::vector<int32_t> order;         // nodes grouped by colour
  std::vector<int32_t> color_off;     // colour c = order[color_off[c] .. color_off[c+1])
  std::vector<int32_t> parent;        // node -> node of the next coarser level
  std::vector<int32_t> child_row, child;  // (this level) node -> children on the finer level
  std::vector<double> child_w;        // restriction weights (volume fractions, sum 1)
};

struct CoarseHierarchy {
  bool ok = false;
  std::vector<CoarseLevel> levels;    // levels[0] = the one-cell-per-cube graph
};

bool build_coarse_hierarchy(const HostMesh& M, CoarseHierarchy& H, int max_levels);

// Device view of one graph level (pointers into the plan workspace).
template <typename T>
struct GLevel {
  int n, ncol;
  int color_off[9];         // up to 8 colours
  const int32_t* row;
  const int32_t* col;
  const T* val;
  const T* diag;
  const T* vol;             // relative node volume (V A is symmetric)
  const int32_t* order;
  const int32_t* parent;    // to the next coarser level (nullptr on the last)
  const int32_t* child_row; // from the next finer level (nullptr on level 0)
  const int32_t* child;
  const T* child_w;
  T* x;
  T* b;
  T* r;
};

constexpr int kMaxGraphLevels = 12;

template <typename T>
struct CoarseMGArgs {
  const T* b_in;            // one-cell-per-cube right-hand side (cube order)
  T* x_out;                 // solution (cube order)
  T* xf_out;                // its face buffer (6 copies per cube)
  const GLevel<T>* lev;     // device array of levels
  int nlev;
  int cycles, pre, post, bottom_iters;
  double* w;                // CG work space for the bottom level (4 * n_last doubles)
};

}  // namespace bcm
