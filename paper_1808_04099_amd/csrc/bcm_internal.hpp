// Internal types shared by the host code and the HIP kernels of the building-cube library.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "bcm.h"
#include "coarse.hpp"

namespace bcm {

// Relation of a cube face to what lies across it (device metadata, one byte per face).
enum FaceKind : int8_t {
  FK_SAME = 0,     // neighbour of the same level
  FK_COARSER = 1,  // neighbour one level coarser: this face covers one quadrant of its face
  FK_FINER = 2,    // four neighbours one level finer cover this face
  FK_OUTFLOW = 3,  // domain boundary, open (p = 0)
  FK_INFLOW = 4,   // domain boundary, prescribed inflow (dp/dn = 0)
  FK_SLIP = 5      // domain boundary, wall without penetration (dp/dn = 0)
};

// Per-cube device metadata: 128 bytes, read once per cube by the workgroup that owns it.
struct alignas(128) CubeMeta {
  int32_t nbr[6][4];  // neighbour cube indices (see bcm.h), -1 where absent
  int8_t kind[6];     // FaceKind per face
  int8_t quad[6];     // FK_COARSER: quadrant (bit0 = half along t1, bit1 = along t2)
  int8_t level;
  int8_t pad[3];
  double h;           // cell width at the finest (input) resolution of this cube
  double vol;         // cube volume relative to the smallest cube (1, 8, 64, ...)
};
static_assert(sizeof(CubeMeta) == 128, "CubeMeta must stay one 128-byte line");

struct HostMesh {
  int32_t n_cubes = 0, n = 0;
  double root_edge = 0;
  std::vector<double> origin;     // [n_cubes][3]
  std::vector<int8_t> level;
  std::vector<int32_t> nbr;       // [n_cubes][6][4]
  std::vector<int8_t> face_bc;    // [n_cubes][6]
  std::vector<CubeMeta> meta;     // derived device metadata
  std::vector<int32_t> launch;    // workgroup -> cube (Z-ordered, XCD-aware)
  std::vector<uint32_t> nb27;     // [launch position][27] resolved neighbours (pack_nb27);
                                  // single-level meshes only, else empty
  int max_level = 0;
  bool multilevel = false;
  bool has_inflow = false;
  CoarseHierarchy coarse;         // multigrid levels of the one-cell-per-cube graph
};

// One entry of the 27-neighbourhood table: the cube that holds the cell at offset
// (dx, dy, dz) in {-1, 0, 1}^3 from a cube, reached by stepping along x, then y, then z; a step
// across a domain boundary stays in the cube and marks that axis as clamped (the ghost mirrors
// the boundary cell), negated once per open (p = 0) face crossed.
//   bits 0..23: cube index; bits 24..26: clamped axes x, y, z; bit 27: negate.
constexpr uint32_t pack_nb27(int cube, int clamped, bool negate) {
  return uint32_t(cube) | (uint32_t(clamped) << 24) | (uint32_t(negate) << 27);
}
constexpr int kNb27MaxCubes = 1 << 24;

void set_error(const std::string& msg);

}  // namespace bcm

struct bcm_mesh {
  bcm::HostMesh m;
};
