// White-box check of the cube-graph hierarchy that bcm_mesh_create builds (host code only):
// every colour class is an independent set covering its level, and the packed 16-bit rows
// decode to the ELL columns exactly when every coupling of the level shares one value.
// Usage: graph_check DIR (DIR holds meta.txt, origin.bin, level.bin, nbr.bin, fbc.bin).
#include <cstdio>
#include <string>
#include <vector>

#include "bcm_internal.hpp"

static bool read_all(const std::string& path, void* dst, size_t bytes) {
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) return false;
  const size_t got = std::fread(dst, 1, bytes, f);
  std::fclose(f);
  return got == bytes;
}

int main(int argc, char** argv) {
  if (argc != 2) return 2;
  const std::string dir = argv[1];
  int nc = 0, n = 0;
  double root = 0.0;
  FILE* f = std::fopen((dir + "/meta.txt").c_str(), "r");
  if (!f || std::fscanf(f, "%d %d %lf", &nc, &n, &root) != 3) return 2;
  std::fclose(f);
  std::vector<double> origin(3 * size_t(nc));
  std::vector<int8_t> level(nc), fbc(6 * size_t(nc));
  std::vector<int32_t> nbr(24 * size_t(nc));
  if (!read_all(dir + "/origin.bin", origin.data(), origin.size() * 8) ||
      !read_all(dir + "/level.bin", level.data(), level.size()) ||
      !read_all(dir + "/nbr.bin", nbr.data(), nbr.size() * 4) ||
      !read_all(dir + "/fbc.bin", fbc.data(), fbc.size()))
    return 2;
  bcm_mesh_desc d{};
  d.n_cubes = nc;
  d.n = n;
  d.origin = origin.data();
  d.level = level.data();
  d.root_edge = root;
  d.nbr = nbr.data();
  d.face_bc = fbc.data();
  bcm_mesh* m = nullptr;
  if (bcm_mesh_create(&d, &m) != BCM_OK) {
    std::printf("mesh rejected: %s\n", bcm_last_error());
    return 1;
  }
  int bad = 0;
  const auto& H = m->m.coarse;
  for (size_t g = 0; g < H.levels.size(); ++g) {
    const bcm::CoarseLevel& L = H.levels[g];
    const int nl = L.n, nco = int(L.color_off.size()) - 1;
    // colour classes: contiguous device ranges, an independent set each, covering the level
    std::vector<int> colour_of(nl, -1);
    for (int c = 0; c < nco; ++c)
      for (int i = L.color_off[c]; i < L.color_off[c + 1]; ++i) colour_of[i] = c;
    for (int i = 0; i < nl; ++i)
      if (colour_of[i] < 0) ++bad, std::printf("level %zu: node %d has no colour\n", g, i);
    bool uniform = !L.val.empty();
    for (double v : L.val) uniform = uniform && v == L.val[0];
    for (int i = 0; i < nl; ++i)
      for (int w = 0; w < L.W; ++w) {
        const int c = L.e_col[size_t(w) * nl + i];
        if (c != i && colour_of[c] == colour_of[i])
          ++bad, std::printf("level %zu: nodes %d and %d couple within colour %d\n", g, i, c, colour_of[i]);
      }
    // packed rows exactly when eligible, decoding to the ELL columns
    const bool eligible = L.W == 6 && nl <= 65535 && uniform;
    if (eligible != !L.e_pcol.empty())
      ++bad, std::printf("level %zu: packed rows %s but eligible %d\n", g, L.e_pcol.empty() ? "absent" : "present", eligible);
    if (!L.e_pcol.empty()) {
      if (L.uval != L.val[0]) ++bad, std::printf("level %zu: uval differs from the couplings\n", g);
      for (int i = 0; i < nl; ++i)
        for (int w = 0; w < 6; ++w) {
          const uint32_t word = L.e_pcol[size_t(w / 2) * nl + i];
          const int c = int(w & 1 ? word >> 16 : word & 0xffffu);
          if (c != L.e_col[size_t(w) * nl + i])
            ++bad, std::printf("level %zu: packed column %d of node %d decodes to %d\n", g, w, i, c);
        }
    }
    std::printf("level %zu: %d nodes, W %d, %d colours, packed %d\n", g, nl, L.W, nco, int(!L.e_pcol.empty()));
  }
  bcm_mesh_destroy(m);
  std::printf(bad ? "FAILED (%d)\n" : "ok\n", bad);
  return bad ? 1 : 0;
}
