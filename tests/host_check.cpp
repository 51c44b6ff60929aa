// Host-side checks of libvie built with AddressSanitizer and
// UndefinedBehaviorSanitizer (host code only; no device is used): the block
// planner on assorted partitions (shape groups, expanded blocks, empty and
// ragged blocks, single layers), argument validation of the C ABI, and the
// plane-wave helper.  Prints "host_check ok" and exits 0 when every check
// holds; a sanitizer finding aborts the program.
#include <cmath>
#include <complex>
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "vie.h"

static int failures = 0;

#define CHECK(cond)                                                 \
  do {                                                              \
    if (!(cond)) {                                                  \
      std::printf("FAILED %s (line %d)\n", #cond, __LINE__);        \
      ++failures;                                                   \
    }                                                               \
  } while (0)

struct Input {
  vie_grid g{};
  std::vector<double> eps;   // interleaved complex
  std::vector<int32_t> bid;
  int n_blocks = 0;
};

// Pillars (one block each) on a slab (one block), like the metasurface case.
static Input pillars(int n, int cells, int nz, int slab) {
  Input in;
  in.g = vie_grid{n, n, nz, 0.025, 0.025, 0.025, 1.0};
  const int64_t nv = (int64_t)n * n * nz;
  in.eps.assign(2 * nv, 0.0);
  in.bid.assign(nv, -1);
  const int cell = n / cells;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < n; ++y)
      for (int x = 0; x < n; ++x) {
        const int64_t v = ((int64_t)z * n + y) * n + x;
        in.eps[2 * v] = 1.0;
        if (z < slab) {
          in.eps[2 * v] = 2.25;
          in.bid[v] = cells * cells;
          continue;
        }
        const int cx = x / cell, cy = y / cell;
        const double dx = x + 0.5 - (cx * cell + 0.5 * cell), dy = y + 0.5 - (cy * cell + 0.5 * cell);
        const double r = 0.2 * cell + 0.02 * (cx + cy);
        if (dx * dx + dy * dy <= r * r) {
          in.eps[2 * v] = 5.8;
          in.bid[v] = cy * cells + cx;
        }
      }
  in.n_blocks = cells * cells + 1;
  return in;
}

// Random mask, permittivity and block ids (some ids unused).
static Input random_input(unsigned seed, int nx, int ny, int nz, int n_blocks, double fill) {
  std::mt19937 rng(seed);
  std::uniform_real_distribution<double> u(0.0, 1.0);
  Input in;
  in.g = vie_grid{nx, ny, nz, 0.03 + 0.02 * u(rng), 0.03 + 0.02 * u(rng), 0.03 + 0.02 * u(rng), 1.0};
  const int64_t nv = (int64_t)nx * ny * nz;
  in.eps.assign(2 * nv, 0.0);
  in.bid.assign(nv, -1);
  for (int64_t v = 0; v < nv; ++v) {
    if (u(rng) < fill) {
      in.eps[2 * v] = 1.5 + 3.0 * u(rng);
      in.eps[2 * v + 1] = -0.3 * u(rng);
      in.bid[v] = (int32_t)(u(rng) * (n_blocks - 1));   // the last id stays empty
    } else {
      in.eps[2 * v] = 1.0;
    }
  }
  in.n_blocks = n_blocks;
  return in;
}

static vie_status plan(const Input& in, int overlap, vie_problem_info* info, std::vector<vie_group_plan>* gp) {
  gp->assign(64, vie_group_plan{});
  std::vector<int32_t> bg(std::max(1, in.n_blocks), -7);
  const vie_status st = vie_plan(&in.g, in.eps.data(), in.bid.empty() ? nullptr : in.bid.data(), in.n_blocks,
                                 overlap, info, gp->data(), (int32_t)gp->size(), in.bid.empty() ? nullptr : bg.data());
  if (st == VIE_OK && !in.bid.empty()) {
    // every non-empty block in exactly one group, in range
    std::vector<int> per(64, 0);
    for (int k = 0; k < in.n_blocks; ++k) {
      CHECK(bg[k] >= -1 && bg[k] < info->n_groups);
      if (bg[k] >= 0 && bg[k] < 64) per[bg[k]]++;
    }
    for (int i = 0; i < info->n_groups && i < 64; ++i) CHECK(per[i] == (*gp)[i].n_systems);
  }
  return st;
}

int main() {
  CHECK(vie_abi_version() == VIE_ABI_VERSION);
  vie_problem_info info{};
  std::vector<vie_group_plan> gp;

  // metasurface-like: 64 pillar blocks in one group, the slab in another
  {
    Input in = pillars(128, 8, 32, 8);
    CHECK(plan(in, 0, &info, &gp) == VIE_OK);
    CHECK(info.lx == 256 && info.ly == 256 && info.lz == 64);
    CHECK(info.n_blocks == 65);
    CHECK(info.n_groups >= 2);
    int systems = 0;
    for (int i = 0; i < info.n_groups; ++i) systems += gp[i].n_systems;
    CHECK(systems == 65);
    CHECK(info.footprint_bytes > 0);
    // expanded blocks grow the boxes
    vie_problem_info info1{};
    std::vector<vie_group_plan> gp1;
    CHECK(plan(in, 2, &info1, &gp1) == VIE_OK);
    CHECK(info1.n_blocks == 65 && info1.footprint_bytes >= info.footprint_bytes);
  }
  // random partitions, ragged shapes, empty ids, single layers, overlap
  for (unsigned seed = 0; seed < 24; ++seed) {
    const int nx = 1 + (int)(seed * 7 % 23), ny = 1 + (int)(seed * 5 % 19), nz = 1 + (int)(seed * 3 % 11);
    Input in = random_input(seed, nx, ny, nz, 2 + (int)(seed % 6), 0.2 + 0.03 * (seed % 20));
    for (int overlap : {0, 1, 3}) {
      const vie_status st = plan(in, overlap, &info, &gp);
      CHECK(st == VIE_OK);
      int systems = 0;
      for (int i = 0; i < info.n_groups && i < 64; ++i) {
        systems += gp[i].n_systems;
        CHECK(2 * gp[i].bx - 1 <= gp[i].lx && 2 * gp[i].by - 1 <= gp[i].ly && 2 * gp[i].bz - 1 <= gp[i].lz);
      }
      CHECK(systems == info.n_blocks);
    }
    // without blocks: no groups
    Input plain = in;
    plain.bid.clear();
    plain.n_blocks = 0;
    CHECK(plan(plain, 0, &info, &gp) == VIE_OK && info.n_groups == 0 && info.n_blocks == 0);
  }
  // all vacuum with blocks given: no non-empty block
  {
    Input in = random_input(99, 5, 4, 3, 3, 0.0);
    CHECK(plan(in, 0, &info, &gp) == VIE_OK && info.n_blocks == 0 && info.n_groups == 0);
  }
  // validation
  {
    Input in = random_input(7, 6, 5, 4, 3, 0.8);
    Input bad = in;
    bad.eps[10] = std::nan("");
    CHECK(plan(bad, 0, &info, &gp) == VIE_EINVAL);
    bad = in;
    for (size_t v = 0; v < bad.bid.size(); ++v)
      if (bad.bid[v] >= 0) {
        bad.bid[v] = bad.n_blocks;   // out of range on a scatterer voxel
        break;
      }
    CHECK(plan(bad, 0, &info, &gp) == VIE_EINVAL);
    bad = in;
    bad.g.nx = 0;
    CHECK(plan(bad, 0, &info, &gp) == VIE_EINVAL);
    bad = in;
    bad.g.nx = 300;
    CHECK(vie_plan(&bad.g, in.eps.data(), nullptr, 0, 0, &info, nullptr, 0, nullptr) == VIE_EINVAL);
    bad = in;
    bad.g.dz = -1.0;
    CHECK(plan(bad, 0, &info, &gp) == VIE_EINVAL);
    CHECK(plan(in, -1, &info, &gp) == VIE_EINVAL);
    CHECK(vie_plan(&in.g, in.eps.data(), in.bid.data(), in.n_blocks, 0, &info, nullptr, 4, nullptr) == VIE_EINVAL);
    CHECK(vie_plan(nullptr, in.eps.data(), nullptr, 0, 0, &info, nullptr, 0, nullptr) == VIE_EINVAL);
    CHECK(std::string(vie_last_error()).size() > 0);
    CHECK(vie_plan(&in.g, in.eps.data(), in.bid.data(), 0, 0, &info, nullptr, 0, nullptr) == VIE_EINVAL);
    CHECK(vie_solve(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == VIE_EINVAL);
    CHECK(vie_matvec(nullptr, 0, nullptr, nullptr, nullptr) == VIE_EINVAL);
    CHECK(vie_problem_destroy(nullptr) == VIE_OK);
    CHECK(vie_context_destroy(nullptr) == VIE_OK);
    CHECK(vie_wait(nullptr, 0.0, nullptr, nullptr, nullptr) == VIE_EINVAL);
    CHECK(vie_cancel(nullptr) == VIE_EINVAL);
  }
  // plane wave: unit amplitude, phase exp(-j k0 z) from the grid centre
  {
    const vie_grid g{5, 4, 7, 0.03, 0.05, 0.04, 0.7};
    const double kdir[3] = {0.0, 0.0, 1.0};
    const double pol[6] = {1.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    std::vector<double> e(2 * 3 * 5 * 4 * 7);
    CHECK(vie_plane_wave(&g, kdir, pol, e.data()) == VIE_OK);
    const double k0 = 2 * M_PI / g.wavelength;
    double err = 0;
    for (int z = 0; z < g.nz; ++z)
      for (int y = 0; y < g.ny; ++y)
        for (int x = 0; x < g.nx; ++x) {
          const int64_t v = ((int64_t)z * g.ny + y) * g.nx + x;
          const double zc = (z - (g.nz - 1) / 2.0) * g.dz;
          const std::complex<double> want = std::exp(std::complex<double>(0.0, -k0 * zc));
          err = std::max(err, std::abs(std::complex<double>(e[2 * v], e[2 * v + 1]) - want));
          const int64_t nv = (int64_t)g.nx * g.ny * g.nz;
          err = std::max(err, std::abs(e[2 * (nv + v)]) + std::abs(e[2 * (2 * nv + v)]));
        }
    CHECK(err <= 1e-13);
    const double bad_dir[3] = {0.0, 0.0, 2.0};
    CHECK(vie_plane_wave(&g, bad_dir, pol, e.data()) == VIE_EINVAL);
  }
  if (failures) {
    std::printf("host_check: %d failures\n", failures);
    return 1;
  }
  std::printf("host_check ok\n");
  return 0;
}
