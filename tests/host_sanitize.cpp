// Host-code checker built with AddressSanitizer and UndefinedBehaviorSanitizer
// (g++ -fsanitize=address,undefined, no device code): drives the library's
// host-only parts -- the pixel mesh builder, the reference-element and
// quadrature builder, the BF16 split of operator entries, and the
// launch-shape table parser -- over ordinary and edge-case inputs, and
// checks their invariants.  Any out-of-bounds access,
// use after free, leak or undefined operation aborts with the sanitizer's
// report; a failed invariant exits with status 1.
//
// Built and run by tests/test_abi_cpu.py.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "../paper_1907_06191_amd/csrc/dgd_internal.h"
#include "../paper_1907_06191_amd/csrc/tune.h"

namespace dgd {
// The tuner's shape helper lives with the kernels (device code); the table
// parser under test never calls it.
Shape element_shape(int64_t E, int epw, int waves, bool xcd_remap, int64_t max_grid) {
  Shape s;
  s.epw = epw;
  s.waves = waves;
  s.remap = xcd_remap;
  s.blocks = (E + (int64_t)epw * waves - 1) / ((int64_t)epw * waves);
  s.grid = max_grid > 0 && max_grid < s.blocks ? max_grid : s.blocks;
  return s;
}
// device fills used only by the timing loop of the tuner (not run here)
void launch_fill_random(double*, int64_t, uint64_t, hipStream_t) { std::abort(); }
void launch_fill_random_f32(float*, int64_t, uint64_t, hipStream_t) { std::abort(); }
}  // namespace dgd

using namespace dgd;

static int g_fail = 0;
#define CHECK(c)                                                       \
  do {                                                                 \
    if (!(c)) {                                                        \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      g_fail = 1;                                                      \
    }                                                                  \
  } while (0)

// Face neighbours are mutual and of the other orientation; the counts agree.
static void check_mesh(const MeshHost& m) {
  const int64_t E = m.n_elements();
  CHECK((int64_t)m.ci.size() == E && (int64_t)m.cj.size() == E);
  CHECK((int64_t)m.nbr.size() == 3 * E);
  int64_t half_faces = 0;
  for (int64_t e = 0; e < E; ++e) {
    CHECK(m.ci[e] >= 0 && m.ci[e] < m.N && m.cj[e] >= 0 && m.cj[e] < m.N);
    CHECK(m.active_cell[(size_t)m.cj[e] * m.N + m.ci[e]] == 1);
    for (int f = 0; f < 3; ++f) {
      const int32_t n = m.nbr[3 * e + f];
      if (n < 0) continue;
      ++half_faces;
      CHECK(n < E);
      if (n >= E) continue;
      CHECK(m.orient[n] != m.orient[e]);
      CHECK(m.nbr[3 * (int64_t)n + f] == (int32_t)e);
    }
  }
  CHECK(half_faces == 2 * m.n_faces);
  CHECK(m.n_components >= (E > 0 ? 1 : 0));
}

static void meshes() {
  std::mt19937_64 rng(19070619);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  const int sizes[] = {1, 2, 3, 7, 16, 33, 64};
  for (int N : sizes) {
    for (int strip : {0, 1, 4, 64}) {
      for (int group : {1, 4}) {
        const double L = 0.37 * N;
        std::vector<double> disks;
        const int nd = (int)(U(rng) * 6);
        for (int d = 0; d < nd; ++d) {
          disks.push_back(U(rng) * L * 1.4 - 0.2 * L);   // may leave the box
          disks.push_back(U(rng) * L * 1.4 - 0.2 * L);
          disks.push_back(U(rng) * 0.3 * L);
        }
        MeshHost m;
        build_mesh_host(L, N, disks.data(), nd, strip, group, m);
        check_mesh(m);
      }
    }
  }
  // every cell removed; no disks; a disk touching centroids exactly (strict test)
  {
    MeshHost m;
    const double all[] = {5.0, 5.0, 100.0};
    build_mesh_host(10.0, 8, all, 1, 64, 4, m);
    CHECK(m.n_elements() == 0 && m.n_faces == 0);
  }
  {
    MeshHost m;
    build_mesh_host(10.0, 8, nullptr, 0, 64, 4, m);
    CHECK(m.n_elements() == 128);
    CHECK(m.n_faces == 64 + 2 * 8 * 7);
    check_mesh(m);
  }
  {
    MeshHost m;
    // centroid (0.5, 0.5) of cell (0, 0) at distance exactly 0.5 from (1, 0.5)
    const double d[] = {1.0, 0.5, 0.5};
    build_mesh_host(2.0, 2, d, 1, 64, 4, m);
    CHECK(m.active_cell[0] == 1);
    check_mesh(m);
  }
}

static void reference_elements() {
  for (int p = 1; p <= 3; ++p) {
    const RefElem R = build_ref_elem(p, 10.0);
    const int np = (p + 1) * (p + 2) / 2;
    CHECK(R.np == np);
    CHECK(R.S.size() == (size_t)2 * 8 * np * np && R.Nb.size() == (size_t)2 * 3 * np * np);
    std::vector<double> phi(np);
    for (int o = 0; o < 2; ++o) {
      // the nodal basis is the identity at the nodes
      for (int i = 0; i < np; ++i) {
        eval_nodal_basis(R, o, R.nodes[((size_t)o * np + i) * 2], R.nodes[((size_t)o * np + i) * 2 + 1],
                         phi.data());
        for (int j = 0; j < np; ++j) CHECK(std::fabs(phi[j] - (i == j ? 1.0 : 0.0)) < 1e-12);
      }
      // constants are annihilated: (S_{o,mask} + sum_{f in mask} N_{o,f}) 1 = 0
      for (int mask = 0; mask < 8; ++mask)
        for (int i = 0; i < np; ++i) {
          double row = 0, mag = 0;
          for (int j = 0; j < np; ++j) {
            double a = R.S[(((size_t)o * 8 + mask) * np + i) * np + j];
            for (int f = 0; f < 3; ++f)
              if (mask & (1 << f)) a += R.Nb[(((size_t)o * 3 + f) * np + i) * np + j];
            row += a;
            mag += std::fabs(a);
          }
          CHECK(std::fabs(row) <= 1e-12 * (mag + 1.0));
        }
    }
    const std::vector<double> q = build_ic_quadrature(R, 12);
    CHECK(q.size() == (size_t)2 * 144 * (np + 3));
  }
}

// The BF16 three-term split of operator entries (matrix-core tables):
// together within 2^-26 of the entry, terms shrinking by 2^-8 or more, a
// value that is already BF16 kept whole, zero split into zeros.
static void check_split(double a) {
  uint16_t t[3];
  split_bf16x3(a, t);
  const double v0 = bf16_value(t[0]), v1 = bf16_value(t[1]), v2 = bf16_value(t[2]);
  CHECK(std::fabs(a - (v0 + v1 + v2)) <= std::ldexp(std::fabs(a), -26));
  CHECK(std::fabs(v1) <= std::ldexp(std::fabs(v0), -8) * (1.0 + 1e-6));
  CHECK(std::fabs(v2) <= std::ldexp(std::fabs(v1), -8) * (1.0 + 1e-6));
}

static void bf16_split() {
  std::mt19937_64 rng(1907);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  std::uniform_int_distribution<int> X(-40, 40);
  for (int k = 0; k < 100000; ++k) check_split(std::ldexp(U(rng), X(rng)));
  for (int p = 1; p <= 3; ++p) {
    const RefElem R = build_ref_elem(p, 10.0);
    for (double a : R.S) check_split(a);
    for (double a : R.Nb) check_split(a);
  }
  for (double a : {1.0, -0.375, std::ldexp(3.0, -20), 0.0}) {
    uint16_t t[3];
    split_bf16x3(a, t);
    CHECK(bf16_value(t[0]) == a && t[1] == 0 && t[2] == 0);
  }
}

static void tune_table() {
  tune_clear();
  CHECK(tune_export().empty());
  const std::string good =
      "gfx950|np6|fp32|valu|R64|E2^17 1 2 1 0 0.18\n"
      "gfx950|np3|fp32|packed|R16|E2^20 4 1 0 8 0.5\n";
  CHECK(tune_import(good) == 2);
  TuneParams p;
  CHECK(tune_find("gfx950|np6|fp32|valu|R64|E2^17", &p) && p.epw == 1 && p.waves == 2 && p.remap == 1);
  CHECK(tune_find("gfx950|np3|fp32|packed|R16|E2^20", &p) && p.grid_per_cu == 8);
  const std::string text = tune_export();
  tune_clear();
  CHECK(tune_import(text) == 2);
  CHECK(tune_export() == text);
  // malformed lines are refused whole (EINVAL), leaving the table as it was
  const char* bad[] = {"key 3 2 1 0 0.1\n", "key 1 2\n", "key 1 8 1 0 0.1\n", "key 1 2 1 999 0.1\n",
                       "key x y z w v\n", "\n\n \t", "ok 1 2 1 0 0.1\nkey 1 2 1 -1 0.1\n"};
  for (const char* b : bad) {
    bool refused = false;
    try {
      (void)tune_import(b);
    } catch (const Error& e) {
      refused = e.code == DGD_EINVAL;
    }
    CHECK(refused);
    CHECK(tune_export() == text);
  }
  tune_clear();
}

int main() {
  meshes();
  reference_elements();
  bf16_split();
  tune_table();
  if (g_fail) return 1;
  std::printf("host checks passed\n");
  return 0;
}
