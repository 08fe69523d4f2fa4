// Host mesh builder: pixel grid -> active triangles -> interior faces.
//
// Section 3.3 of the paper: the square is cut into pixels and each pixel
// into two triangles along a diagonal.  Here the diagonal joins the cell's
// lower-left and upper-right corners; T0 is the lower-right triangle
// {(i,j), (i+1,j), (i+1,j+1)} h and T1 the upper-left one
// {(i,j), (i+1,j+1), (i,j+1)} h.  A cell whose centroid ((i+1/2)h, (j+1/2)h)
// lies strictly inside a disk is an axon cell and is removed with both
// triangles (the reflecting walls of eq. (3) become faces without flux).
//
// Faces per orientation (the neighbour is always the other orientation):
//   T0: 0 bottom -> T1(i, j-1), 1 right -> T1(i+1, j), 2 diagonal -> T1(i, j)
//   T1: 0 top    -> T0(i, j+1), 1 left  -> T0(i-1, j), 2 diagonal -> T0(i, j)
#include <algorithm>
#include <cmath>
#include <queue>

#include "dgd_internal.h"

namespace dgd {

void build_mesh_host(double L, int N, const double* disks, int n_disks, int strip, int group,
                     MeshHost& m) {
  m.L = L;
  m.N = N;
  m.h = L / N;
  const double h = m.h;
  m.active_cell.assign((size_t)N * N, 1);
  for (int d = 0; d < n_disks; ++d) {
    const double cx = disks[3 * d], cy = disks[3 * d + 1], r = disks[3 * d + 2];
    if (!(r > 0)) continue;
    // only cells whose centroid can be inside: |c - center| < r
    int i0 = std::max(0, (int)std::floor((cx - r) / h) - 1);
    int i1 = std::min(N - 1, (int)std::ceil((cx + r) / h) + 1);
    int j0 = std::max(0, (int)std::floor((cy - r) / h) - 1);
    int j1 = std::min(N - 1, (int)std::ceil((cy + r) / h) + 1);
    for (int j = j0; j <= j1; ++j)
      for (int i = i0; i <= i1; ++i) {
        const double dx = (i + 0.5) * h - cx, dy = (j + 0.5) * h - cy;
        if (dx * dx + dy * dy < r * r) m.active_cell[(size_t)j * N + i] = 0;
      }
  }
  // rank active cells: vertical strips of `strip` columns, each strip
  // row-major (j slow, i fast); strip <= 0 or >= N gives plain row-major.
  // With the stage kernel's XCD-banded block order, each XCD then sweeps a
  // few strips top to bottom and the rows above and below the one in flight
  // (the vertical face neighbours) stay in its L2.
  const int W = (strip <= 0 || strip >= N) ? N : strip;
  std::vector<int64_t> rank((size_t)N * N, -1);
  int64_t nc = 0;
  for (int s0 = 0; s0 < N; s0 += W)
    for (int j = 0; j < N; ++j)
      for (int i = s0; i < std::min(N, s0 + W); ++i)
        if (m.active_cell[(size_t)j * N + i]) rank[(size_t)j * N + i] = nc++;
  const int64_t E = 2 * nc;
  // element of ranked cell r and orientation o: runs of `group` cells give
  // their T0 first, then their T1 (group 1: T0, T1 per cell), so aligned
  // runs of up to `group` elements share one orientation
  const int64_t Gc = group < 1 ? 1 : group;
  auto elem_of = [&](int64_t r, int o) -> int64_t {
    const int64_t start = r / Gc * Gc;
    const int64_t gsz = std::min<int64_t>(Gc, nc - start);
    return 2 * start + o * gsz + (r - start);
  };
  m.ci.resize(E);
  m.cj.resize(E);
  m.orient.resize(E);
  m.nbr.assign(E * 3, -1);
  auto cell_rank = [&](int i, int j) -> int64_t {
    if (i < 0 || j < 0 || i >= N || j >= N) return -1;
    return rank[(size_t)j * N + i];
  };
  static const int off[2][3][2] = {{{0, -1}, {1, 0}, {0, 0}}, {{0, 1}, {-1, 0}, {0, 0}}};
  int64_t nf = 0;
  for (int j = 0; j < N; ++j)
    for (int i = 0; i < N; ++i) {
      const int64_t r = rank[(size_t)j * N + i];
      if (r < 0) continue;
      for (int o = 0; o < 2; ++o) {
        const int64_t e = elem_of(r, o);
        m.ci[e] = i;
        m.cj[e] = j;
        m.orient[e] = (int8_t)o;
        for (int f = 0; f < 3; ++f) {
          const int64_t rn = cell_rank(i + off[o][f][0], j + off[o][f][1]);
          if (rn >= 0) {
            m.nbr[e * 3 + f] = (int32_t)elem_of(rn, 1 - o);
            ++nf;
          }
        }
      }
    }
  m.n_faces = nf / 2;
  // faces on the square's edges: -2 (no flux unless an operator absorbs
  // there, eq. (4)); T0 bottom / right, T1 top / left
  for (int64_t e = 0; e < E; ++e) {
    const int i = m.ci[e], j = m.cj[e];
    if (m.orient[e] == 0) {
      if (j == 0) m.nbr[e * 3 + 0] = -2;
      if (i == N - 1) m.nbr[e * 3 + 1] = -2;
    } else {
      if (j == N - 1) m.nbr[e * 3 + 0] = -2;
      if (i == 0) m.nbr[e * 3 + 1] = -2;
    }
  }
  // connected components by breadth-first search over interior faces
  std::vector<int32_t> comp(E, -1);
  int32_t ncomp = 0;
  std::vector<int64_t> queue;
  queue.reserve(1024);
  for (int64_t s = 0; s < E; ++s) {
    if (comp[s] >= 0) continue;
    comp[s] = ncomp;
    queue.clear();
    queue.push_back(s);
    for (size_t q = 0; q < queue.size(); ++q) {
      const int64_t e = queue[q];
      for (int f = 0; f < 3; ++f) {
        const int32_t n = m.nbr[e * 3 + f];
        if (n >= 0 && comp[n] < 0) {
          comp[n] = ncomp;
          queue.push_back(n);
        }
      }
    }
    ++ncomp;
  }
  m.n_components = ncomp;
}

}  // namespace dgd
