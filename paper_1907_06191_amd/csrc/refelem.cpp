// Reference element of the nodal DG space and the SIPG element matrices.
//
// Basis (section 3.1, eq. (8)): Lagrange polynomials of degree p on the
// equispaced nodes (i/p, j/p), i + j <= p, of the unit triangle
// {r, s >= 0, r + s <= 1}, built by inverting the monomial Vandermonde matrix.
// Both element shapes of the pixel mesh are affine images of the unit
// triangle with unit Jacobian determinant (cell-local coordinates in units of
// h, origin at the cell's lower-left corner):
//   T0: (x, y) = (r + s, s)        T1: (x, y) = (r, r + s).
//
// Element matrices in dimensionless form (h = 1, D = 1): with the physical
// operator -M^-1 A = (D / h^2) * (dimensionless), every element of one
// orientation and face mask shares one matrix.  For element K with outward
// unit normal n on face f and neighbour K' (the SIPG form of section 3.1 /
// 3.2 read as the primal interior-penalty method):
//   K     = int_K grad phi_i . grad phi_j
//   Fs_f  = int_f -1/2 (grad phi_j . n) phi_i - 1/2 (grad phi_i . n) phi_j
//                  + eta p^2 phi_i phi_j
//   Fn_f  = int_f -1/2 (grad phi'_j . n) phi_i + 1/2 (grad phi_i . n) phi'_j
//                  - eta p^2 phi_i phi'_j
//   S_{o,mask} = -M^-1 (K + sum_{f in mask} Fs_f),  N_{o,f} = -M^-1 Fn_f.
// Integrals use Gauss-Legendre rules (collapsed product rule on the
// triangle), exact for the polynomial degrees involved.
#include <cmath>
#include <cstring>
#include <stdexcept>

#include "dgd_internal.h"

namespace dgd {
namespace {

// Gauss-Legendre nodes and weights on [0, 1] (Newton on P_n).
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    // recompute derivative at the converged node
    double p0 = 1, p1 = z;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1);
    x[i] = 0.5 * (1 - z);
    w[i] = 1.0 / ((1 - z * z) * dp * dp);  // = 2/((1-z^2) P'^2) scaled by 1/2
  }
}

// In-place inverse of an n x n row-major matrix (Gauss-Jordan, partial pivoting).
std::vector<double> inverse(std::vector<double> a, int n) {
  std::vector<double> inv(n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[i * n + i] = 1;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[r * n + c]) > std::fabs(a[piv * n + c])) piv = r;
    if (std::fabs(a[piv * n + c]) < 1e-300) throw std::runtime_error("singular matrix");
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(a[c * n + k], a[piv * n + k]);
        std::swap(inv[c * n + k], inv[piv * n + k]);
      }
    const double d = 1.0 / a[c * n + c];
    for (int k = 0; k < n; ++k) {
      a[c * n + k] *= d;
      inv[c * n + k] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = a[r * n + c];
      if (f == 0) continue;
      for (int k = 0; k < n; ++k) {
        a[r * n + k] -= f * a[c * n + k];
        inv[r * n + k] -= f * inv[c * n + k];
      }
    }
  }
  return inv;
}

struct Basis {
  int p, np;
  std::vector<int> ea, eb;      // monomial exponents
  std::vector<double> C;        // [m][k] coefficients of phi_k
  // values and gradients (in r, s) at (r, s)
  void eval_rs(double r, double s, double* v, double* gr, double* gs) const {
    for (int k = 0; k < np; ++k) v[k] = gr[k] = gs[k] = 0;
    for (int m = 0; m < np; ++m) {
      const int a = ea[m], b = eb[m];
      const double mv = std::pow(r, a) * std::pow(s, b);
      const double mr = a ? a * std::pow(r, a - 1) * std::pow(s, b) : 0.0;
      const double ms = b ? b * std::pow(r, a) * std::pow(s, b - 1) : 0.0;
      for (int k = 0; k < np; ++k) {
        const double c = C[m * np + k];
        v[k] += c * mv;
        gr[k] += c * mr;
        gs[k] += c * ms;
      }
    }
  }
  // values and physical gradients at a cell-local point for orientation o
  void eval_xy(int o, double x, double y, double* v, double* gx, double* gy) const {
    std::vector<double> gr(np), gs(np);
    double r, s;
    if (o == 0) { r = x - y; s = y; } else { r = x; s = y - x; }
    eval_rs(r, s, v, gr.data(), gs.data());
    for (int k = 0; k < np; ++k) {
      if (o == 0) { gx[k] = gr[k]; gy[k] = -gr[k] + gs[k]; }
      else { gx[k] = gr[k] - gs[k]; gy[k] = gs[k]; }
    }
  }
};

Basis make_basis(int p) {
  Basis B;
  B.p = p;
  B.np = (p + 1) * (p + 2) / 2;
  for (int d = 0; d <= p; ++d)
    for (int b = 0; b <= d; ++b) {
      B.ea.push_back(d - b);
      B.eb.push_back(b);
    }
  std::vector<double> V(B.np * B.np);
  int i = 0;
  for (int j = 0; j <= p; ++j)
    for (int ii = 0; ii <= p - j; ++ii, ++i) {
      const double r = (double)ii / p, s = (double)j / p;
      for (int m = 0; m < B.np; ++m) V[i * B.np + m] = std::pow(r, B.ea[m]) * std::pow(s, B.eb[m]);
    }
  B.C = inverse(V, B.np);  // C[m][k]: phi_k = sum_m C[m][k] mono_m
  return B;
}

}  // namespace

// Collapsed Gauss-Legendre rule (n x n points) on each triangle for the
// projection of the initial pulse: per orientation and point,
// (x, y, w, phi_0 .. phi_{np-1}) in cell-local coordinates, w including the
// collapse Jacobian (unit triangle area element; both shapes have det 1).
std::vector<double> build_ic_quadrature(const RefElem& R, int n) {
  const Basis B = make_basis(R.p);
  const int np = R.np;
  std::vector<double> x, w;
  gauss_legendre01(n, x, w);
  const int nq = n * n;
  std::vector<double> out((size_t)2 * nq * (3 + np));
  std::vector<double> v(np), gr(np), gs(np);
  for (int o = 0; o < 2; ++o)
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        const int q = a * n + b;
        const double r = x[a] * (1 - x[b]), s = x[b];
        double* dst = &out[((size_t)o * nq + q) * (3 + np)];
        dst[0] = (o == 0) ? r + s : r;
        dst[1] = (o == 0) ? s : r + s;
        dst[2] = w[a] * w[b] * (1 - x[b]);
        B.eval_rs(r, s, v.data(), gr.data(), gs.data());
        for (int k = 0; k < np; ++k) dst[3 + k] = v[k];
      }
  return out;
}

RefElem build_ref_elem(int p, double eta) {
  RefElem R;
  R.p = p;
  R.eta = eta;
  const Basis B = make_basis(p);
  const int np = B.np;
  R.np = np;
  // node positions per orientation
  R.nodes.resize(2 * np * 2);
  {
    int i = 0;
    for (int j = 0; j <= p; ++j)
      for (int ii = 0; ii <= p - j; ++ii, ++i) {
        const double r = (double)ii / p, s = (double)j / p;
        R.nodes[(0 * np + i) * 2 + 0] = r + s;
        R.nodes[(0 * np + i) * 2 + 1] = s;
        R.nodes[(1 * np + i) * 2 + 0] = r;
        R.nodes[(1 * np + i) * 2 + 1] = r + s;
      }
  }
  // volume quadrature: collapsed Gauss-Legendre, exact to degree 2n-2
  const int nv = p + 3;
  std::vector<double> gx1, gw1;
  gauss_legendre01(nv, gx1, gw1);
  std::vector<double> qr, qs, qw;
  for (int a = 0; a < nv; ++a)
    for (int b = 0; b < nv; ++b) {
      qr.push_back(gx1[a] * (1 - gx1[b]));
      qs.push_back(gx1[b]);
      qw.push_back(gw1[a] * gw1[b] * (1 - gx1[b]));
    }
  // face quadrature
  const int nf = p + 2;
  std::vector<double> fx, fw;
  gauss_legendre01(nf, fx, fw);
  static const double P0[2][3][2] = {{{0, 0}, {1, 0}, {1, 1}}, {{1, 1}, {0, 1}, {0, 0}}};
  static const double P1[2][3][2] = {{{1, 0}, {1, 1}, {0, 0}}, {{0, 1}, {0, 0}, {1, 1}}};
  const double is2 = 1.0 / std::sqrt(2.0);
  static double NRM[2][3][2];
  NRM[0][0][0] = 0; NRM[0][0][1] = -1;
  NRM[0][1][0] = 1; NRM[0][1][1] = 0;
  NRM[0][2][0] = -is2; NRM[0][2][1] = is2;
  NRM[1][0][0] = 0; NRM[1][0][1] = 1;
  NRM[1][1][0] = -1; NRM[1][1][1] = 0;
  NRM[1][2][0] = is2; NRM[1][2][1] = -is2;
  static const int OFF[2][3][2] = {{{0, -1}, {1, 0}, {0, 0}}, {{0, 1}, {-1, 0}, {0, 0}}};
  const double pen = eta * p * p;

  R.S.assign(2 * 8 * np * np, 0);
  R.Nb.assign(2 * 3 * np * np, 0);
  R.Fs.assign(2 * 3 * np * np, 0);
  R.Bd.assign(2 * 3 * np * np, 0);
  R.Mass.assign(2 * np * np, 0);
  R.Minv.assign(2 * np * np, 0);
  R.W.assign(2 * 6 * np, 0);
  R.MG.assign(2 * 8 * 2 * np * np, 0);
  R.MD.assign(2 * 8 * 2 * np * np, 0);
  R.MN.assign(2 * 3 * 2 * np * np, 0);
  R.MNc.assign(2 * 3 * 2 * np * (p + 1), 0);
  R.MNcol.assign(2 * 3 * (p + 1), 0);
  std::vector<double> v(np), vx(np), vy(np), w2(np), wx(np), wy(np);
  for (int o = 0; o < 2; ++o) {
    std::vector<double> M(np * np, 0), K(np * np, 0), GX(np * np, 0), GY(np * np, 0);
    for (size_t q = 0; q < qw.size(); ++q) {
      double x, y;
      if (o == 0) { x = qr[q] + qs[q]; y = qs[q]; } else { x = qr[q]; y = qr[q] + qs[q]; }
      B.eval_xy(o, x, y, v.data(), vx.data(), vy.data());
      const double xi = x - 0.5, et = y - 0.5;
      const double pw[6] = {1, xi, et, xi * xi, xi * et, et * et};
      for (int i = 0; i < np; ++i) {
        for (int j = 0; j < np; ++j) {
          M[i * np + j] += qw[q] * v[i] * v[j];
          K[i * np + j] += qw[q] * (vx[i] * vx[j] + vy[i] * vy[j]);
          GX[i * np + j] += qw[q] * vx[j] * v[i];
          GY[i * np + j] += qw[q] * vy[j] * v[i];
        }
        for (int a = 0; a < 6; ++a) R.W[(o * 6 + a) * np + i] += qw[q] * pw[a] * v[i];
      }
    }
    const std::vector<double> Mi = inverse(M, np);
    std::vector<double> Fs[3], Fn[3], Fd[3], Ps[3], Pn[3];
    for (int f = 0; f < 3; ++f) {
      Fs[f].assign(np * np, 0);
      Fn[f].assign(np * np, 0);
      Fd[f].assign(np * np, 0);
      Ps[f].assign(np * np, 0);
      Pn[f].assign(np * np, 0);
      const double ex = P1[o][f][0] - P0[o][f][0], ey = P1[o][f][1] - P0[o][f][1];
      const double len = std::sqrt(ex * ex + ey * ey);
      const double nx = NRM[o][f][0], ny = NRM[o][f][1];
      for (int q = 0; q < nf; ++q) {
        const double x = P0[o][f][0] + fx[q] * ex, y = P0[o][f][1] + fx[q] * ey;
        const double wq = fw[q] * len;
        B.eval_xy(o, x, y, v.data(), vx.data(), vy.data());
        B.eval_xy(1 - o, x - OFF[o][f][0], y - OFF[o][f][1], w2.data(), wx.data(), wy.data());
        for (int i = 0; i < np; ++i)
          for (int j = 0; j < np; ++j) {
            const double dni = vx[i] * nx + vy[i] * ny;
            const double dnj = vx[j] * nx + vy[j] * ny;
            const double dnj_n = wx[j] * nx + wy[j] * ny;
            Fs[f][i * np + j] += wq * (-0.5 * dnj * v[i] - 0.5 * dni * v[j] + pen * v[i] * v[j]);
            Fn[f][i * np + j] += wq * (-0.5 * dnj_n * v[i] + 0.5 * dni * w2[j] - pen * v[i] * w2[j]);
            // face on the absorbing box: the same terms with zero outside value
            Fd[f][i * np + j] += wq * (-dnj * v[i] - dni * v[j] + pen * v[i] * v[j]);
            Ps[f][i * np + j] += wq * v[i] * v[j];
            Pn[f][i * np + j] += wq * v[i] * w2[j];
          }
      }
    }
    // the neighbour's nodes on each shared face (its cell-local positions
    // shifted into this cell lie on the segment P0 -> P1)
    for (int f = 0; f < 3; ++f) {
      const double ex = P1[o][f][0] - P0[o][f][0], ey = P1[o][f][1] - P0[o][f][1];
      int k = 0;
      for (int j = 0; j < np; ++j) {
        const double x = R.nodes[((1 - o) * np + j) * 2] + OFF[o][f][0] - P0[o][f][0];
        const double y = R.nodes[((1 - o) * np + j) * 2 + 1] + OFF[o][f][1] - P0[o][f][1];
        const double cross = ex * y - ey * x;
        const double t = (ex * x + ey * y) / (ex * ex + ey * ey);
        if (std::fabs(cross) < 1e-12 && t > -1e-12 && t < 1 + 1e-12) {
          if (k > p) throw std::runtime_error("face node count");
          R.MNcol[((size_t)o * 3 + f) * (p + 1) + k++] = j;
        }
      }
      if (k != p + 1) throw std::runtime_error("face node count");
    }
    // mixed form
    auto mi_times = [&](const std::vector<double>& A, double* dst) {
      for (int i = 0; i < np; ++i)
        for (int j = 0; j < np; ++j) {
          double acc = 0;
          for (int k = 0; k < np; ++k) acc += Mi[i * np + k] * A[k * np + j];
          dst[i * np + j] = acc;
        }
    };
    for (int c = 0; c < 2; ++c) {
      const std::vector<double>& Gc = c == 0 ? GX : GY;
      for (int mask = 0; mask < 8; ++mask) {
        std::vector<double> Tg(np * np), Td(np * np);
        for (int i = 0; i < np; ++i)
          for (int j = 0; j < np; ++j) {
            Tg[i * np + j] = Gc[i * np + j];
            Td[i * np + j] = -Gc[j * np + i];
          }
        for (int f = 0; f < 3; ++f)
          if (mask >> f & 1)
            for (int k = 0; k < np * np; ++k) {
              Tg[k] -= 0.5 * NRM[o][f][c] * Ps[f][k];
              Td[k] += 0.5 * NRM[o][f][c] * Ps[f][k];
            }
        mi_times(Tg, &R.MG[(((size_t)o * 8 + mask) * 2 + c) * np * np]);
        mi_times(Td, &R.MD[(((size_t)o * 8 + mask) * 2 + c) * np * np]);
      }
      for (int f = 0; f < 3; ++f) {
        std::vector<double> Tn(np * np);
        for (int k = 0; k < np * np; ++k) Tn[k] = 0.5 * NRM[o][f][c] * Pn[f][k];
        mi_times(Tn, &R.MN[(((size_t)o * 3 + f) * 2 + c) * np * np]);
      }
    }
    for (int f = 0; f < 3; ++f)
      for (int c = 0; c < 2; ++c)
        for (int i = 0; i < np; ++i)
          for (int k = 0; k <= p; ++k)
            R.MNc[((((size_t)o * 3 + f) * 2 + c) * np + i) * (p + 1) + k] =
                R.MN[((((size_t)o * 3 + f) * 2 + c) * np + i) * np + R.MNcol[((size_t)o * 3 + f) * (p + 1) + k]];
    // the columns left out vanish up to the rounding of the quadrature
    double big = 0, off = 0;
    for (int f = 0; f < 3; ++f)
      for (int c = 0; c < 2; ++c)
        for (int i = 0; i < np; ++i)
          for (int j = 0; j < np; ++j) {
            const double v = std::fabs(R.MN[((((size_t)o * 3 + f) * 2 + c) * np + i) * np + j]);
            bool kept = false;
            for (int k = 0; k <= p; ++k) kept |= R.MNcol[((size_t)o * 3 + f) * (p + 1) + k] == j;
            big = std::max(big, v);
            if (!kept) off = std::max(off, v);
          }
    if (off > 1e-12 * big) throw std::runtime_error("neighbour block has weight off the face nodes");
    for (int mask = 0; mask < 8; ++mask) {
      std::vector<double> T = K;
      for (int f = 0; f < 3; ++f)
        if (mask >> f & 1)
          for (int k = 0; k < np * np; ++k) T[k] += Fs[f][k];
      for (int i = 0; i < np; ++i)
        for (int j = 0; j < np; ++j) {
          double acc = 0;
          for (int k = 0; k < np; ++k) acc += Mi[i * np + k] * T[k * np + j];
          R.S[((o * 8 + mask) * np + i) * np + j] = -acc;
        }
    }
    for (int f = 0; f < 3; ++f)
      for (int i = 0; i < np; ++i)
        for (int j = 0; j < np; ++j) {
          double acc = 0, accs = 0, accd = 0;
          for (int k = 0; k < np; ++k) {
            acc += Mi[i * np + k] * Fn[f][k * np + j];
            accs += Mi[i * np + k] * Fs[f][k * np + j];
            accd += Mi[i * np + k] * Fd[f][k * np + j];
          }
          R.Nb[((o * 3 + f) * np + i) * np + j] = -acc;
          R.Fs[((o * 3 + f) * np + i) * np + j] = -accs;
          R.Bd[((o * 3 + f) * np + i) * np + j] = -accd;
        }
    for (int k = 0; k < np * np; ++k) {
      R.Mass[o * np * np + k] = M[k];
      R.Minv[o * np * np + k] = Mi[k];
    }
  }
  return R;
}

double bf16_value(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

void split_bf16x3(double a, uint16_t t[3]) {
  double rest = a;
  for (int k = 0; k < 3; ++k) {
    const float f = (float)rest;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    t[k] = (uint16_t)(u >> 16);
    rest -= bf16_value(t[k]);
  }
}

void eval_nodal_basis(const RefElem& R, int o, double x, double y, double* out) {
  const Basis B = make_basis(R.p);
  std::vector<double> gx(R.np), gy(R.np);
  B.eval_xy(o, x, y, out, gx.data(), gy.data());
}

}  // namespace dgd
