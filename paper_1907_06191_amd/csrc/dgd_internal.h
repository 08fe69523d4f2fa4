// Internal types of libdgd (host side).  Not part of the C-ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/dgd.h"
#include "launch.h"

namespace dgd {

// Error plumbing: the last message per host thread, exceptions internal only.
struct Error {
  int code;
  std::string msg;
};
void set_error(int code, const std::string& msg);
void clear_error();

#define DGD_HIP_CHECK(expr)                                                       \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess)                                                         \
      throw ::dgd::Error{DGD_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
  } while (0)

// Element metadata packed for one 16-byte load per element:
//   x, y, z = neighbour element across faces 0, 1, 2 (-1: wall, -2: box edge),
//   w = orientation | face mask << 1 | cell_i << 4 | cell_j << 18.
struct MeshHost {
  double L = 0, h = 0;
  int N = 0;
  std::vector<uint8_t> active_cell;  // [j * N + i]
  std::vector<int32_t> ci, cj;       // per element
  std::vector<int8_t> orient;
  std::vector<int32_t> nbr;          // [E][3]
  int64_t n_faces = 0;
  int32_t n_components = 0;
  int64_t n_elements() const { return (int64_t)orient.size(); }
};

// Reference element data, FP64, dimensionless (h = 1, D = 1).
struct RefElem {
  int p = 0, np = 0;
  double eta = 0;
  std::vector<double> nodes;        // [2][np][2] cell-local positions (units of h)
  std::vector<double> S;            // [2][8][np][np]  -M^-1 (K + sum_{f in mask} Fself_f)
  std::vector<double> Nb;           // [2][3][np][np]  -M^-1 Fnbr_f
  std::vector<double> Fs;           // [2][3][np][np]  -M^-1 Fself_f: S_{o,7} - S_{o,mask} =
                                    //   sum over faces f not in mask of Fs_{o,f}
  std::vector<double> Bd;           // [2][3][np][np]  -M^-1 Fdir_f: face f on the absorbing box
                                    //   (u = 0 outside, Nitsche terms)
  // the paper's mixed form (q = grad u with the central u-flux lifting,
  // u_t = div(k q) with the harmonic-mean q-flux), dimensionless:
  //   MG[o][mask][c] = M^-1 (G_c - sum_{f in mask} 1/2 n_{f,c} Ps_f)   q from own nodes
  //   MD[o][mask][c] = M^-1 (-G_c^T + sum_{f in mask} 1/2 n_{f,c} Ps_f) u_t from own q
  //   MN[o][f][c]    = M^-1 1/2 n_{f,c} Pn_f      neighbour nodes (both passes)
  // G_c[i][j] = int (d phi_j / d x_c) phi_i, Ps_f / Pn_f the face mass with
  // the own / neighbour basis, n the outward unit normal.
  std::vector<double> MG, MD;       // [2][8][2][np][np]
  std::vector<double> MN;           // [2][3][2][np][np]
  // MN keeps only the neighbour's p + 1 nodes on the shared face (a nodal
  // basis function of a node off the face vanishes on it):
  //   MNc[o][f][c][i][k] = MN[o][f][c][i][MNcol[o][f][k]],  k < p + 1
  std::vector<double> MNc;          // [2][3][2][np][p+1]
  std::vector<int32_t> MNcol;       // [2][3][p+1]
  std::vector<double> Mass;         // [2][np][np]
  std::vector<double> Minv;         // [2][np][np]
  std::vector<double> W;            // [2][6][np] int phi_j xi^a eta^b over the triangle,
                                    //   xi = x - x_c (units of h), powers 1,x,y,xx,xy,yy
};

RefElem build_ref_elem(int p, double eta);
// Nodal basis values at a cell-local point (units of h, origin at the
// cell's lower-left corner) of the orientation-o triangle.
void eval_nodal_basis(const RefElem& R, int o, double x, double y, double* out);
std::vector<double> build_ic_quadrature(const RefElem& R, int n);
// An operator entry as three BF16 terms t[0] + t[1] + t[2] (bit patterns),
// each the remainder of the ones before rounded to nearest even (through
// FP32): together 24 significant bits, |a - sum| below about 2^-26 |a|.
void split_bf16x3(double a, uint16_t t[3]);
double bf16_value(uint16_t b);
// Element order: cells ranked in vertical strips of `strip` columns (each
// strip row by row; strip <= 0: plain rows); the ranked cells are taken in
// runs of `group` cells, each run giving the T0 of its cells, then their T1.
void build_mesh_host(double L, int N, const double* disks, int n_disks, int strip, int group,
                     MeshHost& m);

}  // namespace dgd

// Opaque handles of the C-ABI.
struct dgd_mesh {
  dgd::MeshHost host;
  int device = 0;
  std::vector<int4> packed;  // [E] packed metadata (host copy)
  int4* d_elem = nullptr;    // [E] packed metadata on the device (uploaded on first use)
  // Element tables of the packed stage kernel (order[0]: 2 elements per
  // wave, order[1]: 4): elements grouped by class in windows and padded per
  // class run (see member_table in abi.cpp), built with d_elem.
  struct Order {
    std::vector<int4> table;                     // host copy
    std::vector<std::vector<int64_t>> index;     // [1][E]: table position of mesh element e
    int4* d_elem = nullptr;
  };
  Order order[2];
};

struct dgd_op {
  const dgd_mesh* mesh = nullptr;
  dgd::RefElem ref;
  int precision = DGD_FP64;
  double D = 0;
  double dt_nom = 0, lambda_max = 0;
  const char* dt_rule = "";   // which term set dt_nom: "formula", "stability" or "caller"
  void* d_S = nullptr;    // [2][8][np][np] FP64
  void* d_N = nullptr;    // [2][3][np][np] FP64
  void* d_F = nullptr;    // [2][3][np][np] FP64 self-face blocks (packed stage kernel)
  int outer = DGD_OUTER_REFLECT;
  void* d_B = nullptr;    // [2][3][np][np] FP64 absorbing-box face blocks (DGD_OUTER_ABSORB)
  // mixed form (dgd_operator_build_mixed): k = 0 in axon cells, kept in the mesh
  int form = 0;
  void* d_MG = nullptr;
  void* d_MD = nullptr;
  void* d_MN = nullptr;          // compacted neighbour blocks
  int* d_MNcol = nullptr;        // their columns
  uint8_t* d_meta = nullptr;
  int4* d_elem_ic = nullptr;
  std::vector<uint8_t> axon_cell;   // [j * N + i]
  double* d_Minv = nullptr;  // [2][np][np] FP64
  double* d_W = nullptr;     // [2][6][np] FP64 physical moment weights
  double* d_Mass = nullptr;  // [2][np][np] FP64 physical mass
  double* d_quad = nullptr;  // [2][nq][np+3]: reference quadrature for the initial data
  std::vector<double> quad;  // host copy of d_quad
  int nq = 0;
  // P3 matrix-core path (FP32 state): A operands in lane order, FP64 flux
  // coefficients and mass-row weights (see the MFMA stage kernel)
  float* d_Atab = nullptr;   // [16][10][64]
  // DGD_BF16X3: the same operands split into BF16 hi + mid + lo, and every
  // P3 stage on the split-product kernel
  bool bf16x3 = false;
  uint16_t* d_Atab_bf = nullptr;  // [16][2][3][64][8]
  double* d_Ctab = nullptr;  // [16][40]
  double* d_Wtab = nullptr;  // [2][16]
  double wsum = 0;
};

namespace dgd {

// What a run advances: an element table (one mesh, or several meshes
// concatenated as disconnected components) and the element operator.
struct RunTarget {
  const int4* elem = nullptr;
  int64_t E = 0;
  int np = 0, prec = 0;
  const void* S = nullptr;       // FP64 [2][8][np][np]
  const void* N = nullptr;       // FP64 [2][3][np][np]
  const void* F = nullptr;       // FP64 [2][3][np][np] self-face blocks
  const void* B = nullptr;       // FP64 [2][3][np][np] absorbing-box face blocks (NULL: zero flux)
  double D = 0, h = 0;
  const double* W = nullptr;     // physical moment weights [2][6][np]
  const double* Minv = nullptr;  // reference inverse mass [2][np][np]
  const double* quad = nullptr;  // initial-data quadrature
  const double* quad_host = nullptr;  // its host copy (owned by the op)
  int nq = 0;
  int G = 1;                     // geometries
  const int* blk_geom = nullptr; // device [nblk_red] geometry of each reduction block (G > 1)
  const int* blk_start = nullptr;// device [G + 1] reduction-block range of each geometry (G > 1)
  int64_t nblk_red = 0;          // reduction blocks covering the elements
  const float* Atab = nullptr;   // P3 matrix-core tables (NULL: VALU path only)
  const uint16_t* Atab_bf = nullptr;  // BF16 hi/mid/lo tables; non-NULL: every stage on them
  const double* Ctab = nullptr;
  const double* Wtab = nullptr;
  double wsum = 0;
  const RefElem* ref = nullptr;  // reference element (host)
  // the paper's mixed form on all pixels (form 1; form 0: primal SIPG)
  int form = 0;
  const void* MG = nullptr;      // FP64 [2][8][2][np][np]
  const void* MD = nullptr;      // FP64 [2][8][2][np][np]
  const void* MN = nullptr;      // FP64 [2][3][2][np][p+1] (face-node columns)
  const int* MNcol = nullptr;    // int32 [2][3][p+1]
  const uint8_t* meta = nullptr; // device [E] q-flux face mask | 8 if extracellular
  const int4* elem_ic = nullptr; // element table with axon cells as padding (initial data)
  const uint8_t* axon_host = nullptr;  // host [N * N] 1 = axon cell (form 1)
  void* qbuf = nullptr;          // scratch q of the run, [E][2][np][R]
  // host mesh of each geometry and the row of its first element in the table
  std::vector<std::pair<const MeshHost*, int64_t>> hosts;
  // batched runs: table position of each member's mesh elements, [member][e]
  // (NULL: member g's element e sits at hosts[g].second + e)
  const std::vector<std::vector<int64_t>>* member_index = nullptr;
};

}  // namespace dgd

struct dgd_run {
  dgd::RunTarget t;
  int R = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool own_ws = false;
  void* U = nullptr;   // state u^n
  void* U1 = nullptr;  // stage 1
  void* U2 = nullptr;  // stage 2
  double* d_x0 = nullptr;     // [G][R][2]
  double* d_part = nullptr;   // [nblk_red][R][6] partial sums
  double* d_mom = nullptr;    // [G][R][6]
  int* d_blk_start = nullptr; // [G + 1] (plain runs: {0, nblk_red})
  uint32_t* d_step = nullptr; // steps taken (salt of the stochastic rounding)
  int64_t steps = 0;
  bool eager = false;         // never capture step graphs (allocation-free solve)
  dgd::Shape sh;              // stage launch shape
  int kind = 0;               // stage kernel (VALU, packed, matrix cores)
  std::vector<double> x0;
  double t_ms = 0;
  // captured step graphs keyed by (dt bits, steps)
  std::map<std::pair<uint64_t, int64_t>, hipGraphExec_t> graphs;
};

// Several geometries solved together, grouped by polynomial degree: each
// group is one run over the concatenated element tables of its geometries.
struct dgd_batch {
  int G = 0, R = 0;
  std::vector<dgd_op*> ops;
  struct Group {
    int p = 0;
    std::vector<int> geoms;        // batch indices of the member geometries
    int4* d_elem = nullptr;
    int* d_blk_geom = nullptr;
    int* d_blk_start = nullptr;
    int64_t E = 0;                 // padded elements
    int64_t dof = 0;               // active DoF per right-hand side
    double dt = 0;                 // min of the members' nominal steps
    std::vector<std::vector<int64_t>> member_index;   // [member][mesh element] -> table position
    dgd_run* run = nullptr;
  };
  std::vector<Group> groups;
};
