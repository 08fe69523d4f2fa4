// C-ABI of libdgd: meshes, operators, runs, batches and the whole solve.
//
// The solve follows section 4.1 of the paper: one diffusion problem per
// start point, carried to each diffusion time, and the covariance of the
// normalised solution about its start point.  Everything that touches the
// state runs in the HIP kernels of kernels.hip; the host only builds tables
// (mesh, reference element), schedules steps and reads back six FP64
// moments per start point and diffusion time.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>

#include "dgd_internal.h"
#include "launch.h"
#include "tune.h"

namespace dgd {

thread_local std::string g_last_error;

void set_error(int code, const std::string& msg) {
  (void)code;
  g_last_error = msg;
}
void clear_error() { g_last_error.clear(); }

namespace {

struct Options {
  bool graphs = true;
  int64_t graph_steps = 32;
  int stage_epw = 1;        // elements per wave in the stage kernel
  int stage_waves = 4;      // waves per workgroup in the stage kernel
  bool xcd_remap = true;    // XCD-banded block order
  int64_t stage_grid = 0;   // > 0: persistent stage kernel with this many workgroups
  int mesh_strip = 64;      // element order: vertical strips of this many cell columns (0: rows)
  int mesh_group = 4;       // element order: runs of this many cells give their T0, then their T1
  bool packed = true;       // R <= 32: several elements per wave (packed stage kernel)
  int p3_mfma = 2;          // P3 FP32 stages on matrix cores: 0 never, 1 always, 2 when faster
  bool autotune = true;     // tune the stage launch shape per key on first use
  int sort_classes = 0;     // packed runs on class-sorted element tables: 0 never, 1 always
};
Options g_opt;

constexpr int kEpwReduce = 16;      // reduction kernels: 16 elements per wave, 4 waves
constexpr int kReducePer = 64;      // elements per reduction block
constexpr double kCutoff = 12.0;    // initial pulse evaluated within 12 sigma0 of x0
constexpr int kQuadN = 12;          // 12 x 12 collapsed Gauss-Legendre points per triangle
constexpr int kPadCell = 0x3fff;    // cell index of batch padding elements
constexpr int kMaxCells = 16383;

Shape stage_shape(int64_t E) {
  return element_shape(E, g_opt.stage_epw, g_opt.stage_waves, g_opt.xcd_remap, g_opt.stage_grid);
}
Shape reduce_shape(int64_t E) { return element_shape(E, kEpwReduce, 4, true, 0); }

template <typename F>
int guarded(F&& f) {
  try {
    clear_error();
    return f();
  } catch (const Error& e) {
    set_error(e.code, e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error(DGD_ENOMEM, "host allocation failed");
    return DGD_ENOMEM;
  } catch (const std::exception& e) {
    set_error(DGD_EINVAL, e.what());
    return DGD_EINVAL;
  } catch (...) {
    set_error(DGD_EINVAL, "unknown error");
    return DGD_EINVAL;
  }
}

[[noreturn]] void fail(int code, const std::string& msg) { throw Error{code, msg}; }

size_t state_bytes(int prec) { return prec == DGD_FP64 ? 8 : 4; }

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Real root of x^3/6 - x^2/2 + x - 2 = 0: the edge of the SSP-RK3 stability
// interval on the negative real axis, where R(z) = 1 + z + z^2/2 + z^3/6 = -1.
double rk3_limit() {
  double x = 2.5;
  for (int i = 0; i < 60; ++i) {
    const double f = x * x * x / 6 - x * x / 2 + x - 2;
    const double d = x * x / 2 - x + 1;
    x -= f / d;
  }
  return x;
}

template <typename T>
void* upload(const std::vector<T>& v) {
  void* d = nullptr;
  DGD_HIP_CHECK(hipMalloc(&d, std::max<size_t>(v.size(), 1) * sizeof(T)));
  if (!v.empty()) DGD_HIP_CHECK(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return d;
}

// Element table of a mesh in the order the packed stage kernel (G
// elements per wave, G > 1) runs it, in plain and batched runs alike: the
// elements of each window of kSortWindow consecutive mesh elements are
// grouped by class (orientation and face mask: the low four bits of the
// record) and every class run is padded with inert elements of its class
// to a multiple of G, so that each wave sees one face mask and skips the
// terms of absent faces.  Windows keep face neighbours close in memory.
// Neighbour indices are local to the member; index[e] is the position of
// mesh element e.  G = 1 keeps the mesh order.
constexpr int64_t kSortWindow = 512;

void member_table(const dgd_mesh* m, int G, std::vector<int4>* tab, std::vector<int64_t>* index) {
  const std::vector<int4>& src = m->packed;
  const int64_t E = (int64_t)src.size();
  tab->clear();
  index->assign(E, -1);
  if (G <= 1) {
    tab->assign(src.begin(), src.end());
    for (int64_t e = 0; e < E; ++e) (*index)[e] = e;
    return;
  }
  tab->reserve(E + E / 8);
  std::vector<int64_t> bucket[16];
  for (int64_t w0 = 0; w0 < E; w0 += kSortWindow) {
    const int64_t w1 = std::min(E, w0 + kSortWindow);
    for (auto& v : bucket) v.clear();
    for (int64_t e = w0; e < w1; ++e) bucket[src[e].w & 15].push_back(e);
    for (int cls = 0; cls < 16; ++cls) {
      for (int64_t e : bucket[cls]) {
        (*index)[e] = (int64_t)tab->size();
        tab->push_back(src[e]);
      }
      int4 pad;
      pad.x = pad.y = pad.z = -1;
      pad.w = (int)((uint32_t)cls | ((uint32_t)kPadCell << 4) | ((uint32_t)kPadCell << 18));
      while (bucket[cls].size() % G) {
        tab->push_back(pad);
        bucket[cls].push_back(-1);
      }
    }
  }
  for (int4& c : *tab) {
    if (c.x >= 0) c.x = (int)(*index)[c.x];
    if (c.y >= 0) c.y = (int)(*index)[c.y];
    if (c.z >= 0) c.z = (int)(*index)[c.z];
  }
}

// The element tables go to the device on first use (operator build), so
// that meshes can be built and inspected on a host without a GPU.
void ensure_mesh_on_device(const dgd_mesh* cm) {
  dgd_mesh* m = const_cast<dgd_mesh*>(cm);
  if (m->d_elem) return;
  DGD_HIP_CHECK(hipGetDevice(&m->device));
  for (int k = 0; k < 2; ++k) {
    dgd_mesh::Order& o = m->order[k];
    o.index.assign(1, {});
    member_table(m, k ? 4 : 2, &o.table, &o.index[0]);
    o.d_elem = (int4*)upload(o.table);
  }
  m->d_elem = (int4*)upload(m->packed);
}

RunTarget plain_target(const dgd_op* op) {
  RunTarget t;
  t.elem = op->mesh->d_elem;
  t.E = op->mesh->host.n_elements();
  t.np = op->ref.np;
  t.prec = op->precision;
  t.S = op->d_S;
  t.N = op->d_N;
  t.F = op->d_F;
  t.B = op->d_B;
  t.D = op->D;
  t.h = op->mesh->host.h;
  t.W = op->d_W;
  t.Minv = op->d_Minv;
  t.quad = op->d_quad;
  t.quad_host = op->quad.data();
  t.nq = op->nq;
  t.G = 1;
  t.nblk_red = reduce_shape(t.E).blocks;
  t.Atab = op->d_Atab;
  t.Atab_bf = op->bf16x3 ? op->d_Atab_bf : nullptr;
  t.Ctab = op->d_Ctab;
  t.Wtab = op->d_Wtab;
  t.wsum = op->wsum;
  t.ref = &op->ref;
  t.hosts = {{&op->mesh->host, 0}};
  t.form = op->form;
  t.MG = op->d_MG;
  t.MD = op->d_MD;
  t.MN = op->d_MN;
  t.MNcol = op->d_MNcol;
  t.meta = op->d_meta;
  t.elem_ic = op->d_elem_ic;
  t.axon_host = op->axon_cell.empty() ? nullptr : op->axon_cell.data();
  return t;
}

// Whether the P3 matrix-core kernel can run a stage on (t, R).
bool mfma_possible(const RunTarget& t, int R) {
  return t.Atab && !t.B && t.form == 0 && t.prec == DGD_FP32 && t.np == 10 && R % 16 == 0 &&
         (double)t.E * 10.0 * (double)R < 2147483647.0;
}

// Stage kernels: one element and up to 64 right-hand sides per wave
// (VALU); for R <= 32 several elements per wave (packed); P3 FP32 with R a
// multiple of 16 on matrix cores, FP32 products (mfma) or BF16 hi/lo split
// products (mfma_bf16x3, the DGD_BF16X3 precision).
enum StageKind { kValu = 0, kPacked = 1, kMfma = 2, kMfmaBf16 = 3 };
const char* const kKindName[4] = {"valu", "packed", "mfma", "mfma_bf16x3"};

// The VALU kernel for (t, R): packed when R <= 32.
StageKind valu_kind(const RunTarget& t, int R) {
  return g_opt.packed && t.F && t.form == 0 && R <= 32 ? kPacked : kValu;
}

int packed_group(int R) { return R <= 16 ? 4 : 2; }

// The target a plain run of R right-hand sides steps: the class-sorted
// element table when the packed stage kernel runs it, else the mesh order.
// Host buffers of the state stay in mesh order (dgd_run_get_state).
RunTarget run_target(const dgd_op* op, int R) {
  RunTarget t = plain_target(op);
  if (valu_kind(t, R) != kPacked || !g_opt.sort_classes) return t;
  const dgd_mesh::Order& o = op->mesh->order[packed_group(R) == 4 ? 1 : 0];
  if (!o.d_elem) fail(DGD_EINVAL, "internal: sorted element table missing");
  t.elem = o.d_elem;
  t.E = (int64_t)o.table.size();
  t.nblk_red = reduce_shape(t.E).blocks;
  t.member_index = &o.index;
  return t;
}

// Work units a stage launch shape counts: elements, or element groups of
// the packed kernel.
int64_t stage_units(const RunTarget& t, int R, StageKind k) {
  if (k != kPacked) return t.E;
  const int G = packed_group(R);
  return (t.E + G - 1) / G;
}

std::string kind_key(const RunTarget& t, int R, StageKind k) {
  return tune_key(t.np, t.prec, t.form == 1 ? "mixed" : kKindName[k], R, t.E);
}

// The kernel for (t, R) without timing: the matrix cores when forced
// ("p3_mfma" 1), else the faster of the tuned kinds when both are in the
// table ("p3_mfma" 2, autotuning on), else the VALU kernel.
StageKind stage_kind(const RunTarget& t, int R) {
  if (t.Atab_bf) {
    if (!mfma_possible(t, R))
      fail(DGD_EINVAL, "DGD_BF16X3 runs P3 stages on matrix cores in blocks of 16 right-hand "
                       "sides: the count must be a multiple of 16 (and E * 10 * R < 2^31)");
    return kMfmaBf16;
  }
  const StageKind v = valu_kind(t, R);
  if (!mfma_possible(t, R) || g_opt.p3_mfma == 0) return v;
  if (g_opt.p3_mfma == 1) return kMfma;
  TuneParams pm, pv;
  if (g_opt.autotune && tune_find(kind_key(t, R, kMfma), &pm) && tune_find(kind_key(t, R, v), &pv))
    return pm.ms < pv.ms ? kMfma : v;
  return v;
}

// Launch shape of the stage kernel of `kind` on (t, R): the tuned one for
// its key when autotuning is on and the key has been tuned, else the
// options.
Shape pick_shape(const RunTarget& t, int R, StageKind kind) {
  const int64_t units = stage_units(t, R, kind);
  if (g_opt.autotune) {
    TuneParams p;
    if (tune_find(kind_key(t, R, kind), &p)) return tune_shape(p, units);
  }
  return element_shape(units, g_opt.stage_epw, g_opt.stage_waves, g_opt.xcd_remap, g_opt.stage_grid);
}

void stage(const RunTarget& t, StageKind kind, const Shape& sh, const void* us, const void* ub,
           void* out, int mode, double cb, double cg, int R, hipStream_t st,
           const uint32_t* step = nullptr, int stage_id = 0) {
  if (t.form == 1) {
    if (!t.qbuf) fail(DGD_EINVAL, "internal: mixed-form stage without its q buffer");
    launch_mixed_stage(t.prec == DGD_FP64 ? 0 : 1, t.np, us, ub, out, t.qbuf, t.elem, t.meta, t.E,
                       t.MG, t.MD, t.MN, t.MNcol, mode, cb, cg, R, sh, st, step, stage_id);
    return;
  }
  switch (kind) {
    case kMfma:
    case kMfmaBf16:
      launch_stage_p3_mfma(kind == kMfmaBf16, us, ub, out, t.elem, t.E,
                           kind == kMfmaBf16 ? (const void*)t.Atab_bf : (const void*)t.Atab,
                           t.Ctab, t.Wtab, t.wsum, mode, cb, cg, R, sh, st, step, stage_id);
      break;
    case kPacked:
      launch_stage_packed(t.prec == DGD_FP64 ? 0 : 1, t.np, packed_group(R), us, ub, out, t.elem,
                          t.E, t.S, t.F, t.N, mode, cb, cg, R, sh, st, step, stage_id, t.B);
      break;
    default:
      launch_stage(t.prec == DGD_FP64 ? 0 : 1, t.np, us, ub, out, t.elem, t.E, t.S, t.N, mode, cb,
                   cg, R, sh, st, step, stage_id, t.B);
  }
}

// Tune the launch shape of the stage kernel `kind` on (t, R) with a and b
// as scratch (and base read, NULL: a): the common stage
// out = base + 1/4 (u - base) + g L(u) with a small g, so the values stay
// bounded over the timed launches.
TuneParams tune_kind(const RunTarget& t, int R, StageKind kind, void* a, void* b, const void* base,
                     hipStream_t st) {
  auto one = [&](const Shape& sh, const void* src, const void* bs, void* dst) {
    stage(t, kind, sh, src, bs, dst, 1, 0.25, 1e-3, R, st);
  };
  return tune_stage(kind_key(t, R, kind), stage_units(t, R, kind), t.prec,
                    t.E * t.np * (int64_t)R, a, b, base, one, st);
}

// Tune every kernel kind that may run (t, R) whose key is not yet in the
// table (force: tune them again); returns the kind stage_kind then picks.
StageKind tune_target(const RunTarget& t, int R, void* a, void* b, const void* base,
                      hipStream_t st, bool force) {
  std::vector<StageKind> kinds{valu_kind(t, R)};
  if (mfma_possible(t, R) && g_opt.p3_mfma != 0) kinds.push_back(kMfma);
  if (g_opt.p3_mfma == 1 && mfma_possible(t, R)) kinds = {kMfma};
  if (t.Atab_bf) kinds = {stage_kind(t, R)};
  for (StageKind k : kinds) {
    TuneParams p;
    if (force || !tune_find(kind_key(t, R, k), &p)) tune_kind(t, R, k, a, b, base, st);
  }
  return stage_kind(t, R);
}

// Mixed form on the op's mesh: axon cells are the cells whose centroid lies
// strictly inside a disk (the test that removes cells); per element the
// face mask of the q-flux (both sides extracellular) and the extracellular
// flag; the element table of the initial data with axon elements as
// padding; the pass matrices.
void build_mixed_tables(dgd_op* op, const double* disks, int n_disks) {
  const MeshHost& mh = op->mesh->host;
  MeshHost tmp;
  build_mesh_host(mh.L, mh.N, disks, n_disks, 0, 1, tmp);
  op->axon_cell.resize(tmp.active_cell.size());
  for (size_t k = 0; k < tmp.active_cell.size(); ++k) op->axon_cell[k] = tmp.active_cell[k] ? 0 : 1;
  const int64_t E = mh.n_elements();
  auto axon = [&](int64_t e) { return op->axon_cell[(size_t)mh.cj[e] * mh.N + mh.ci[e]] != 0; };
  std::vector<uint8_t> meta(E);
  std::vector<int4> eic = op->mesh->packed;
  for (int64_t e = 0; e < E; ++e) {
    const bool ext = !axon(e);
    int fm = 0;
    if (ext)
      for (int f = 0; f < 3; ++f) {
        const int32_t nb = mh.nbr[(size_t)e * 3 + f];
        if (nb >= 0 && !axon(nb)) fm |= 1 << f;
      }
    meta[e] = (uint8_t)(fm | (ext ? 8 : 0));
    if (!ext) eic[e].w = (int)((uint32_t)(eic[e].w & 1) | ((uint32_t)kPadCell << 4) | ((uint32_t)kPadCell << 18));
  }
  op->d_meta = (uint8_t*)upload(meta);
  op->d_elem_ic = (int4*)upload(eic);
  op->d_MG = upload(op->ref.MG);
  op->d_MD = upload(op->ref.MD);
  op->d_MN = upload(op->ref.MNc);
  op->d_MNcol = (int*)upload(op->ref.MNcol);
  op->form = 1;
}

// Tables of the P3 matrix-core kernel: for class (o, mask) the stacked
// stencil matrix A = [S | N_0 | N_1 | N_2] (10 x 40, missing faces zero,
// rows 10..15 zero), in FP32 and in the lane order of v_mfma_f32_16x16x4
// (lane l, step s holds A[l % 16][4 s + l / 16], stored [class][s][lane]); C = w^T A in FP64 with
// w the row sums of the reference mass matrix; W = w padded to 16.  With
// DGD_BF16X3 also A = A_hi + A_mid + A_lo in BF16 (each term the rounded
// remainder of the ones before) in the lane order of v_mfma_f32_16x16x32_bf16
// as the kernel uses it: lane l, step h, slot j < 5 holds
// A[l % 16][20 h + 5 (l / 16) + j], slots 5..7 zero, stored
// [class][h][hi, mid, lo][lane][slot].
void build_p3_tables(dgd_op* op) {
  const RefElem& R = op->ref;
  const int np = R.np;  // 10
  std::vector<float> At(16 * 64 * 10, 0.f);
  std::vector<uint16_t> Ab(op->bf16x3 ? 16 * 2 * 3 * 64 * 8 : 0, 0);
  std::vector<double> Ct(16 * 40, 0.0), Wt(2 * 16, 0.0);
  double wsum = 0;
  for (int o = 0; o < 2; ++o) {
    std::vector<double> w(np, 0.0);
    for (int i = 0; i < np; ++i)
      for (int j = 0; j < np; ++j) w[i] += R.Mass[(o * np + i) * np + j];
    for (int i = 0; i < np; ++i) Wt[o * 16 + i] = w[i];
    if (o == 0)
      for (double x : w) wsum += x;
    for (int mask = 0; mask < 8; ++mask) {
      const int cls = o * 8 + mask;
      std::vector<double> A(16 * 40, 0.0);
      for (int m = 0; m < np; ++m)
        for (int k = 0; k < np; ++k) {
          A[m * 40 + k] = R.S[((o * 8 + mask) * np + m) * np + k];
          for (int f = 0; f < 3; ++f)
            if (mask >> f & 1) A[m * 40 + 10 * (f + 1) + k] = R.Nb[((o * 3 + f) * np + m) * np + k];
        }
      for (int k = 0; k < 40; ++k) {
        double c = 0;
        for (int m = 0; m < np; ++m) c += w[m] * A[m * 40 + k];
        Ct[cls * 40 + k] = c;
      }
      // [cls][s][lane]: the ten operand loads of a wave are each one
      // contiguous 256-byte row
      for (int s = 0; s < 10; ++s)
        for (int l = 0; l < 64; ++l) At[(cls * 10 + s) * 64 + l] = (float)A[(l % 16) * 40 + 4 * s + l / 16];
      if (!op->bf16x3) continue;
      for (int h = 0; h < 2; ++h)
        for (int l = 0; l < 64; ++l)
          for (int j = 0; j < 5; ++j) {
            uint16_t t[3];
            split_bf16x3(A[(l % 16) * 40 + 20 * h + 5 * (l / 16) + j], t);
            for (int term = 0; term < 3; ++term)
              Ab[((((size_t)cls * 2 + h) * 3 + term) * 64 + l) * 8 + j] = t[term];
          }
    }
  }
  op->d_Atab = (float*)upload(At);
  if (op->bf16x3) op->d_Atab_bf = (uint16_t*)upload(Ab);
  op->d_Ctab = (double*)upload(Ct);
  op->d_Wtab = (double*)upload(Wt);
  op->wsum = wsum;
}

// Largest eigenvalue of -M^-1 A (dimensionless) by power iteration in FP64
// on the device: 16 random columns, each step scaled by the row-sum bound g
// (so nothing overflows), Rayleigh quotient (x, A x)/(x, M x) at the end.
double power_lambda(dgd_op* op, int iters) {
  const dgd_mesh* mesh = op->mesh;
  const int64_t E = mesh->host.n_elements();
  const int np = op->ref.np;
  const int R = 16;
  const int64_t n = E * np * R;
  double g = 0;
  for (int o = 0; o < 2; ++o)
    for (int mask = 0; mask < 8; ++mask)
      for (int i = 0; i < np; ++i) {
        double s = 0;
        for (int j = 0; j < np; ++j) s += std::fabs(op->ref.S[((o * 8 + mask) * np + i) * np + j]);
        for (int f = 0; f < 3; ++f)
          if (mask >> f & 1)
            for (int j = 0; j < np; ++j) s += std::fabs(op->ref.Nb[((o * 3 + f) * np + i) * np + j]);
        if (op->d_B)
          for (int f = 0; f < 2; ++f)
            for (int j = 0; j < np; ++j) s += std::fabs(op->ref.Bd[((o * 3 + f) * np + i) * np + j]);
        g = std::max(g, s);
      }
  if (op->form == 1) {
    // row-sum bounds of the two passes, multiplied
    const RefElem& Rf = op->ref;
    double gg = 0, gd = 0;
    for (int o = 0; o < 2; ++o)
      for (int mask = 0; mask < 8; ++mask)
        for (int i = 0; i < np; ++i) {
          double sg = 0, sd = 0;
          for (int c = 0; c < 2; ++c) {
            for (int j = 0; j < np; ++j) {
              sg += std::fabs(Rf.MG[((((size_t)o * 8 + mask) * 2 + c) * np + i) * np + j]);
              sd += std::fabs(Rf.MD[((((size_t)o * 8 + mask) * 2 + c) * np + i) * np + j]);
            }
            for (int f = 0; f < 3; ++f)
              for (int j = 0; j < np; ++j) {
                const double v = std::fabs(Rf.MN[((((size_t)o * 3 + f) * 2 + c) * np + i) * np + j]);
                sg += v;
                sd += v;
              }
          }
          gg = std::max(gg, sg);
          gd = std::max(gd, sd);
        }
    g = gg * gd;
  }
  double* Mass = (double*)upload(op->ref.Mass);
  double *x = nullptr, *y = nullptr, *part = nullptr, *red = nullptr, *q = nullptr;
  int* bs = nullptr;
  const Shape sh = stage_shape(E);
  const Shape shr = reduce_shape(E);
  auto cleanup = [&]() {
    (void)hipFree(Mass); (void)hipFree(x); (void)hipFree(y); (void)hipFree(part);
    (void)hipFree(red); (void)hipFree(bs); (void)hipFree(q);
  };
  // y = cg L x in FP64 (the stage kernel's mode 0)
  auto apply = [&](const double* in, double* out, double cg, hipStream_t st) {
    if (op->form == 1)
      launch_mixed_stage(DGD_FP64, np, in, nullptr, out, q, mesh->d_elem, op->d_meta, E, op->d_MG,
                         op->d_MD, op->d_MN, op->d_MNcol, 0, 0.0, cg, R, sh, st);
    else
      launch_stage(DGD_FP64, np, in, nullptr, out, mesh->d_elem, E, op->d_S, op->d_N, 0, 0.0, cg, R,
                   sh, st, nullptr, 0, op->d_B);
  };
  try {
    if (op->form == 1) DGD_HIP_CHECK(hipMalloc(&q, 2 * n * sizeof(double)));
    DGD_HIP_CHECK(hipMalloc(&x, n * sizeof(double)));
    DGD_HIP_CHECK(hipMalloc(&y, n * sizeof(double)));
    DGD_HIP_CHECK(hipMalloc(&part, shr.blocks * R * 6 * sizeof(double)));
    DGD_HIP_CHECK(hipMalloc(&red, R * 6 * sizeof(double)));
    bs = (int*)upload(std::vector<int>{0, (int)shr.blocks});
    hipStream_t st = nullptr;
    launch_fill_random(x, n, 0x1907061900ull, st);
    const int4* elem = mesh->d_elem;
    std::vector<double> nrm(R * 6);
    for (int it = 0; it < iters; ++it) {
      apply(x, y, 1.0 / g, st);
      std::swap(x, y);
      // each step shrinks x by about lambda / g: rescale every 16 steps by
      // the largest column norm so that nothing underflows
      if (it % 16 == 15) {
        launch_dot_mass(np, x, x, elem, E, Mass, R, shr, part, st);
        launch_reduce(part, bs, 1, R, red, st);
        DGD_HIP_CHECK(hipMemcpy(nrm.data(), red, R * 6 * sizeof(double), hipMemcpyDeviceToHost));
        double mx = 0;
        for (int r = 0; r < R; ++r) mx = std::max(mx, nrm[r * 6]);
        if (!(mx > 0) || !std::isfinite(mx)) fail(DGD_EUNSTABLE, "power iteration lost its iterate");
        launch_axpby(y, x, 1.0 / std::sqrt(mx), 0.0, n, st);
        std::swap(x, y);
      }
    }
    DGD_HIP_CHECK(hipGetLastError());
    // y = L x (unscaled); lambda = -(x, M y) / (x, M x)
    apply(x, y, 1.0, st);
    std::vector<double> xmy(R * 6), xmx(R * 6);
    launch_dot_mass(np, x, y, elem, E, Mass, R, shr, part, st);
    launch_reduce(part, bs, 1, R, red, st);
    DGD_HIP_CHECK(hipMemcpy(xmy.data(), red, R * 6 * sizeof(double), hipMemcpyDeviceToHost));
    launch_dot_mass(np, x, x, elem, E, Mass, R, shr, part, st);
    launch_reduce(part, bs, 1, R, red, st);
    DGD_HIP_CHECK(hipMemcpy(xmx.data(), red, R * 6 * sizeof(double), hipMemcpyDeviceToHost));
    double lam = 0;
    for (int r = 0; r < R; ++r)
      if (xmx[r * 6] > 0) lam = std::max(lam, -xmy[r * 6] / xmx[r * 6]);
    cleanup();
    return lam;
  } catch (...) {
    cleanup();
    throw;
  }
}

// Named range around a phase of a solve (roctx: visible in rocprofv3
// traces with --marker-trace, free otherwise).
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

// One JSON line per solve appended to the file named by DGD_RUN_LOG (if
// set): entry point, configuration (of the first geometry for a batch),
// step rule, steps (of the longest group), wall time, update rate, status,
// mass drift and the start-point mean of Sigma per Delta.  moments:
// [n_points][n_deltas][6] (all geometries' start points for a batch), or
// NULL; entries a failed solve did not reach (M0 = 0) are left out.
void log_run(const char* entry, const dgd_op* op, int n_geoms, int64_t elements, int n_points,
             const double* deltas, int n_deltas, int64_t steps, double updates, double seconds,
             int status, const double* moments, const char* kernel) {
  const char* path = std::getenv("DGD_RUN_LOG");
  if (!path || !*path || !op) return;
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  std::FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "{\"entry\": \"%s\", \"p\": %d, \"precision\": \"%s\", \"form\": \"%s\", "
               "\"outer\": \"%s\", \"geometries\": %d, \"elements\": %lld, \"n_points\": %d, "
               "\"deltas_ms\": [",
               entry, op->ref.p,
               op->bf16x3 ? "bf16x3" : (op->precision == DGD_FP64 ? "fp64" : "fp32"),
               op->form == 1 ? "mixed" : "primal", op->outer == DGD_OUTER_ABSORB ? "absorb" : "reflect",
               n_geoms, (long long)elements, n_points);
  for (int k = 0; k < n_deltas; ++k) std::fprintf(f, "%s%.17g", k ? ", " : "", deltas[k]);
  std::fprintf(f, "], \"dt_ms\": %.17g, \"dt_rule\": \"%s\", \"lambda_max_per_ms\": %.17g, "
               "\"steps\": %lld, \"seconds\": %.6f, \"gdof_updates_per_s\": %.6g, "
               "\"kernel\": \"%s\", \"status\": %d",
               op->dt_nom, op->dt_rule, op->lambda_max, (long long)steps, seconds,
               seconds > 0 ? updates / seconds / 1e9 : 0.0, kernel ? kernel : "", status);
  if (moments) {
    double drift = 0;
    std::fprintf(f, ", \"sigma_mean\": [");
    for (int k = 0; k < n_deltas; ++k) {
      double sx = 0, sy = 0, sz = 0;
      int n = 0;
      for (int r = 0; r < n_points; ++r) {
        const double* m = moments + ((size_t)r * n_deltas + k) * 6;
        if (!(m[0] != 0) || !std::isfinite(m[0])) continue;
        drift = std::max(drift, std::fabs(m[0] - 1.0));
        sx += m[3] / m[0];
        sy += m[4] / m[0];
        sz += m[5] / m[0];
        ++n;
      }
      if (n)
        std::fprintf(f, "%s[%.10g, %.10g, %.10g]", k ? ", " : "", sx / n, sy / n, sz / n);
      else
        std::fprintf(f, "%snull", k ? ", " : "");
    }
    std::fprintf(f, "], \"max_mass_drift\": %.6g", drift);
  }
  std::fprintf(f, "}\n");
  std::fclose(f);
}

double seconds_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// ---------------------------------------------------------------- runs ----

void ws_layout(const RunTarget& t, int R, size_t* total, size_t off[9]) {
  const size_t st = align256((size_t)t.E * t.np * R * state_bytes(t.prec));
  size_t o = 0;
  off[0] = o; o += st;                                            // U
  off[1] = o; o += st;                                            // U1
  off[2] = o; o += st;                                            // U2
  off[3] = o; o += align256((size_t)t.G * R * 2 * 8);             // x0
  off[4] = o; o += align256((size_t)t.nblk_red * R * 6 * 8);      // partials
  off[5] = o; o += align256((size_t)t.G * R * 6 * 8);             // moments
  off[6] = o; o += align256((size_t)(t.G + 1) * sizeof(int));     // block ranges
  off[7] = o; o += 256;                                           // step counter
  off[8] = o;                                                     // q (mixed form)
  if (t.form == 1) o += align256((size_t)t.E * 2 * t.np * R * state_bytes(t.prec));
  *total = o;
}

void run_destroy(dgd_run* run) {
  if (!run) return;
  if (run->stream) (void)hipStreamSynchronize(run->stream);
  for (auto& kv : run->graphs) (void)hipGraphExecDestroy(kv.second);
  if (run->own_ws) (void)hipFree(run->ws);
  if (run->own_stream) (void)hipStreamDestroy(run->stream);
  delete run;
}

// Projected point masses (sigma0 = 0) of every (geometry, start point):
// the triangle holding x0 (T0 on or below the cell's diagonal, else T1) and
// its coefficients M_K^-1 phi(x0) = Mhat^-1 phi(x0) / h^2, on the host; the
// device state is cleared and the columns scattered in.
void init_point_mass(dgd_run* run) {
  const RunTarget& t = run->t;
  const int np = t.np, R = run->R;
  const size_t n = (size_t)t.G * R;
  std::vector<int64_t> pe(n, -1);
  std::vector<int> col(n);
  std::vector<double> vals(n * np), phi(np);
  for (int g = 0; g < t.G; ++g) {
    const MeshHost& m = *t.hosts[g].first;
    std::vector<double> fx(R), fy(R);
    std::unordered_map<int64_t, std::vector<int>> want;   // (cell, orientation) -> columns
    for (int r = 0; r < R; ++r) {
      const double x = run->x0[((size_t)g * R + r) * 2] / m.h;
      const double y = run->x0[((size_t)g * R + r) * 2 + 1] / m.h;
      const int i = std::min(m.N - 1, (int)std::floor(x)), j = std::min(m.N - 1, (int)std::floor(y));
      if (t.axon_host && t.axon_host[(size_t)j * m.N + i])
        fail(DGD_ENOTFREE, "start point " + std::to_string((size_t)g * R + r) + " lies in an axon cell");
      fx[r] = x - i;
      fy[r] = y - j;
      want[((int64_t)j * m.N + i) * 2 + (fx[r] >= fy[r] ? 0 : 1)].push_back(r);
    }
    for (int64_t e = 0; e < m.n_elements(); ++e) {
      auto it = want.find(((int64_t)m.cj[e] * m.N + m.ci[e]) * 2 + m.orient[e]);
      if (it == want.end()) continue;
      const int64_t at = t.member_index ? (*t.member_index)[g][e] : t.hosts[g].second + e;
      for (int r : it->second) pe[(size_t)g * R + r] = at;
    }
    for (int r = 0; r < R; ++r) {
      const size_t k = (size_t)g * R + r;
      if (pe[k] < 0) fail(DGD_ENOTFREE, "start point " + std::to_string(k) + " lies in a removed cell");
      const int o = fx[r] >= fy[r] ? 0 : 1;
      eval_nodal_basis(*t.ref, o, fx[r], fy[r], phi.data());
      for (int i = 0; i < np; ++i) {
        double a = 0;
        for (int j = 0; j < np; ++j) a += t.ref->Minv[((size_t)o * np + i) * np + j] * phi[j];
        vals[k * np + i] = a / (m.h * m.h);
      }
      col[k] = r;
    }
  }
  void *dpe = nullptr, *dcol = nullptr, *dval = nullptr;
  auto cleanup = [&]() { (void)hipFree(dpe); (void)hipFree(dcol); (void)hipFree(dval); };
  try {
    dpe = upload(pe);
    dcol = upload(col);
    dval = upload(vals);
    DGD_HIP_CHECK(hipMemsetAsync(run->U, 0, (size_t)t.E * np * R * state_bytes(t.prec), run->stream));
    launch_ic_point(t.prec == DGD_FP64 ? 0 : 1, (const int64_t*)dpe, (const int*)dcol,
                    (const double*)dval, (int)n, np, R, run->U, run->stream);
    DGD_HIP_CHECK(hipGetLastError());
    DGD_HIP_CHECK(hipStreamSynchronize(run->stream));
  } catch (...) {
    cleanup();
    throw;
  }
  cleanup();
}

// Allocate (or adopt) the workspace, copy the start points, and project
// the initial pulse of every (geometry, start point) (sigma0 = 0: the
// point mass).  no_alloc: the caller's workspace and stream (NULL: the null
// stream) are used as given, nothing is tuned and no step graph is captured,
// so the run makes no device allocation; point-mass data (sigma0 = 0) are
// refused (their upload allocates).
dgd_run* run_create(const RunTarget& t, const double* x0, int R, double sigma0, void* d_ws,
                    size_t ws_bytes, void* hip_stream, bool no_alloc = false) {
  Range range("dgd:run_create");
  size_t total, off[9];
  ws_layout(t, R, &total, off);
  if (no_alloc && (!d_ws || sigma0 == 0))
    fail(DGD_EINVAL, "internal: allocation-free run without a workspace or with a point mass");
  auto* run = new dgd_run();
  try {
    run->t = t;
    run->R = R;
    run->eager = no_alloc;
    run->x0.assign(x0, x0 + (size_t)t.G * R * 2);
    if (d_ws) {
      if (ws_bytes < total) fail(DGD_ENOMEM, "workspace smaller than the size the library reports");
      run->ws = d_ws;
      run->ws_bytes = ws_bytes;
    } else {
      DGD_HIP_CHECK(hipMalloc(&run->ws, total));
      run->own_ws = true;
      run->ws_bytes = total;
    }
    if (hip_stream || no_alloc) {
      run->stream = (hipStream_t)hip_stream;
    } else {
      DGD_HIP_CHECK(hipStreamCreateWithFlags(&run->stream, hipStreamNonBlocking));
      run->own_stream = true;
    }
    char* base = (char*)run->ws;
    run->U = base + off[0];
    run->U1 = base + off[1];
    run->U2 = base + off[2];
    run->d_x0 = (double*)(base + off[3]);
    run->d_part = (double*)(base + off[4]);
    run->d_mom = (double*)(base + off[5]);
    run->d_blk_start = (int*)(base + off[6]);
    run->d_step = (uint32_t*)(base + off[7]);
    if (t.form == 1) run->t.qbuf = base + off[8];
    DGD_HIP_CHECK(hipMemsetAsync(run->d_step, 0, sizeof(uint32_t), run->stream));
    if (!t.blk_start) {
      // one geometry: all reduction blocks
      const int bs[2] = {0, (int)t.nblk_red};
      DGD_HIP_CHECK(hipMemcpyAsync(run->d_blk_start, bs, sizeof(bs), hipMemcpyHostToDevice,
                                   run->stream));
    } else {
      DGD_HIP_CHECK(hipMemcpyAsync(run->d_blk_start, t.blk_start, (size_t)(t.G + 1) * sizeof(int),
                                   hipMemcpyDeviceToDevice, run->stream));
    }
    DGD_HIP_CHECK(hipMemcpyAsync(run->d_x0, run->x0.data(), run->x0.size() * sizeof(double),
                                 hipMemcpyHostToDevice, run->stream));
    // the stage launch shape, tuned on first use of its key (the two stage
    // buffers are free until the first step)
    if (g_opt.autotune && !no_alloc)
      tune_target(run->t, R, run->U1, run->U2, run->U, run->stream, false);
    if (t.form == 1) {
      // the mixed-form stage kernels skip axon elements (u = 0 there): the
      // stage buffers start at zero (after the tuner used them as scratch)
      const size_t sb = (size_t)t.E * t.np * R * state_bytes(t.prec);
      DGD_HIP_CHECK(hipMemsetAsync(run->U1, 0, sb, run->stream));
      DGD_HIP_CHECK(hipMemsetAsync(run->U2, 0, sb, run->stream));
    }
    run->kind = (int)stage_kind(t, R);
    run->sh = pick_shape(t, R, (StageKind)run->kind);
    if (sigma0 == 0) {
      init_point_mass(run);
      return run;
    }
    const Shape shr = reduce_shape(t.E);
    // the mixed form keeps the axon cells; the pulse is restricted to the
    // extracellular ones (axon elements enter as padding)
    const int4* eic = t.elem_ic ? t.elem_ic : t.elem;
    launch_ic_mass(t.np, eic, t.E, t.quad, t.nq, run->d_x0, t.blk_geom, sigma0, t.h, kCutoff, R,
                   shr, run->d_part, run->stream);
    launch_reduce(run->d_part, run->d_blk_start, t.G, R, run->d_mom, run->stream);
    launch_ic_project(t.prec == DGD_FP64 ? 0 : 1, t.np, eic, t.E, t.quad, t.nq, t.Minv,
                      run->d_x0, t.blk_geom, run->d_mom, sigma0, t.h, kCutoff, R, shr, run->U,
                      run->stream);
    DGD_HIP_CHECK(hipGetLastError());
    std::vector<double> mass((size_t)t.G * R * 6);
    DGD_HIP_CHECK(hipMemcpyAsync(mass.data(), run->d_mom, mass.size() * sizeof(double),
                                 hipMemcpyDeviceToHost, run->stream));
    DGD_HIP_CHECK(hipStreamSynchronize(run->stream));
    for (int k = 0; k < t.G * R; ++k)
      if (!(mass[(size_t)k * 6] > 0) || !std::isfinite(mass[(size_t)k * 6]))
        fail(DGD_ENOTFREE, "start point " + std::to_string(k) + " has no pulse mass on active cells");
  } catch (...) {
    run_destroy(run);
    throw;
  }
  return run;
}

void run_stage_steps(dgd_run* run, int64_t n, double dt) {
  const RunTarget& t = run->t;
  const double gam = dt * t.D / (t.h * t.h);
  for (int64_t s = 0; s < n; ++s) {
    // Shu-Osher SSP-RK3 as corrections of u^n:
    //   u1 = u + dt L u;  u2 = u + 1/4 (u1 - u) + 1/4 dt L u1;  u' = u + 2/3 (u2 - u) + 2/3 dt L u2
    const StageKind k = (StageKind)run->kind;
    stage(t, k, run->sh, run->U, nullptr, run->U1, 1, 0.0, gam, run->R, run->stream, run->d_step, 0);
    stage(t, k, run->sh, run->U1, run->U, run->U2, 1, 0.25, 0.25 * gam, run->R, run->stream,
          run->d_step, 1);
    stage(t, k, run->sh, run->U2, run->U, run->U, 1, 2.0 / 3.0, 2.0 / 3.0 * gam, run->R,
          run->stream, run->d_step, 2);
    launch_step_bump(run->d_step, run->stream);
  }
}

// Most step graphs a run keeps (a dt's set is at most 14: graph_steps and
// the powers of two up to 4096).
constexpr size_t kMaxRunGraphs = 128;

hipGraphExec_t step_graph(dgd_run* run, int64_t n, double dt) {
  uint64_t bits;
  std::memcpy(&bits, &dt, sizeof(bits));
  auto key = std::make_pair(bits, n);
  auto it = run->graphs.find(key);
  if (it != run->graphs.end()) return it->second;
  hipGraph_t g = nullptr;
  DGD_HIP_CHECK(hipStreamBeginCapture(run->stream, hipStreamCaptureModeThreadLocal));
  run_stage_steps(run, n, dt);
  DGD_HIP_CHECK(hipStreamEndCapture(run->stream, &g));
  hipGraphExec_t ex = nullptr;
  const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) fail(DGD_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  run->graphs[key] = ex;
  // upload now, so that the first replay (which may fall in a caller's timed
  // region) costs what later ones do
  DGD_HIP_CHECK(hipGraphUpload(ex, run->stream));
  return ex;
}

void run_advance(dgd_run* run, int64_t n_steps, double dt) {
  Range range("dgd:advance");
  if (n_steps < 0) fail(DGD_EINVAL, "n_steps must be >= 0");
  if (!(dt > 0) || !std::isfinite(dt)) fail(DGD_EINVAL, "dt must be positive");
  if (n_steps == 0) return;
  int64_t left = n_steps;
  if (g_opt.graphs && !run->eager) {
    // Graphs of graph_steps steps and of every power of two up to it, all
    // captured on the first advance with this dt: any step count then runs as
    // replays (whole graphs, then the remainder's binary digits, each below
    // the largest power of two not above graph_steps), and a later advance
    // with the same dt, of whatever length, captures nothing.
    const int64_t G = g_opt.graph_steps;
    int64_t top = 1;
    while (2 * top <= G) top *= 2;
    // The graphs are a cache: a run advanced with many different steps (one
    // per Delta interval, or a caller's own schedule) drops them all, once
    // its stream has drained, before the set of a new dt would pass
    // kMaxRunGraphs.
    uint64_t bits;
    std::memcpy(&bits, &dt, sizeof(bits));
    if (!run->graphs.count(std::make_pair(bits, G)) && run->graphs.size() + 14 > kMaxRunGraphs) {
      DGD_HIP_CHECK(hipStreamSynchronize(run->stream));
      for (auto& kv : run->graphs) (void)hipGraphExecDestroy(kv.second);
      run->graphs.clear();
    }
    std::vector<std::pair<int64_t, hipGraphExec_t>> ladder;
    ladder.emplace_back(G, step_graph(run, G, dt));
    for (int64_t s = top; s >= 1; s /= 2)
      if (s != G) ladder.emplace_back(s, step_graph(run, s, dt));
    for (const auto& g : ladder)
      for (; left >= g.first; left -= g.first) DGD_HIP_CHECK(hipGraphLaunch(g.second, run->stream));
  }
  run_stage_steps(run, left, dt);
  DGD_HIP_CHECK(hipGetLastError());
  run->t_ms += n_steps * dt;
  run->steps += n_steps;
}

// FP64 moments [G][R][6]; returns DGD_EUNSTABLE (moments filled anyway) on a
// non-finite value or mass drift beyond the precision's tolerance.
int run_moments(dgd_run* run, double* out, std::string* why) {
  Range range("dgd:moments");
  const RunTarget& t = run->t;
  const Shape shr = reduce_shape(t.E);
  launch_moments(t.prec == DGD_FP64 ? 0 : 1, t.np, run->U, t.elem, t.E, t.W, run->d_x0,
                 t.blk_geom, t.h, run->R, shr, run->d_part, run->stream);
  launch_reduce(run->d_part, run->d_blk_start, t.G, run->R, run->d_mom, run->stream);
  DGD_HIP_CHECK(hipGetLastError());
  const size_t n = (size_t)t.G * run->R;
  DGD_HIP_CHECK(hipMemcpyAsync(out, run->d_mom, n * 6 * sizeof(double), hipMemcpyDeviceToHost,
                               run->stream));
  DGD_HIP_CHECK(hipStreamSynchronize(run->stream));
  // With an absorbing box the mass decays; the discrete solution is not
  // positive everywhere (the projected pulse undershoots), so near the box
  // the outflow can briefly turn inward and M0 exceed 1 by a discretisation
  // error (1e-8 at P1 on a point mass): the check then only catches blow-up.
  const bool absorbing = t.B != nullptr;
  const double tol = t.prec == DGD_FP64 ? (absorbing ? 1e-6 : 1e-9) : 1e-5;
  for (size_t k = 0; k < n; ++k) {
    for (int c = 0; c < 6; ++c)
      if (!std::isfinite(out[k * 6 + c])) {
        *why = "non-finite moment for start point " + std::to_string(k);
        return DGD_EUNSTABLE;
      }
    const double m0 = out[k * 6];
    if (absorbing ? (m0 < -tol || m0 > 1.0 + tol) : std::fabs(m0 - 1.0) > tol) {
      *why = "mass drift beyond tolerance for start point " + std::to_string(k);
      return DGD_EUNSTABLE;
    }
  }
  return DGD_OK;
}

constexpr double kSignalMaxQH = 4.0;   // |q| h bound of the element rule (error < 1e-16)

// q-space signal of a plain run's current state: out [R][nq][2] = (re, im)
// of int u exp(i q.(x - x0)) dx.  Element integrals of the nodal basis
// times exp(i q.(x - c_K)) use the 12 x 12 collapsed Gauss-Legendre rule of
// the initial data (exact to rounding for |q| h <= 4).
void run_signal(dgd_run* run, const double* q, int nq, double* out) {
  const RunTarget& t = run->t;
  if (t.G != 1) fail(DGD_EINVAL, "the signal is computed for plain runs");
  const int np = t.np, R = run->R;
  std::vector<double> W((size_t)nq * 2 * np * 2, 0.0);
  for (int k = 0; k < nq; ++k) {
    const double qx = q[2 * k], qy = q[2 * k + 1];
    if (!std::isfinite(qx) || !std::isfinite(qy)) fail(DGD_EINVAL, "non-finite wave vector");
    if (std::hypot(qx, qy) * t.h > kSignalMaxQH) fail(DGD_EINVAL, "|q| h must be <= 4");
    for (int o = 0; o < 2; ++o)
      for (int p = 0; p < t.nq; ++p) {
        const double* Q = t.quad_host + ((size_t)o * t.nq + p) * (3 + np);
        const double ph = t.h * (qx * (Q[0] - 0.5) + qy * (Q[1] - 0.5));
        const double wc = Q[2] * t.h * t.h * std::cos(ph), ws = Q[2] * t.h * t.h * std::sin(ph);
        for (int j = 0; j < np; ++j) {
          W[(((size_t)k * 2 + o) * np + j) * 2] += wc * Q[3 + j];
          W[(((size_t)k * 2 + o) * np + j) * 2 + 1] += ws * Q[3 + j];
        }
      }
  }
  const Shape sh = element_shape(t.E, 64, 4, true, 0);
  double *dW = nullptr, *dq = nullptr, *part = nullptr, *dout = nullptr;
  int* bs = nullptr;
  auto cleanup = [&]() {
    (void)hipFree(dW); (void)hipFree(dq); (void)hipFree(part); (void)hipFree(dout); (void)hipFree(bs);
  };
  try {
    dW = (double*)upload(W);
    dq = (double*)upload(std::vector<double>(q, q + 2 * (size_t)nq));
    bs = (int*)upload(std::vector<int>{0, (int)sh.blocks});
    DGD_HIP_CHECK(hipMalloc(&part, (size_t)sh.blocks * R * nq * 2 * sizeof(double)));
    DGD_HIP_CHECK(hipMalloc(&dout, (size_t)R * nq * 2 * sizeof(double)));
    launch_signal(t.prec == DGD_FP64 ? 0 : 1, np, run->U, t.elem, t.E, dW, dq, nq, run->d_x0, t.h, R,
                  sh, part, run->stream);
    launch_reduce_width(part, bs, 1, R, nq * 2, dout, run->stream);
    DGD_HIP_CHECK(hipGetLastError());
    DGD_HIP_CHECK(hipMemcpyAsync(out, dout, (size_t)R * nq * 2 * sizeof(double),
                                 hipMemcpyDeviceToHost, run->stream));
    DGD_HIP_CHECK(hipStreamSynchronize(run->stream));
  } catch (...) {
    cleanup();
    throw;
  }
  cleanup();
}

void check_points(const MeshHost& mh, const double* points, int n, int offset = 0) {
  for (int r = 0; r < n; ++r) {
    const double x = points[2 * r], y = points[2 * r + 1];
    if (!std::isfinite(x) || !std::isfinite(y) || x < 0 || y < 0 || x >= mh.L || y >= mh.L)
      fail(DGD_ENOTFREE, "start point " + std::to_string(offset + r) + " lies outside the box");
    const int i = std::min(mh.N - 1, (int)(x / mh.h)), j = std::min(mh.N - 1, (int)(y / mh.h));
    if (!mh.active_cell[(size_t)j * mh.N + i])
      fail(DGD_ENOTFREE, "start point " + std::to_string(offset + r) + " lies in a removed cell");
  }
}

// Mixed form: start points must lie in extracellular cells.
void check_axon_cells(const dgd_op* op, const double* points, int n) {
  if (op->axon_cell.empty()) return;
  const MeshHost& mh = op->mesh->host;
  for (int r = 0; r < n; ++r) {
    const int i = std::min(mh.N - 1, (int)(points[2 * r] / mh.h));
    const int j = std::min(mh.N - 1, (int)(points[2 * r + 1] / mh.h));
    if (op->axon_cell[(size_t)j * mh.N + i])
      fail(DGD_ENOTFREE, "start point " + std::to_string(r) + " lies in an axon cell");
  }
}

std::vector<std::pair<int64_t, double>> schedule(const double* deltas, int n, double dt_nom) {
  std::vector<std::pair<int64_t, double>> s;
  double prev = 0;
  for (int k = 0; k < n; ++k) {
    if (!std::isfinite(deltas[k]) || !(deltas[k] > prev))
      fail(DGD_EINVAL, "Delta list must be finite, positive and strictly increasing");
    const double span = deltas[k] - prev;
    int64_t m = (int64_t)std::ceil(span / dt_nom - 1e-9);
    if (m < 1) m = 1;
    s.emplace_back(m, span / (double)m);
    prev = deltas[k];
  }
  return s;
}

// Coefficients c_k = e^-z I_k(z) (times 2 for k >= 1) of
// exp(t L) = sum_k c_k T_k(I + 2 L / b), z = t b / 2, by Miller's backward
// recurrence I_{k-1} = (2k / z) I_k + I_{k+1} normalised with
// I_0 + 2 sum_{k>=1} I_k = e^z; cut where the tail falls below 1e-17
// (the c_k sum to 1).
std::vector<double> cheb_coefficients(double z) {
  if (!(z > 0)) return {1.0};
  int K = (int)std::ceil(12.0 * std::sqrt(z) + 60.0);
  const int start = K + 40;
  std::vector<double> I(start + 2, 0.0);
  I[start + 1] = 0.0;
  I[start] = 1e-300;
  for (int k = start; k >= 1; --k) {
    I[k - 1] = (2.0 * k / z) * I[k] + I[k + 1];
    if (I[k - 1] > 1e250)
      for (int j = k - 1; j <= start; ++j) I[j] *= 1e-250;
  }
  double S = I[0];
  for (int k = 1; k <= start; ++k) S += 2.0 * I[k];
  std::vector<double> c(start + 1);
  for (int k = 0; k <= start; ++k) c[k] = (k == 0 ? 1.0 : 2.0) * I[k] / S;
  double tail = 0;
  int last = start;
  for (int k = start; k >= 0; --k) {
    tail += c[k];
    if (tail > 1e-17) {
      last = k;
      break;
    }
  }
  c.resize(std::max(last + 1, 2));
  return c;
}

// ------------------------------------------------------------- batches ----

void batch_destroy(dgd_batch* b) {
  if (!b) return;
  for (auto& g : b->groups) {
    run_destroy(g.run);
    (void)hipFree(g.d_elem);
    (void)hipFree(g.d_blk_geom);
    (void)hipFree(g.d_blk_start);
  }
  delete b;
}

// Group geometries by p (each group shares one step size).
void batch_plan(dgd_batch* b) {
  for (int g = 0; g < b->G; ++g)
    if (b->ops[g]->form != 0) fail(DGD_EINVAL, "batches take primal (removed-cell) operators only");
  for (int g = 0; g < b->G; ++g) {
    const int p = b->ops[g]->ref.p;
    auto it = std::find_if(b->groups.begin(), b->groups.end(),
                           [&](const dgd_batch::Group& x) { return x.p == p; });
    if (it == b->groups.end()) {
      b->groups.emplace_back();
      b->groups.back().p = p;
      it = b->groups.end() - 1;
    }
    it->geoms.push_back(g);
  }
}

// Target and workspace bytes of a group: its geometries' element tables
// concatenated, each padded to whole reduction blocks.
// Elements per wave the group's stage kernel packs (1: one per wave).
int batch_pack(const RunTarget& t, int R) {
  return valu_kind(t, R) == kPacked && g_opt.sort_classes ? packed_group(R) : 1;
}

size_t batch_group_bytes(const dgd_batch::Group& grp, const dgd_batch* b, RunTarget* t_out) {
  RunTarget t = plain_target(b->ops[grp.geoms[0]]);
  const int Gp = batch_pack(t, b->R);
  int64_t E = 0;
  std::vector<int4> tab;
  std::vector<int64_t> index;
  for (int g : grp.geoms) {
    member_table(b->ops[g]->mesh, Gp, &tab, &index);
    const int64_t Eg = (int64_t)tab.size();
    E += (Eg + kReducePer - 1) / kReducePer * kReducePer;
  }
  t.E = E;
  t.G = (int)grp.geoms.size();
  t.nblk_red = E / kReducePer;
  size_t total, off[9];
  ws_layout(t, b->R, &total, off);
  if (t_out) *t_out = t;
  return total;
}

// Advance a plain run through the Delta list, writing Sigma_A [R][nd][3]
// and (if non-NULL) the moments [R][nd][6]; stops at the first Delta whose
// moments fail the mass check and reports it.
void solve_deltas(dgd_run* run, const std::vector<std::pair<int64_t, double>>& sched, int n_points,
                  int n_deltas, double* sigma_out, double* moments_out,
                  std::vector<double>* all = nullptr) {
  std::vector<double> mom((size_t)n_points * 6);
  if (all) all->assign((size_t)n_points * n_deltas * 6, 0.0);
  std::string why;
  for (int k = 0; k < n_deltas; ++k) {
    run_advance(run, sched[k].first, sched[k].second);
    const int mrc = run_moments(run, mom.data(), &why);
    for (int r = 0; r < n_points; ++r) {
      const double* m = &mom[(size_t)r * 6];
      double* s = &sigma_out[((size_t)r * n_deltas + k) * 3];
      s[0] = m[3] / m[0];
      s[1] = m[4] / m[0];
      s[2] = m[5] / m[0];
      if (moments_out) std::memcpy(&moments_out[((size_t)r * n_deltas + k) * 6], m, 6 * sizeof(double));
      if (all) std::memcpy(&(*all)[((size_t)r * n_deltas + k) * 6], m, 6 * sizeof(double));
    }
    if (mrc) fail(mrc, why);
  }
}

// Device scratch of the allocation-free solve: a fixed array in the code
// object, so each GPU the library runs on holds its own copy until the
// process ends.  In host code `scratch` is only a host-side stand-in for
// the symbol: each device's copy is resolved once, with that device
// current, through hipGetSymbolAddress, and only that address is passed on.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

void* scratch_address(int device) {
  static std::mutex mu;
  static std::map<int, void*> addr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(device);
  if (it != addr.end()) return it->second;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    fail(DGD_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  addr[device] = p;
  return p;
}

}  // namespace
}  // namespace dgd

using namespace dgd;

extern "C" {

int dgd_version(void) { return 200; }

const char* dgd_last_error(void) { return g_last_error.c_str(); }

int dgd_set_option(const char* name, int64_t value) {
  return guarded([&]() -> int {
    if (!name) fail(DGD_EINVAL, "option name is NULL");
    const std::string n(name);
    if (n == "graphs") g_opt.graphs = value != 0;
    else if (n == "graph_steps") {
      if (value < 1 || value > 4096) fail(DGD_EINVAL, "graph_steps must be in [1, 4096]");
      g_opt.graph_steps = value;
    } else if (n == "stage_epw") {
      if (value < 1 || value > 256) fail(DGD_EINVAL, "stage_epw must be in [1, 256]");
      g_opt.stage_epw = (int)value;
    } else if (n == "stage_waves") {
      if (value < 1 || value > 4) fail(DGD_EINVAL, "stage_waves must be in [1, 4]");
      g_opt.stage_waves = (int)value;
    } else if (n == "xcd_remap") {
      g_opt.xcd_remap = value != 0;
    } else if (n == "stage_grid") {
      if (value < 0 || value > (1 << 24)) fail(DGD_EINVAL, "stage_grid must be in [0, 2^24]");
      g_opt.stage_grid = value;
    } else if (n == "p3_mfma") {
      if (value < 0 || value > 2) fail(DGD_EINVAL, "p3_mfma must be 0, 1 or 2");
      g_opt.p3_mfma = (int)value;
    } else if (n == "mesh_strip") {
      if (value < 0 || value > 16384) fail(DGD_EINVAL, "mesh_strip must be in [0, 16384]");
      g_opt.mesh_strip = (int)value;
    } else if (n == "mesh_group") {
      if (value < 1 || value > 64) fail(DGD_EINVAL, "mesh_group must be in [1, 64]");
      g_opt.mesh_group = (int)value;
    } else if (n == "packed") {
      g_opt.packed = value != 0;
    } else if (n == "sort_classes") {
      if (value < 0 || value > 1) fail(DGD_EINVAL, "sort_classes must be 0 or 1");
      g_opt.sort_classes = (int)value;
    } else if (n == "autotune") {
      g_opt.autotune = value != 0;
    } else fail(DGD_EINVAL, "unknown option " + n);
    return DGD_OK;
  });
}

int dgd_autotune(dgd_op* op, int32_t n_points, void* hip_stream, int32_t* shape_out,
                 double* ms_out) {
  void* a = nullptr;
  void* b = nullptr;
  void* c = nullptr;
  void* qb = nullptr;
  int rc = guarded([&]() -> int {
    if (!op) fail(DGD_EINVAL, "op is NULL");
    if (n_points < 1) fail(DGD_EINVAL, "n_points must be >= 1");
    RunTarget t = run_target(op, n_points);
    const size_t bytes = (size_t)t.E * t.np * n_points * state_bytes(t.prec);
    DGD_HIP_CHECK(hipMalloc(&a, bytes));
    DGD_HIP_CHECK(hipMalloc(&b, bytes));
    DGD_HIP_CHECK(hipMalloc(&c, bytes));
    if (t.form == 1) {
      DGD_HIP_CHECK(hipMalloc(&qb, 2 * bytes));
      t.qbuf = qb;
    }
    const int64_t n = (int64_t)(bytes / state_bytes(t.prec));
    if (t.prec == DGD_FP64)
      launch_fill_random((double*)c, n, 0xba5eull, (hipStream_t)hip_stream);
    else
      launch_fill_random_f32((float*)c, n, 0xba5eull, (hipStream_t)hip_stream);
    tune_target(t, n_points, a, b, c, (hipStream_t)hip_stream, true);
    const StageKind kind = stage_kind(t, n_points);
    TuneParams p;
    if (!tune_find(kind_key(t, n_points, kind), &p)) fail(DGD_EDEVICE, "tuning left no entry");
    if (shape_out) {
      shape_out[0] = p.epw;
      shape_out[1] = p.waves;
      shape_out[2] = p.remap;
      shape_out[3] = p.grid_per_cu;
    }
    if (ms_out) *ms_out = p.ms;
    return DGD_OK;
  });
  (void)hipFree(a);
  (void)hipFree(b);
  (void)hipFree(c);
  (void)hipFree(qb);
  return rc;
}

int dgd_tune_export(char* buf, size_t cap, size_t* len_out) {
  return guarded([&]() -> int {
    const std::string s = tune_export();
    if (len_out) *len_out = s.size() + 1;
    if (buf) {
      if (cap < s.size() + 1) fail(DGD_EINVAL, "buffer smaller than the table");
      std::memcpy(buf, s.c_str(), s.size() + 1);
    }
    return DGD_OK;
  });
}

int dgd_tune_import(const char* text) {
  return guarded([&]() -> int {
    if (!text) fail(DGD_EINVAL, "text is NULL");
    return tune_import(text) >= 0 ? DGD_OK : DGD_EINVAL;
  });
}

void dgd_tune_clear(void) { tune_clear(); }

int dgd_mesh_create(double L_um, int32_t n_cells, const double* disks, int32_t n_disks,
                    dgd_mesh** out) {
  return guarded([&]() -> int {
    if (!out) fail(DGD_EINVAL, "out is NULL");
    *out = nullptr;
    if (!(L_um > 0) || !std::isfinite(L_um)) fail(DGD_EINVAL, "L must be positive and finite");
    if (n_cells < 1 || n_cells > kMaxCells) fail(DGD_EINVAL, "n_cells must be in [1, 16383]");
    if (n_disks < 0 || (n_disks > 0 && !disks)) fail(DGD_EINVAL, "bad disk list");
    for (int d = 0; d < n_disks; ++d)
      for (int k = 0; k < 3; ++k)
        if (!std::isfinite(disks[3 * d + k])) fail(DGD_EINVAL, "disk list holds a non-finite value");
    auto* m = new dgd_mesh();
    try {
      build_mesh_host(L_um, n_cells, disks, n_disks, g_opt.mesh_strip, g_opt.mesh_group, m->host);
      const int64_t E = m->host.n_elements();
      if (E > ((int64_t)1 << 31) - 1) fail(DGD_EINVAL, "too many elements");
      std::vector<int4> pk(E);
      for (int64_t e = 0; e < E; ++e) {
        int mask = 0;
        for (int f = 0; f < 3; ++f)
          if (m->host.nbr[e * 3 + f] >= 0) mask |= 1 << f;
        pk[e].x = m->host.nbr[e * 3 + 0];
        pk[e].y = m->host.nbr[e * 3 + 1];
        pk[e].z = m->host.nbr[e * 3 + 2];
        pk[e].w = (int)((uint32_t)m->host.orient[e] | ((uint32_t)mask << 1) |
                        ((uint32_t)m->host.ci[e] << 4) | ((uint32_t)m->host.cj[e] << 18));
      }
      m->packed = std::move(pk);
    } catch (...) {
      delete m;
      throw;
    }
    *out = m;
    return DGD_OK;
  });
}

int dgd_mesh_info(const dgd_mesh* mesh, int64_t* n_active, int64_t* n_faces, int32_t* n_components,
                  double* removed_fraction) {
  return guarded([&]() -> int {
    if (!mesh) fail(DGD_EINVAL, "mesh is NULL");
    if (n_active) *n_active = mesh->host.n_elements();
    if (n_faces) *n_faces = mesh->host.n_faces;
    if (n_components) *n_components = mesh->host.n_components;
    if (removed_fraction) {
      int64_t act = 0;
      for (auto a : mesh->host.active_cell) act += a;
      *removed_fraction = 1.0 - (double)act / (double)mesh->host.active_cell.size();
    }
    return DGD_OK;
  });
}

int dgd_mesh_elements(const dgd_mesh* mesh, int32_t* cell_i, int32_t* cell_j, int8_t* orient) {
  return guarded([&]() -> int {
    if (!mesh) fail(DGD_EINVAL, "mesh is NULL");
    const int64_t E = mesh->host.n_elements();
    if (cell_i) std::memcpy(cell_i, mesh->host.ci.data(), E * sizeof(int32_t));
    if (cell_j) std::memcpy(cell_j, mesh->host.cj.data(), E * sizeof(int32_t));
    if (orient) std::memcpy(orient, mesh->host.orient.data(), E * sizeof(int8_t));
    return DGD_OK;
  });
}

int dgd_mesh_faces(const dgd_mesh* mesh, int32_t* nbr_out) {
  return guarded([&]() -> int {
    if (!mesh || !nbr_out) fail(DGD_EINVAL, "NULL argument");
    std::memcpy(nbr_out, mesh->host.nbr.data(), mesh->host.nbr.size() * sizeof(int32_t));
    return DGD_OK;
  });
}

int dgd_mesh_occupancy(const dgd_mesh* mesh, int32_t size, uint8_t* image_out) {
  return guarded([&]() -> int {
    if (!mesh || !image_out || size < 1 || size > 16384) fail(DGD_EINVAL, "bad argument");
    const MeshHost& m = mesh->host;
    for (int j = 0; j < size; ++j)
      for (int i = 0; i < size; ++i) {
        const int ci = std::min(m.N - 1, (int)(((i + 0.5) / size) * m.N));
        const int cj = std::min(m.N - 1, (int)(((j + 0.5) / size) * m.N));
        image_out[(size_t)j * size + i] = m.active_cell[(size_t)cj * m.N + ci] ? 0 : 1;
      }
    return DGD_OK;
  });
}

void dgd_mesh_destroy(dgd_mesh* mesh) {
  if (!mesh) return;
  if (mesh->d_elem) (void)hipFree(mesh->d_elem);
  for (auto& o : mesh->order)
    if (o.d_elem) (void)hipFree(o.d_elem);
  delete mesh;
}

int dgd_operator_build(const dgd_mesh* mesh, int32_t p, double D_um2_per_ms, double eta,
                       int32_t precision, double dt_max_ms, dgd_op** out) {
  return dgd_operator_build_outer(mesh, p, D_um2_per_ms, eta, precision, dt_max_ms,
                                  DGD_OUTER_REFLECT, out);
}

// Operator build shared by the entry points: form 0 is the primal SIPG
// operator (outer condition `outer`), form 1 the mixed form with k = 0 in
// the cells of `disks`.
static int build_operator(const dgd_mesh* mesh, int32_t p, double D_um2_per_ms, double eta,
                   int32_t precision, double dt_max_ms, int32_t outer, int form,
                   const double* disks, int32_t n_disks, dgd_op** out) {
  return guarded([&]() -> int {
    if (!out) fail(DGD_EINVAL, "out is NULL");
    if (outer != DGD_OUTER_REFLECT && outer != DGD_OUTER_ABSORB)
      fail(DGD_EINVAL, "outer must be DGD_OUTER_REFLECT or DGD_OUTER_ABSORB");
    *out = nullptr;
    if (!mesh) fail(DGD_EINVAL, "mesh is NULL");
    if (p < 1 || p > 3) fail(DGD_EINVAL, "p must be 1, 2 or 3");
    if (!(D_um2_per_ms > 0) || !std::isfinite(D_um2_per_ms)) fail(DGD_EINVAL, "D must be positive");
    if (!(eta > 0) || !std::isfinite(eta)) fail(DGD_EINVAL, "eta must be positive");
    if (precision != DGD_FP64 && precision != DGD_FP32 && precision != DGD_BF16X3)
      fail(DGD_EINVAL, "precision must be DGD_FP64, DGD_FP32 or DGD_BF16X3");
    if (precision == DGD_BF16X3 && (p != 3 || form != 0 || outer != DGD_OUTER_REFLECT))
      fail(DGD_EINVAL, "DGD_BF16X3 (BF16 hi/lo split products on matrix cores) is the P3 "
                       "primal operator with zero-flux walls only");
    if (!std::isfinite(dt_max_ms)) fail(DGD_EINVAL, "dt_max_ms must be finite");
    if (mesh->host.n_elements() == 0) fail(DGD_EINVAL, "mesh has no active element");
    auto* op = new dgd_op();
    try {
      ensure_mesh_on_device(mesh);
      op->mesh = mesh;
      op->precision = precision == DGD_BF16X3 ? DGD_FP32 : precision;   // state precision
      op->bf16x3 = precision == DGD_BF16X3;
      op->D = D_um2_per_ms;
      op->ref = build_ref_elem(p, eta);
      const RefElem& R = op->ref;
      const int np = R.np;
      // element matrices stay FP64 for both state precisions (FP64 element arithmetic)
      op->d_S = upload(R.S);
      op->d_N = upload(R.Nb);
      op->d_F = upload(R.Fs);
      op->outer = outer;
      if (outer == DGD_OUTER_ABSORB) op->d_B = upload(R.Bd);
      op->d_Minv = (double*)upload(R.Minv);
      const double h = mesh->host.h;
      std::vector<double> Wp(R.W.size()), Mp(R.Mass.size());
      for (int o = 0; o < 2; ++o)
        for (int a = 0; a < 6; ++a) {
          const double s = h * h * (a == 0 ? 1.0 : (a < 3 ? h : h * h));
          for (int j = 0; j < np; ++j) Wp[(o * 6 + a) * np + j] = R.W[(o * 6 + a) * np + j] * s;
        }
      for (size_t k = 0; k < Mp.size(); ++k) Mp[k] = R.Mass[k] * h * h;
      op->d_W = (double*)upload(Wp);
      op->d_Mass = (double*)upload(Mp);
      if (p == 3 && op->precision == DGD_FP32 && form == 0) build_p3_tables(op);
      if (form == 1) build_mixed_tables(op, disks, n_disks);
      op->quad = build_ic_quadrature(R, kQuadN);
      op->nq = kQuadN * kQuadN;
      op->d_quad = (double*)upload(op->quad);
      const double dt_formula = 0.1 * h * h / (D_um2_per_ms * (p + 1) * (p + 1));
      if (dt_max_ms > 0) {
        op->dt_nom = std::min(dt_formula, dt_max_ms);
        op->lambda_max = 0;
        op->dt_rule = dt_formula <= dt_max_ms ? "formula" : "caller";
      } else {
        const double lam = power_lambda(op, 400) * D_um2_per_ms / (h * h);
        op->lambda_max = lam;
        const double dt_stab = 0.9 * rk3_limit() / (1.05 * lam);
        op->dt_nom = std::min(dt_formula, dt_stab);
        op->dt_rule = dt_formula <= dt_stab ? "formula" : "stability";
      }
    } catch (...) {
      dgd_operator_destroy(op);
      throw;
    }
    *out = op;
    return DGD_OK;
  });
}

int dgd_operator_build_outer(const dgd_mesh* mesh, int32_t p, double D_um2_per_ms, double eta,
                             int32_t precision, double dt_max_ms, int32_t outer, dgd_op** out) {
  return build_operator(mesh, p, D_um2_per_ms, eta, precision, dt_max_ms, outer, 0, nullptr, 0, out);
}

int dgd_operator_build_mixed(const dgd_mesh* mesh, const double* disks, int32_t n_disks, int32_t p,
                             double D_um2_per_ms, int32_t precision, double dt_max_ms,
                             dgd_op** out) {
  if (n_disks < 0 || (n_disks > 0 && !disks)) {
    set_error(DGD_EINVAL, "bad disk list");
    return DGD_EINVAL;
  }
  for (int d = 0; d < n_disks; ++d)
    if (!std::isfinite(disks[3 * d]) || !std::isfinite(disks[3 * d + 1]) ||
        !std::isfinite(disks[3 * d + 2])) {
      set_error(DGD_EINVAL, "non-finite disk");
      return DGD_EINVAL;
    }
  // the penalty of the primal matrices built alongside is unused
  return build_operator(mesh, p, D_um2_per_ms, 10.0, precision, dt_max_ms, DGD_OUTER_REFLECT, 1,
                        disks, n_disks, out);
}

int dgd_operator_dt(const dgd_op* op, double* dt_nom_ms, double* lambda_max_per_ms) {
  return guarded([&]() -> int {
    if (!op) fail(DGD_EINVAL, "op is NULL");
    if (dt_nom_ms) *dt_nom_ms = op->dt_nom;
    if (lambda_max_per_ms) *lambda_max_per_ms = op->lambda_max;
    return DGD_OK;
  });
}

int dgd_operator_info(const dgd_op* op, int32_t* np, double* nodes, int32_t* precision) {
  return guarded([&]() -> int {
    if (!op) fail(DGD_EINVAL, "op is NULL");
    if (np) *np = op->ref.np;
    if (nodes) std::memcpy(nodes, op->ref.nodes.data(), op->ref.nodes.size() * sizeof(double));
    if (precision) *precision = op->bf16x3 ? DGD_BF16X3 : op->precision;
    return DGD_OK;
  });
}

int dgd_workspace_size(const dgd_op* op, int32_t n_points, size_t* bytes) {
  return guarded([&]() -> int {
    if (!op || !bytes) fail(DGD_EINVAL, "NULL argument");
    if (n_points < 1) fail(DGD_EINVAL, "n_points must be >= 1");
    size_t off[9];
    ws_layout(run_target(op, n_points), n_points, bytes, off);
    return DGD_OK;
  });
}

int dgd_operator_apply(dgd_op* op, const void* d_in, void* d_out, int32_t n_rhs, void* hip_stream) {
  return guarded([&]() -> int {
    if (!op || !d_in || !d_out) fail(DGD_EINVAL, "NULL argument");
    if (n_rhs < 1) fail(DGD_EINVAL, "n_rhs must be >= 1");
    if (d_in == d_out) fail(DGD_EINVAL, "input and output must not overlap");
    const double h = op->mesh->host.h;
    RunTarget t = plain_target(op);
    const StageKind kind = stage_kind(t, n_rhs);
    void* q = nullptr;
    if (t.form == 1) {
      // the gradient pass needs [E][2][np][n_rhs] scratch: allocated per call
      DGD_HIP_CHECK(hipMalloc(&q, (size_t)t.E * 2 * t.np * n_rhs * state_bytes(t.prec)));
      t.qbuf = q;
    }
    try {
      stage(t, kind, pick_shape(t, n_rhs, kind), d_in, nullptr, d_out, 0, 0.0, op->D / (h * h),
            n_rhs, (hipStream_t)hip_stream);
      DGD_HIP_CHECK(hipGetLastError());
      if (q) DGD_HIP_CHECK(hipStreamSynchronize((hipStream_t)hip_stream));
    } catch (...) {
      if (q) {
        (void)hipStreamSynchronize((hipStream_t)hip_stream);
        (void)hipFree(q);
      }
      throw;
    }
    if (q) DGD_HIP_CHECK(hipFree(q));
    return DGD_OK;
  });
}

void dgd_operator_destroy(dgd_op* op) {
  if (!op) return;
  (void)hipFree(op->d_S);
  (void)hipFree(op->d_N);
  (void)hipFree(op->d_F);
  (void)hipFree(op->d_B);
  (void)hipFree(op->d_MG);
  (void)hipFree(op->d_MD);
  (void)hipFree(op->d_MN);
  (void)hipFree(op->d_MNcol);
  (void)hipFree(op->d_meta);
  (void)hipFree(op->d_elem_ic);
  (void)hipFree(op->d_Minv);
  (void)hipFree(op->d_W);
  (void)hipFree(op->d_Mass);
  (void)hipFree(op->d_quad);
  (void)hipFree(op->d_Atab);
  (void)hipFree(op->d_Atab_bf);
  (void)hipFree(op->d_Ctab);
  (void)hipFree(op->d_Wtab);
  delete op;
}

int dgd_run_create(dgd_op* op, const double* points, int32_t n_points, double sigma0_um, void* d_ws,
                   size_t ws_bytes, void* hip_stream, dgd_run** out) {
  return guarded([&]() -> int {
    if (!out) fail(DGD_EINVAL, "out is NULL");
    *out = nullptr;
    if (!op || !points) fail(DGD_EINVAL, "NULL argument");
    if (n_points < 1) fail(DGD_EINVAL, "n_points must be >= 1");
    if (!(sigma0_um >= 0) || !std::isfinite(sigma0_um)) fail(DGD_EINVAL, "sigma0 must be >= 0");
    check_points(op->mesh->host, points, n_points);
    check_axon_cells(op, points, n_points);
    *out = run_create(run_target(op, n_points), points, n_points, sigma0_um, d_ws, ws_bytes, hip_stream);
    return DGD_OK;
  });
}

int dgd_run_advance(dgd_run* run, int64_t n_steps, double dt_ms) {
  return guarded([&]() -> int {
    if (!run) fail(DGD_EINVAL, "run is NULL");
    run_advance(run, n_steps, dt_ms);
    return DGD_OK;
  });
}

int dgd_run_moments(dgd_run* run, double* moments_out, size_t n_doubles) {
  return guarded([&]() -> int {
    if (!run || !moments_out) fail(DGD_EINVAL, "NULL argument");
    if (n_doubles < (size_t)run->t.G * run->R * 6)
      fail(DGD_EINVAL, "moments buffer of " + std::to_string(n_doubles) + " doubles; the run needs " +
                           std::to_string((size_t)run->t.G * run->R * 6));
    std::string why;
    const int rc = run_moments(run, moments_out, &why);
    if (rc) fail(rc, why);
    return DGD_OK;
  });
}

int dgd_run_signal(dgd_run* run, const double* q, int32_t n_q, double* signal_out) {
  return guarded([&]() -> int {
    if (!run || !q || !signal_out) fail(DGD_EINVAL, "NULL argument");
    if (n_q < 1) fail(DGD_EINVAL, "n_q must be >= 1");
    run_signal(run, q, n_q, signal_out);
    return DGD_OK;
  });
}

// Mesh elements whose state a plain run's host buffers hold: the run's own
// table may be class-sorted and padded (run_target), the host layout is
// the mesh order.
static int64_t mesh_elements(const dgd_run* run) {
  return run->t.member_index ? (int64_t)(*run->t.member_index)[0].size() : run->t.E;
}

int dgd_run_shape(const dgd_run* run, int64_t* n_values, int32_t* n_points, int32_t* value_bytes) {
  return guarded([&]() -> int {
    if (!run) fail(DGD_EINVAL, "run is NULL");
    if (n_values) *n_values = mesh_elements(run) * run->t.np * (int64_t)run->R;
    if (n_points) *n_points = run->R;
    if (value_bytes) *value_bytes = (int32_t)state_bytes(run->t.prec);
    return DGD_OK;
  });
}

int dgd_run_get_state(dgd_run* run, void* host_out, size_t bytes) {
  return guarded([&]() -> int {
    if (!run || !host_out) fail(DGD_EINVAL, "NULL argument");
    const RunTarget& t = run->t;
    const size_t eb = (size_t)t.np * run->R * state_bytes(t.prec);   // bytes per element
    const size_t n = (size_t)mesh_elements(run) * eb;
    if (bytes < n)
      fail(DGD_EINVAL, "state buffer of " + std::to_string(bytes) + " bytes; the run needs " +
                           std::to_string(n));
    if (!t.member_index) {
      DGD_HIP_CHECK(hipMemcpyAsync(host_out, run->U, n, hipMemcpyDeviceToHost, run->stream));
      DGD_HIP_CHECK(hipStreamSynchronize(run->stream));
      return DGD_OK;
    }
    std::vector<char> buf((size_t)t.E * eb);
    DGD_HIP_CHECK(hipMemcpyAsync(buf.data(), run->U, buf.size(), hipMemcpyDeviceToHost, run->stream));
    DGD_HIP_CHECK(hipStreamSynchronize(run->stream));
    const std::vector<int64_t>& at = (*t.member_index)[0];
    for (size_t e = 0; e < at.size(); ++e)
      std::memcpy((char*)host_out + e * eb, &buf[(size_t)at[e] * eb], eb);
    return DGD_OK;
  });
}

int dgd_run_set_state(dgd_run* run, const void* host_in, size_t bytes) {
  return guarded([&]() -> int {
    if (!run || !host_in) fail(DGD_EINVAL, "NULL argument");
    const RunTarget& t = run->t;
    const size_t eb = (size_t)t.np * run->R * state_bytes(t.prec);
    const size_t n = (size_t)mesh_elements(run) * eb;
    if (bytes != n)
      fail(DGD_EINVAL, "state buffer of " + std::to_string(bytes) + " bytes; the run holds " +
                           std::to_string(n));
    if (t.member_index) {
      // padding elements of the sorted table stay zero
      std::vector<char> buf((size_t)t.E * eb, 0);
      const std::vector<int64_t>& at = (*t.member_index)[0];
      for (size_t e = 0; e < at.size(); ++e)
        std::memcpy(&buf[(size_t)at[e] * eb], (const char*)host_in + e * eb, eb);
      DGD_HIP_CHECK(hipMemcpyAsync(run->U, buf.data(), buf.size(), hipMemcpyHostToDevice, run->stream));
      DGD_HIP_CHECK(hipStreamSynchronize(run->stream));
      return DGD_OK;
    }
    if (t.form == 1) {
      // mixed form: u is zero in axon cells (k = 0, no flux in); the stage
      // kernels never touch those blocks, so they are cleared here
      const MeshHost& m = *t.hosts[0].first;
      const size_t blk = (size_t)t.np * run->R * state_bytes(t.prec);
      std::vector<char> buf((const char*)host_in, (const char*)host_in + n);
      for (int64_t e = 0; e < t.E; ++e)
        if (t.axon_host[(size_t)m.cj[e] * m.N + m.ci[e]]) std::memset(&buf[e * blk], 0, blk);
      DGD_HIP_CHECK(hipMemcpyAsync(run->U, buf.data(), n, hipMemcpyHostToDevice, run->stream));
      DGD_HIP_CHECK(hipStreamSynchronize(run->stream));
      return DGD_OK;
    }
    DGD_HIP_CHECK(hipMemcpyAsync(run->U, host_in, n, hipMemcpyHostToDevice, run->stream));
    DGD_HIP_CHECK(hipStreamSynchronize(run->stream));
    return DGD_OK;
  });
}

int dgd_run_kernel(const dgd_run* run, int32_t* kernel_out, int64_t* shape_out) {
  return guarded([&]() -> int {
    if (!run) fail(DGD_EINVAL, "run is NULL");
    if (kernel_out) *kernel_out = run->kind;
    if (shape_out) {
      shape_out[0] = run->sh.epw;
      shape_out[1] = run->sh.waves;
      shape_out[2] = run->sh.remap ? 1 : 0;
      shape_out[3] = run->sh.grid;
    }
    return DGD_OK;
  });
}

int dgd_run_step_count(const dgd_run* run, int64_t* steps_out) {
  return guarded([&]() -> int {
    if (!run || !steps_out) fail(DGD_EINVAL, "NULL argument");
    *steps_out = run->steps;
    return DGD_OK;
  });
}

int dgd_run_set_step_count(dgd_run* run, int64_t steps) {
  return guarded([&]() -> int {
    if (!run) fail(DGD_EINVAL, "run is NULL");
    if (steps < 0) fail(DGD_EINVAL, "steps must be >= 0");
    const uint32_t v = (uint32_t)steps;
    DGD_HIP_CHECK(hipMemcpyAsync(run->d_step, &v, sizeof(v), hipMemcpyHostToDevice, run->stream));
    DGD_HIP_CHECK(hipStreamSynchronize(run->stream));
    run->steps = steps;
    return DGD_OK;
  });
}

void dgd_run_destroy(dgd_run* run) { run_destroy(run); }

int dgd_eap_solve(dgd_op* op, const double* points, int32_t n_points, double sigma0_um,
                  const double* deltas_ms, int32_t n_deltas, double* sigma_out, double* moments_out,
                  void* d_ws, size_t ws_bytes, void* hip_stream) {
  dgd_run* run = nullptr;
  std::vector<std::pair<int64_t, double>> sched;
  int rc = guarded([&]() -> int {
    if (!op || !deltas_ms || !sigma_out) fail(DGD_EINVAL, "NULL argument");
    if (n_deltas < 1) fail(DGD_EINVAL, "n_deltas must be >= 1");
    sched = schedule(deltas_ms, n_deltas, op->dt_nom);
    return DGD_OK;
  });
  if (rc) return rc;
  Range range("dgd:eap_solve");
  const auto t0 = std::chrono::steady_clock::now();
  rc = dgd_run_create(op, points, n_points, sigma0_um, d_ws, ws_bytes, hip_stream, &run);
  if (rc) return rc;
  std::vector<double> all;
  rc = guarded([&]() -> int {
    solve_deltas(run, sched, n_points, n_deltas, sigma_out, moments_out, &all);
    return DGD_OK;
  });
  int64_t steps = 0;
  for (const auto& s : sched) steps += s.first;
  const int64_t E = op->mesh->host.n_elements();
  log_run("dgd_eap_solve", op, 1, E, n_points, deltas_ms, n_deltas, steps,
          (double)E * op->ref.np * n_points * steps, seconds_since(t0), rc, all.data(),
          kKindName[run->kind]);
  dgd_run_destroy(run);
  return rc;
}

int dgd_eap_solve_noalloc(dgd_op* op, const double* points, int32_t n_points, double sigma0_um,
                          const double* deltas_ms, int32_t n_deltas, double* sigma_out,
                          double* moments_out, void* hip_stream) {
  dgd_run* run = nullptr;
  const int rc = guarded([&]() -> int {
    if (!op || !points || !deltas_ms || !sigma_out) fail(DGD_EINVAL, "NULL argument");
    if (n_points < 1) fail(DGD_EINVAL, "n_points must be >= 1");
    if (n_deltas < 1) fail(DGD_EINVAL, "n_deltas must be >= 1");
    if (!(sigma0_um > 0) || !std::isfinite(sigma0_um))
      fail(DGD_EINVAL, "the allocation-free solve needs sigma0 > 0 (point-mass data allocate)");
    int dev = -1;
    DGD_HIP_CHECK(hipGetDevice(&dev));
    if (dev != op->mesh->device)
      fail(DGD_EINVAL, "the current device is not the one the operator was built on");
    const auto sched = schedule(deltas_ms, n_deltas, op->dt_nom);
    const RunTarget t = run_target(op, n_points);
    size_t total, off[9];
    ws_layout(t, n_points, &total, off);
    if (total > kScratchBytes)
      fail(DGD_ENOMEM, "the allocation-free solve needs " + std::to_string(total) +
                           " bytes of device scratch; its limit is " +
                           std::to_string(kScratchBytes) + " bytes (64 MiB)");
    check_points(op->mesh->host, points, n_points);
    check_axon_cells(op, points, n_points);
    run = run_create(t, points, n_points, sigma0_um, scratch_address(dev), kScratchBytes,
                     hip_stream, true);
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<double> all;
    int status = DGD_OK;
    std::string why;
    try {
      solve_deltas(run, sched, n_points, n_deltas, sigma_out, moments_out, &all);
    } catch (const Error& e) {
      status = e.code;
      why = e.msg;
    }
    int64_t steps = 0;
    for (const auto& s : sched) steps += s.first;
    const int64_t E = op->mesh->host.n_elements();
    log_run("dgd_eap_solve_noalloc", op, 1, E, n_points, deltas_ms, n_deltas, steps,
            (double)E * op->ref.np * n_points * steps, seconds_since(t0), status, all.data(),
            kKindName[run->kind]);
    if (status) fail(status, why);
    return DGD_OK;
  });
  run_destroy(run);
  return rc;
}

int dgd_eap_solve_signal(dgd_op* op, const double* points, int32_t n_points, double sigma0_um,
                         const double* deltas_ms, int32_t n_deltas, const double* q, int32_t n_q,
                         double* signal_out, double* moments_out, void* d_ws, size_t ws_bytes,
                         void* hip_stream) {
  dgd_run* run = nullptr;
  std::vector<std::pair<int64_t, double>> sched;
  int rc = guarded([&]() -> int {
    if (!op || !deltas_ms || !q || !signal_out) fail(DGD_EINVAL, "NULL argument");
    if (n_deltas < 1 || n_q < 1) fail(DGD_EINVAL, "bad counts");
    sched = schedule(deltas_ms, n_deltas, op->dt_nom);
    return DGD_OK;
  });
  if (rc) return rc;
  rc = dgd_run_create(op, points, n_points, sigma0_um, d_ws, ws_bytes, hip_stream, &run);
  if (rc) return rc;
  rc = guarded([&]() -> int {
    std::vector<double> mom((size_t)n_points * 6), sig((size_t)n_points * n_q * 2);
    std::string why;
    for (int k = 0; k < n_deltas; ++k) {
      run_advance(run, sched[k].first, sched[k].second);
      const int mrc = run_moments(run, mom.data(), &why);
      if (mrc) fail(mrc, why);
      run_signal(run, q, n_q, sig.data());
      for (int r = 0; r < n_points; ++r) {
        std::memcpy(&signal_out[(((size_t)r * n_deltas + k) * n_q) * 2], &sig[(size_t)r * n_q * 2],
                    (size_t)n_q * 2 * sizeof(double));
        if (moments_out)
          std::memcpy(&moments_out[((size_t)r * n_deltas + k) * 6], &mom[(size_t)r * 6],
                      6 * sizeof(double));
      }
    }
    return DGD_OK;
  });
  dgd_run_destroy(run);
  return rc;
}

int dgd_eap_solve_expm(dgd_op* op, const double* points, int32_t n_points, double sigma0_um,
                       const double* deltas_ms, int32_t n_deltas, double lambda_bound,
                       double* sigma_out, double* moments_out, int64_t* n_applies) {
  dgd_run* run = nullptr;
  double* buf = nullptr;
  int rc = guarded([&]() -> int {
    if (!op || !points || !deltas_ms || !sigma_out) fail(DGD_EINVAL, "NULL argument");
    if (n_points < 1 || n_deltas < 1) fail(DGD_EINVAL, "bad counts");
    if (!(sigma0_um >= 0) || !std::isfinite(sigma0_um)) fail(DGD_EINVAL, "sigma0 must be >= 0");
    if (op->form != 0)
      fail(DGD_EINVAL, "the Chebyshev exponential needs a real spectrum: primal operators only");
    schedule(deltas_ms, n_deltas, 1.0);  // validates the list
    check_points(op->mesh->host, points, n_points);
    double b = lambda_bound;
    if (!(b > 0)) {
      double lam = op->lambda_max;
      if (!(lam > 0)) lam = power_lambda(op, 400) * op->D / (op->mesh->host.h * op->mesh->host.h);
      b = 1.05 * lam;
    }
    RunTarget t = plain_target(op);
    t.prec = DGD_FP64;           // the recurrence runs on an FP64 state
    t.Atab = nullptr;
    t.Atab_bf = nullptr;
    run = run_create(t, points, n_points, sigma0_um, nullptr, 0, nullptr);
    const int64_t n = t.E * t.np * (int64_t)n_points;
    DGD_HIP_CHECK(hipMalloc(&buf, (size_t)n * sizeof(double)));
    double* res = (double*)run->U;   // u, then the running sum
    double* T[3] = {(double*)run->U1, (double*)run->U2, buf};
    // the recurrence runs the one-element-per-wave kernel
    const Shape sh = pick_shape(t, n_points, kValu);
    const double cg = 2.0 * t.D / (b * t.h * t.h);    // X = I + (2 / b) L, L = (D / h^2) Lhat
    int64_t applies = 0;
    std::vector<double> mom((size_t)n_points * 6);
    int status = DGD_OK;
    std::string why;
    double prev = 0;
    for (int kd = 0; kd < n_deltas && status == DGD_OK; ++kd) {
      const std::vector<double> c = cheb_coefficients(0.5 * b * (deltas_ms[kd] - prev));
      prev = deltas_ms[kd];
      // T0 = u; T_{-1} = X T0 (so that T1 = 2 X T0 - T_{-1} = X T0); res = c0 T0
      launch_axpby(T[0], res, 1.0, 0.0, n, run->stream);
      launch_stage(0, t.np, T[0], nullptr, T[2], t.elem, t.E, t.S, t.N, 1, 0.0, cg, n_points, sh,
                   run->stream, nullptr, 0, t.B);
      launch_axpby(res, T[0], c[0], 0.0, n, run->stream);
      applies += 1;
      int cur = 0, prv = 2;
      for (size_t k = 1; k < c.size(); ++k) {
        const int nxt = 3 - cur - prv;
        launch_cheb(t.np, T[cur], T[prv], T[nxt], res, t.elem, t.E, t.S, t.N, cg, c[k], n_points, sh,
                    run->stream, t.B);
        prv = cur;
        cur = nxt;
        ++applies;
      }
      DGD_HIP_CHECK(hipGetLastError());
      const int mrc = run_moments(run, mom.data(), &why);
      for (int r = 0; r < n_points; ++r) {
        const double* m = &mom[(size_t)r * 6];
        double* s = &sigma_out[((size_t)r * n_deltas + kd) * 3];
        s[0] = m[3] / m[0];
        s[1] = m[4] / m[0];
        s[2] = m[5] / m[0];
        if (moments_out)
          std::memcpy(&moments_out[((size_t)r * n_deltas + kd) * 6], m, 6 * sizeof(double));
      }
      if (mrc) status = mrc;
    }
    if (n_applies) *n_applies = applies;
    if (status) fail(status, why);
    return DGD_OK;
  });
  if (run) run_destroy(run);
  if (buf) (void)hipFree(buf);
  return rc;
}

// ---------------------------------------------------------------- batch ----

int dgd_batch_workspace_size(dgd_op* const* ops, int32_t n_geoms, int32_t n_points, size_t* bytes) {
  return guarded([&]() -> int {
    if (!ops || !bytes || n_geoms < 1 || n_points < 1) fail(DGD_EINVAL, "bad argument");
    dgd_batch b;
    b.G = n_geoms;
    b.R = n_points;
    b.ops.assign(ops, ops + n_geoms);
    for (auto* o : b.ops)
      if (!o) fail(DGD_EINVAL, "NULL operator");
    batch_plan(&b);
    size_t total = 0;
    for (auto& g : b.groups) total += align256(batch_group_bytes(g, &b, nullptr));
    *bytes = total;
    return DGD_OK;
  });
}

int dgd_batch_create(dgd_op* const* ops, int32_t n_geoms, const double* points, int32_t n_points,
                     double sigma0_um, void* d_ws, size_t ws_bytes, void* hip_stream,
                     dgd_batch** out) {
  return guarded([&]() -> int {
    if (!out) fail(DGD_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ops || !points || n_geoms < 1 || n_points < 1) fail(DGD_EINVAL, "bad argument");
    if (!(sigma0_um >= 0) || !std::isfinite(sigma0_um)) fail(DGD_EINVAL, "sigma0 must be >= 0");
    for (int g = 0; g < n_geoms; ++g) {
      if (!ops[g]) fail(DGD_EINVAL, "NULL operator");
      if (ops[g]->bf16x3) fail(DGD_EINVAL, "batched solves take DGD_FP64 or DGD_FP32 operators");
      const dgd_op* a = ops[g];
      const dgd_op* z = ops[0];
      if (a->mesh->host.h != z->mesh->host.h || a->D != z->D || a->ref.eta != z->ref.eta ||
          a->precision != z->precision || a->outer != z->outer)
        fail(DGD_EINVAL, "batched operators must share h, D, eta, precision and outer condition");
      check_points(a->mesh->host, points + (size_t)g * n_points * 2, n_points, g * n_points);
    }
    auto* b = new dgd_batch();
    try {
      b->G = n_geoms;
      b->R = n_points;
      b->ops.assign(ops, ops + n_geoms);
      batch_plan(b);
      size_t used = 0;
      for (auto& grp : b->groups) {
        RunTarget t;
        const size_t need = batch_group_bytes(grp, b, &t);
        // concatenated element table, block -> geometry map, block ranges
        std::vector<int4> elem;
        elem.reserve(t.E);
        std::vector<int> blk_geom, blk_start;
        grp.dt = 1e300;
        t.hosts.clear();
        const int Gp = batch_pack(t, b->R);
        std::vector<int4> tab;
        grp.member_index.assign(grp.geoms.size(), {});
        for (int k = 0; k < (int)grp.geoms.size(); ++k) {
          const dgd_op* op = b->ops[grp.geoms[k]];
          const int64_t off = (int64_t)elem.size();
          t.hosts.emplace_back(&op->mesh->host, off);
          blk_start.push_back((int)(off / kReducePer));
          member_table(op->mesh, Gp, &tab, &grp.member_index[k]);
          for (int64_t& i : grp.member_index[k]) i += off;
          for (const int4& e : tab) {
            int4 c = e;
            if (c.x >= 0) c.x += (int)off;
            if (c.y >= 0) c.y += (int)off;
            if (c.z >= 0) c.z += (int)off;
            elem.push_back(c);
          }
          int4 pad;
          pad.x = pad.y = pad.z = -1;
          pad.w = (int)(((uint32_t)kPadCell << 4) | ((uint32_t)kPadCell << 18));
          while (elem.size() % kReducePer) elem.push_back(pad);
          while ((int64_t)blk_geom.size() < (int64_t)elem.size() / kReducePer) blk_geom.push_back(k);
          grp.dt = std::min(grp.dt, op->dt_nom);
          grp.dof += op->mesh->host.n_elements() * op->ref.np;
        }
        blk_start.push_back((int)(elem.size() / kReducePer));
        if ((int64_t)elem.size() != t.E) fail(DGD_EINVAL, "internal: batch size mismatch");
        grp.E = t.E;
        t.member_index = &grp.member_index;
        grp.d_elem = (int4*)upload(elem);
        grp.d_blk_geom = (int*)upload(blk_geom);
        grp.d_blk_start = (int*)upload(blk_start);
        t.elem = grp.d_elem;
        t.blk_geom = grp.d_blk_geom;
        t.blk_start = grp.d_blk_start;
        std::vector<double> x0;
        for (int g : grp.geoms)
          x0.insert(x0.end(), points + (size_t)g * n_points * 2,
                    points + (size_t)(g + 1) * n_points * 2);
        void* ws = nullptr;
        if (d_ws) {
          if (used + need > ws_bytes)
            fail(DGD_ENOMEM, "workspace smaller than dgd_batch_workspace_size");
          ws = (char*)d_ws + used;
          used += align256(need);
        }
        grp.run = run_create(t, x0.data(), n_points, sigma0_um, ws, ws ? need : 0, hip_stream);
      }
    } catch (...) {
      batch_destroy(b);
      throw;
    }
    *out = b;
    return DGD_OK;
  });
}

int dgd_batch_groups(const dgd_batch* b, int32_t* n_groups, int32_t* group_p, int32_t* group_size,
                     double* group_dt, int64_t* group_dof) {
  return guarded([&]() -> int {
    if (!b) fail(DGD_EINVAL, "batch is NULL");
    if (n_groups) *n_groups = (int32_t)b->groups.size();
    for (size_t k = 0; k < b->groups.size(); ++k) {
      if (group_p) group_p[k] = b->groups[k].p;
      if (group_size) group_size[k] = (int32_t)b->groups[k].geoms.size();
      if (group_dt) group_dt[k] = b->groups[k].dt;
      if (group_dof) group_dof[k] = b->groups[k].dof;
    }
    return DGD_OK;
  });
}

int dgd_batch_advance(dgd_batch* b, int32_t group, int64_t n_steps, double dt_ms) {
  return guarded([&]() -> int {
    if (!b || group < 0 || group >= (int)b->groups.size()) fail(DGD_EINVAL, "bad batch or group");
    run_advance(b->groups[group].run, n_steps, dt_ms);
    return DGD_OK;
  });
}

int dgd_batch_shape(const dgd_batch* b, int32_t* n_geoms, int32_t* n_points) {
  return guarded([&]() -> int {
    if (!b) fail(DGD_EINVAL, "batch is NULL");
    if (n_geoms) *n_geoms = b->G;
    if (n_points) *n_points = b->R;
    return DGD_OK;
  });
}

int dgd_batch_moments(dgd_batch* b, double* moments_out, size_t n_doubles) {
  return guarded([&]() -> int {
    if (!b || !moments_out) fail(DGD_EINVAL, "NULL argument");
    if (n_doubles < (size_t)b->G * b->R * 6)
      fail(DGD_EINVAL, "moments buffer of " + std::to_string(n_doubles) + " doubles; the batch needs " +
                           std::to_string((size_t)b->G * b->R * 6));
    int status = DGD_OK;
    std::string why;
    for (auto& grp : b->groups) {
      std::vector<double> m((size_t)grp.geoms.size() * b->R * 6);
      std::string w;
      const int rc = run_moments(grp.run, m.data(), &w);
      if (rc && !status) {
        status = rc;
        why = w;
      }
      for (size_t k = 0; k < grp.geoms.size(); ++k)
        std::memcpy(moments_out + (size_t)grp.geoms[k] * b->R * 6, &m[k * b->R * 6],
                    (size_t)b->R * 6 * sizeof(double));
    }
    if (status) fail(status, why);
    return DGD_OK;
  });
}

void dgd_batch_destroy(dgd_batch* b) { batch_destroy(b); }

int dgd_eap_solve_batch(dgd_op* const* ops, int32_t n_geoms, const double* points,
                        int32_t n_points, double sigma0_um, const double* deltas_ms,
                        int32_t n_deltas, double* sigma_out, double* moments_out, void* d_ws,
                        size_t ws_bytes, void* hip_stream) {
  dgd_batch* b = nullptr;
  int rc = guarded([&]() -> int {
    if (!deltas_ms || !sigma_out || n_deltas < 1) fail(DGD_EINVAL, "bad Delta list or output");
    schedule(deltas_ms, n_deltas, 1.0);  // validates the list
    return DGD_OK;
  });
  if (rc) return rc;
  Range range("dgd:eap_solve_batch");
  const auto t0 = std::chrono::steady_clock::now();
  rc = dgd_batch_create(ops, n_geoms, points, n_points, sigma0_um, d_ws, ws_bytes, hip_stream, &b);
  if (rc) return rc;
  std::vector<double> all((size_t)n_geoms * n_points * n_deltas * 6, 0.0);
  int64_t steps_max = 0;
  double updates = 0;
  rc = guarded([&]() -> int {
    const int R = n_points;
    int status = DGD_OK;
    std::string why;
    for (auto& grp : b->groups) {
      const auto sched = schedule(deltas_ms, n_deltas, grp.dt);
      int64_t gsteps = 0;
      for (const auto& s : sched) gsteps += s.first;
      steps_max = std::max(steps_max, gsteps);
      updates += (double)grp.dof * R * gsteps;
      std::vector<double> m((size_t)grp.geoms.size() * R * 6);
      for (int k = 0; k < n_deltas; ++k) {
        run_advance(grp.run, sched[k].first, sched[k].second);
        std::string w;
        const int mrc = run_moments(grp.run, m.data(), &w);
        for (size_t q = 0; q < grp.geoms.size(); ++q) {
          const int g = grp.geoms[q];
          for (int r = 0; r < R; ++r) {
            const double* mm = &m[(q * R + r) * 6];
            double* s = &sigma_out[(((size_t)g * R + r) * n_deltas + k) * 3];
            s[0] = mm[3] / mm[0];
            s[1] = mm[4] / mm[0];
            s[2] = mm[5] / mm[0];
            if (moments_out)
              std::memcpy(&moments_out[(((size_t)g * R + r) * n_deltas + k) * 6], mm,
                          6 * sizeof(double));
            std::memcpy(&all[(((size_t)g * R + r) * n_deltas + k) * 6], mm, 6 * sizeof(double));
          }
        }
        if (mrc && !status) {
          status = mrc;
          why = w;
        }
      }
    }
    if (status) fail(status, why);
    return DGD_OK;
  });
  int64_t elements = 0;
  for (int g = 0; g < n_geoms; ++g) elements += ops[g]->mesh->host.n_elements();
  log_run("dgd_eap_solve_batch", ops[0], n_geoms, elements, n_geoms * n_points, deltas_ms, n_deltas,
          steps_max, updates, seconds_since(t0), rc, all.data(), "batched");
  dgd_batch_destroy(b);
  return rc;
}

}  // extern "C"
