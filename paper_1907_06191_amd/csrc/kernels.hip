// HIP kernels of the DG diffusion solve (gfx950, 64-wide waves).
//
// Layout: the state of R solves is u[e][j][r] (element, node, right-hand
// side), r fastest, so that a wave's 64 lanes read 64 consecutive values of
// one node of one element: every state access is a fully coalesced
// 256-byte (FP32) or 512-byte (FP64) row.  A wave owns one element at a
// time, so the element's orientation, face mask and neighbours are
// wave-uniform: they come in through one scalar load, and the element
// matrices (shared by all elements of one orientation and mask) are read
// through the scalar cache and used as SGPR operands of the VALU FMAs.
//
// Several geometries can share one launch: their element tables are
// concatenated (disconnected components of one mesh), and the reduction
// kernels read the geometry of each block from `blk_geom` to pick the start
// points of that geometry.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "launch.h"

namespace dgd {
namespace {

constexpr int WAVE = 64;
// Cell index of the padding elements that align each geometry of a batch to
// whole reduction blocks (meshes have at most 16383 cells per side).
constexpr int kPadCell = 0x3fff;

// Logical blocks walked by this workgroup.  Workgroups are dispatched
// round-robin over the 8 XCDs (blockIdx.x mod 8).  With `remap`, XCD x owns
// the contiguous logical range [x * per, (x + 1) * per) and its workgroups
// stride through it in dispatch order, so rows of cells that are face
// neighbours are read while still in that XCD's L2.  A grid smaller than the
// number of logical blocks makes the kernel persistent (each workgroup loops).
struct BlockIter {
  int64_t first, stride, end;
};

__device__ inline BlockIter block_iter(int64_t nblocks, int remap) {
  BlockIter it;
  const int64_t G = gridDim.x;
  if (remap) {
    const int64_t per = (nblocks + 7) / 8;
    const int64_t x = blockIdx.x % 8;
    it.first = x * per + blockIdx.x / 8;
    it.stride = G / 8;
    const int64_t hi = (x + 1) * per;
    it.end = hi < nblocks ? hi : nblocks;
  } else {
    it.first = blockIdx.x;
    it.stride = G;
    it.end = nblocks;
  }
  return it;
}

// Stochastic rounding of an FP64 value to FP32: the FP32 neighbour below
// or above v in magnitude, the upper one with probability equal to the
// fraction of an FP32 ulp that v lies above the lower one, so the rounding
// error has zero mean.  Rounding every stored state to nearest loses
// increments below half an ulp the same way every step (the state then
// drifts, mass included, over 10^5 - 10^6 steps); with stochastic rounding
// the error is a zero-mean random walk.
//
// For v in the FP32 normal range the low 29 of the 52 FP64 mantissa bits
// are that fraction: adding a uniform 29-bit integer r to the magnitude bits
// and clearing those 29 bits carries into the kept part with probability
// fraction / 2^29 (a carry into the exponent is the correct next binade),
// and the result converts to FP32 exactly.  Zero stays zero.  Below the
// FP32 normal range (|v| < 2^-126 ~ 1.2e-38) the truncated value converts
// with the hardware's rounding, an error below 2^-149 that no moment can
// see; |v| >= 2^127 does not occur in a unit-mass state (and overflows to
// infinity, which the mass check reports).
__device__ __forceinline__ float round_stochastic(double v, uint32_t r) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint64_t t = (b + (uint64_t)(r >> 3)) & ~0x1fffffffull;
  return (float)__longlong_as_double((long long)t);
}

// Random bits of the stored values.  A value's bits come from a hash of
// (element, step and stage within the step) XOR a hash of its right-hand
// side, rotated by an amount that depends on its node.  The element part
// is wave-uniform in the one-element-per-wave kernels (scalar ALU work)
// and the right-hand-side part is a constant of the lane, so a stored
// value costs one rotate and one shift of random bits.  Every node's bits
// are uniform and independent of the value they round, and for a fixed
// right-hand side they change with the element and with every step: with
// a threshold fixed in time, a slot whose per-step increment stays below
// it would never move (the stagnation of rounding to nearest, for that
// share of slots), which shows near equilibrium, where increments are a
// small fraction of an ulp step after step.  Nothing depends on where an
// element sits in memory, so a geometry gives the same bits alone or in a
// batch.
__device__ __forceinline__ uint32_t sr_mix(uint32_t x) {
  x *= 0x9E3779B1u;
  x ^= x >> 16;
  x *= 0x85EBCA77u;
  x ^= x >> 13;
  return x;
}
// element part: the element's record word (cell, orientation, face mask)
// and the step/stage mix
__device__ __forceinline__ uint32_t elem_salt(int meta, uint32_t smix) {
  return sr_mix((uint32_t)meta + smix);
}
// right-hand-side part
__device__ __forceinline__ uint32_t rhs_salt(int rhs) {
  return sr_mix((uint32_t)rhs * 0x85EBCA6Bu ^ 0x6A09E667u);
}
__device__ __forceinline__ uint32_t state_salt(int meta, int rhs, uint32_t smix) {
  return elem_salt(meta, smix) ^ rhs_salt(rhs);
}
// the bits of node `node` (node < 32): distinct rotations, so the nodes of
// one element draw from different windows of the hash
__device__ __forceinline__ uint32_t sr_node(uint32_t h, int node) {
  return __builtin_rotateright32(h, (uint32_t)(node * 11) & 31u);
}

// Per-launch part of the salt; step is the run's device step counter
// (NULL: 0), stage_id 0..2 the stage within the RK3 step.
__device__ __forceinline__ uint32_t step_mix(const uint32_t* step, int stage_id) {
  const uint32_t k = step ? step[0] : 0u;
  return (k * 3u + (uint32_t)stage_id) * 0x9E3779B9u;
}
__device__ __forceinline__ void store_state(float* p, int64_t i, double v, uint32_t h, int node) {
  p[i] = round_stochastic(v, sr_node(h, node));
}
__device__ __forceinline__ void store_state(double* p, int64_t i, double v, uint32_t, int) { p[i] = v; }
// the same with a non-temporal store (a stage output is not read again
// within the launch)
__device__ __forceinline__ void store_state_nt(float* p, int64_t i, double v, uint32_t h, int node) {
  __builtin_nontemporal_store(round_stochastic(v, sr_node(h, node)), p + i);
}
__device__ __forceinline__ void store_state_nt(double* p, int64_t i, double v, uint32_t, int) {
  __builtin_nontemporal_store(v, p + i);
}

// Rows of state through a buffer resource based at p (raw addressing, no
// range limit): a load or store names a lane offset (VGPR, fixed for the
// kernel) and a wave-uniform byte offset (SGPR), so per-element address
// arithmetic runs on the scalar unit and costs no vector instructions.
// Cache policy of the state streams (gfx950 buffer instructions: bit 1 =
// non-temporal).  The stage output and the RK base state are touched once
// per launch, so they stream past the caches; the stage input stays
// temporal (face neighbours read it again from L2).
#ifndef DGD_CPOL_OUT
#define DGD_CPOL_OUT 2
#endif
#ifndef DGD_CPOL_BASE
#define DGD_CPOL_BASE 2
#endif
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rows_at(const void* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, -1, 0x00020000);
}
template <int CP>
__device__ __forceinline__ float buf_ld(float*, __amdgpu_buffer_rsrc_t rs, uint32_t voff,
                                        uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, CP));
}
template <int CP>
__device__ __forceinline__ double buf_ld(double*, __amdgpu_buffer_rsrc_t rs, uint32_t voff,
                                         uint32_t soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, CP));
}
template <typename T, int CP = 0>
__device__ __forceinline__ T ld_row(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
  return buf_ld<CP>((T*)nullptr, rs, voff, soff);
}
template <int CP = 0>
__device__ __forceinline__ void st_row(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff,
                                       float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), rs, voff, soff, CP);
}
template <int CP = 0>
__device__ __forceinline__ void st_row(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff,
                                       double v) {
  typedef __attribute__((ext_vector_type(2))) unsigned int u32x2;
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), rs, voff, soff, CP);
}
// a state value rounded for storage: FP32 stochastically, FP64 as is
__device__ __forceinline__ float to_state(float*, double v, uint32_t h, int node) {
  return round_stochastic(v, sr_node(h, node));
}
__device__ __forceinline__ double to_state(double*, double v, uint32_t, int) { return v; }

// mode 0 (operator apply):  out = cg * L(us)
// mode 1 (SSP-RK3 stage):    out = base + cb * (us - base) + cg * L(us),
//                            base = ub when given, else us.
// L(us)_K = S_{o,mask}(us_K - c) + sum_{f in mask} N_{o,f}(us_f - c),
// c = us_K[node 0] (exact zero on constants whatever the rounding of S, N).
// Writing the stage as a correction of `base` keeps the weight of the base
// state exactly 1 (in FP32, fl(1/3) + fl(2/3) = 1 + 3e-8, which the textbook
// form 1/3 u + 2/3 u2 would turn into a mass growth of 3e-8 per step).
//
// TS is the storage type of the state (float or double); all element
// arithmetic runs in FP64 with FP64 matrices.  FP32 accumulation of the
// matrix products leaves a systematic mass drift that grows over the 10^5 -
// 10^6 steps of a solve; with packed FP32 off, gfx950 issues FP64 and FP32
// FMAs at the same rate, so the FP64 arithmetic costs no VALU throughput
// and the HBM traffic is that of the FP32 state.
//
// mode 2 (Chebyshev recurrence of exp(t L), see launch_cheb):
//   out = 2 (us + cg L(us)) - ub,  res += ck * out
// (res loaded with the other loads; out and res stored non-temporally).
// MODE is the runtime mode fixed at compile time.  With SPLIT the presence
// of the base state (BASE) and of absorbing box blocks (ABS) is fixed too;
// without it both are tested at run time.  Which instantiation is faster
// depends on the register allocation: P3 gains from SPLIT, P1 and P2 lose
// (measured on gfx950), so the launcher splits for np = 10 only.  P3 with
// an FP32 state is held to 96 VGPRs (five waves per SIMD instead of four;
// no spills).
template <typename TS, int NP, int MODE, bool SPLIT, bool BASE, bool ABS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NP == 10 && sizeof(TS) == 4 ? 5 : 1))) k_stage(const TS* __restrict__ us, const TS* ub, TS* out,
                                               const int4* __restrict__ elem, int64_t E,
                                               const double* __restrict__ S,
                                               const double* __restrict__ Nm, int mode, double cb,
                                               double cg, int R, int epw, int64_t nblocks,
                                               int remap, const uint32_t* step, int stage_id,
                                               const double* __restrict__ Bm, TS* res = nullptr,
                                               double ck = 0.0) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  // right-hand sides: 64 per wave, chunk blockIdx.y; lanes past R load a
  // valid column and skip the store
  const int r_raw = blockIdx.y * WAVE + lane;
  const bool live = r_raw < R;
  const int r = live ? r_raw : R - 1;
  // the lane's byte offset within a node row, and the bytes per node row
  const uint32_t voff = (uint32_t)r * (uint32_t)sizeof(TS);
  const uint32_t row = (uint32_t)R * (uint32_t)sizeof(TS);
  const int64_t elen = (int64_t)NP * R;     // values per element
  const bool use_base = SPLIT ? BASE : ub != nullptr;
  const bool absorb = SPLIT ? ABS : Bm != nullptr;
  const uint32_t smix = MODE == 1 ? step_mix(step, stage_id) : 0u;
  const uint32_t hrhs = rhs_salt(r);
  const BlockIter it = block_iter(nblocks, remap);
  for (int64_t b = it.first; b < it.end; b += it.stride) {
    const int64_t e0 = (b * (blockDim.x / WAVE) + w) * (int64_t)epw;
    const int64_t e1 = e0 + epw < E ? e0 + epw : E;
    for (int64_t e = e0; e < e1; ++e) {
      const int4 m = elem[e];
      const int o = m.w & 1;
      const int mask = (m.w >> 1) & 7;
      // issue every load of the element first: own nodes, the three
      // neighbours (a missing neighbour reads the element itself, a cache
      // hit, and its product is skipped below), the RK base state
      const TS* pe = us + e * elen;
      const __amdgpu_buffer_rsrc_t ru = rows_at(pe);
      const __amdgpu_buffer_rsrc_t r0 = rows_at(m.x >= 0 ? us + (int64_t)m.x * elen : pe);
      const __amdgpu_buffer_rsrc_t r1 = rows_at(m.y >= 0 ? us + (int64_t)m.y * elen : pe);
      const __amdgpu_buffer_rsrc_t r2 = rows_at(m.z >= 0 ? us + (int64_t)m.z * elen : pe);
      TS su[NP], s0[NP], s1[NP], s2[NP], sb[NP];
#pragma unroll
      for (int j = 0; j < NP; ++j) {
        su[j] = ld_row<TS>(ru, voff, j * row);
        s0[j] = ld_row<TS>(r0, voff, j * row);
        s1[j] = ld_row<TS>(r1, voff, j * row);
        s2[j] = ld_row<TS>(r2, voff, j * row);
      }
      if (use_base) {
        const __amdgpu_buffer_rsrc_t rb = rows_at(ub + e * elen);
#pragma unroll
        for (int j = 0; j < NP; ++j) sb[j] = ld_row<TS, DGD_CPOL_BASE>(rb, voff, j * row);
      }
      TS sr[NP];
      if constexpr (MODE == 2) {
        const __amdgpu_buffer_rsrc_t rr = rows_at(res + e * elen);
#pragma unroll
        for (int j = 0; j < NP; ++j) sr[j] = ld_row<TS, DGD_CPOL_BASE>(rr, voff, j * row);
      }
      const double c = (double)su[0];
      double acc[NP];
      {
        const double* Se = S + (o * 8 + mask) * NP * NP;
        double d[NP];
        d[0] = 0.0;
#pragma unroll
        for (int j = 1; j < NP; ++j) d[j] = (double)su[j] - c;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          double a = 0.0;
#pragma unroll
          for (int j = 1; j < NP; ++j) a = fma(Se[i * NP + j], d[j], a);
          acc[i] = a;
        }
      }
#define DGD_FACE(F, SV)                                                                   \
      if (mask & (1 << F)) {                                                              \
        const double* Nf = Nm + (o * 3 + F) * NP * NP;                                    \
        double dn[NP];                                                                    \
        _Pragma("unroll") for (int j = 0; j < NP; ++j) dn[j] = (double)SV[j] - c;         \
        _Pragma("unroll") for (int i = 0; i < NP; ++i) {                                  \
          double a = acc[i];                                                              \
          _Pragma("unroll") for (int j = 0; j < NP; ++j) a = fma(Nf[i * NP + j], dn[j], a); \
          acc[i] = a;                                                                     \
        }                                                                                 \
      }
      DGD_FACE(0, s0)
      DGD_FACE(1, s1)
      DGD_FACE(2, s2)
#undef DGD_FACE
      // faces on the absorbing box (neighbour code -2; faces 0 and 1 only):
      // the outside value is zero, so the term acts on u itself
      if (absorb && (m.x == -2 || m.y == -2)) {
#pragma unroll
        for (int f = 0; f < 2; ++f) {
          if ((f == 0 ? m.x : m.y) != -2) continue;
          const double* Bf = Bm + (o * 3 + f) * NP * NP;
#pragma unroll
          for (int i = 0; i < NP; ++i) {
            double a = acc[i];
#pragma unroll
            for (int j = 0; j < NP; ++j) a = fma(Bf[i * NP + j], (double)su[j], a);
            acc[i] = a;
          }
        }
      }
      if (!live) continue;
      const __amdgpu_buffer_rsrc_t ro = rows_at(out + e * elen);
      if constexpr (MODE == 0) {
#pragma unroll
        for (int i = 0; i < NP; ++i) st_row(ro, voff, i * row, (TS)(cg * acc[i]));
      } else if constexpr (MODE == 2) {
        const __amdgpu_buffer_rsrc_t rr = rows_at(res + e * elen);
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          const double t = 2.0 * ((double)su[i] + cg * acc[i]) - (double)sb[i];
          st_row<DGD_CPOL_OUT>(ro, voff, i * row, (TS)t);
          st_row<DGD_CPOL_OUT>(rr, voff, i * row, (TS)((double)sr[i] + ck * t));
        }
      } else {
        const uint32_t hsr = elem_salt(m.w, smix) ^ hrhs;
        if (use_base) {
#pragma unroll
          for (int i = 0; i < NP; ++i) {
            const double b0 = (double)sb[i];
            st_row<DGD_CPOL_OUT>(ro, voff, i * row,
                   to_state((TS*)nullptr, b0 + cb * ((double)su[i] - b0) + cg * acc[i], hsr, i));
          }
        } else {
#pragma unroll
          for (int i = 0; i < NP; ++i)
            st_row<DGD_CPOL_OUT>(ro, voff, i * row,
                   to_state((TS*)nullptr, (double)su[i] + cg * acc[i], hsr, i));
        }
      }
    }
  }
}

// The paper's mixed form (eq. (6)-(7), fluxes of section 3.2) on all
// pixels, as two passes per stage.
//
// Pass 1 (k_mixed_grad): per element K and right-hand side r, the scaled
// gradient qh = h q = MG_{o,mask}(u_K - c) + sum_{f in mask} MN_{o,f}(u_f - c)
// for both components (c = u_K[node 0]: G annihilates constants, so a
// constant field gives exactly q = 0).  mask: faces with a neighbour element
// (axon cells included: the central u-flux reads their value).  MN is the
// compacted neighbour block: a nodal basis function of a node off the
// shared face vanishes on it, so a neighbour enters through its p + 1 face
// nodes (columns MNcol) only.  Stored in
// the state type, round to nearest, layout [E][2][NP][R].
//
// Pass 2 (k_mixed_div): u_t = (D / h^2) (MD_{o,fm} qh_K + sum_{f in fm}
// MN_{o,f} qh_f) on extracellular elements, zero on axon elements (k = 0).
// u is zero in axon cells and stays so: both passes skip axon elements
// (the stage buffers are cleared once when a run is created), except that
// the operator apply (mode 0) writes their zero derivative;
// fm: faces whose both sides are extracellular (the harmonic mean of k is
// zero otherwise).  meta[e] = fm | extracellular << 3.  The stage combine and
// the stochastic rounding of FP32 stores are those of k_stage (modes 0, 1).
// The P3 FP32 divergence pass is held to 128 VGPRs (four waves per SIMD
// instead of three; no spills).
template <typename TS, int NP>
__global__ void __launch_bounds__(256) k_mixed_grad(const TS* __restrict__ us, TS* __restrict__ qout,
                                                    const int4* __restrict__ elem,
                                                    const uint8_t* __restrict__ meta, int64_t E,
                                                    const double* __restrict__ MG,
                                                    const double* __restrict__ MN,
                                                    const int* __restrict__ MNcol, int R, int epw,
                                                    int64_t nblocks, int remap) {
  constexpr int NF = NP == 3 ? 2 : (NP == 6 ? 3 : 4);    // nodes on a face (p + 1)
  const int lane = threadIdx.x & (WAVE - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const int r_raw = blockIdx.y * WAVE + lane;
  const bool live = r_raw < R;
  const int r = live ? r_raw : R - 1;
  // state rows through buffer resources, as in k_stage
  const uint32_t voff = (uint32_t)r * (uint32_t)sizeof(TS);
  const uint32_t row = (uint32_t)R * (uint32_t)sizeof(TS);
  const int64_t elen = (int64_t)NP * R;
  const BlockIter it = block_iter(nblocks, remap);
  for (int64_t b = it.first; b < it.end; b += it.stride) {
    const int64_t e0 = (b * (blockDim.x / WAVE) + w) * (int64_t)epw;
    const int64_t e1 = e0 + epw < E ? e0 + epw : E;
    for (int64_t e = e0; e < e1; ++e) {
      // q of an axon element is never read (its q-flux faces are all off)
      if (!((meta[e] >> 3) & 1)) continue;
      const int4 m = elem[e];
      const int o = m.w & 1;
      const int mask = (m.w >> 1) & 7;
      const TS* pe = us + e * elen;
      const __amdgpu_buffer_rsrc_t ru = rows_at(pe);
      const __amdgpu_buffer_rsrc_t r0 = rows_at(m.x >= 0 ? us + (int64_t)m.x * elen : pe);
      const __amdgpu_buffer_rsrc_t r1 = rows_at(m.y >= 0 ? us + (int64_t)m.y * elen : pe);
      const __amdgpu_buffer_rsrc_t r2 = rows_at(m.z >= 0 ? us + (int64_t)m.z * elen : pe);
      // a neighbour enters only through its nodes on the shared face
      const int* c0 = MNcol + (o * 3 + 0) * NF;
      const int* c1 = MNcol + (o * 3 + 1) * NF;
      const int* c2 = MNcol + (o * 3 + 2) * NF;
      TS su[NP], s0[NF], s1[NF], s2[NF];
#pragma unroll
      for (int j = 0; j < NP; ++j) su[j] = ld_row<TS>(ru, voff, j * row);
#pragma unroll
      for (int k = 0; k < NF; ++k) {
        s0[k] = ld_row<TS>(r0, voff, (uint32_t)c0[k] * row);
        s1[k] = ld_row<TS>(r1, voff, (uint32_t)c1[k] * row);
        s2[k] = ld_row<TS>(r2, voff, (uint32_t)c2[k] * row);
      }
      const double c = (double)su[0];
      double d[NP];
      d[0] = 0.0;
#pragma unroll
      for (int j = 1; j < NP; ++j) d[j] = (double)su[j] - c;
      double ax[NP], ay[NP];
      {
        const double* Gx = MG + ((o * 8 + mask) * 2 + 0) * NP * NP;
        const double* Gy = MG + ((o * 8 + mask) * 2 + 1) * NP * NP;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          double a = 0.0, bb = 0.0;
#pragma unroll
          for (int j = 1; j < NP; ++j) {
            a = fma(Gx[i * NP + j], d[j], a);
            bb = fma(Gy[i * NP + j], d[j], bb);
          }
          ax[i] = a;
          ay[i] = bb;
        }
      }
#define DGD_MFACE(F, SV)                                                                    \
      if (mask & (1 << F)) {                                                                \
        const double* Nx = MN + ((o * 3 + F) * 2 + 0) * NP * NF;                            \
        const double* Ny = MN + ((o * 3 + F) * 2 + 1) * NP * NF;                            \
        double dn[NF];                                                                      \
        _Pragma("unroll") for (int k = 0; k < NF; ++k) dn[k] = (double)SV[k] - c;           \
        _Pragma("unroll") for (int i = 0; i < NP; ++i) {                                    \
          double a = ax[i], bb = ay[i];                                                     \
          _Pragma("unroll") for (int k = 0; k < NF; ++k) {                                  \
            a = fma(Nx[i * NF + k], dn[k], a);                                              \
            bb = fma(Ny[i * NF + k], dn[k], bb);                                            \
          }                                                                                 \
          ax[i] = a;                                                                        \
          ay[i] = bb;                                                                       \
        }                                                                                   \
      }
      DGD_MFACE(0, s0)
      DGD_MFACE(1, s1)
      DGD_MFACE(2, s2)
#undef DGD_MFACE
      if (!live) continue;
      const __amdgpu_buffer_rsrc_t rq = rows_at(qout + 2 * e * elen);
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        st_row<DGD_CPOL_OUT>(rq, voff, i * row, (TS)ax[i]);
        st_row<DGD_CPOL_OUT>(rq, voff, (NP + i) * row, (TS)ay[i]);
      }
    }
  }
}

template <typename TS, int NP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(TS) == 4 && NP == 10 ? 4 : 1)))
k_mixed_div(const TS* __restrict__ q, const TS* __restrict__ us,
                                                   const TS* ub, TS* out,
                                                   const int4* __restrict__ elem,
                                                   const uint8_t* __restrict__ meta, int64_t E,
                                                   const double* __restrict__ MD,
                                                   const double* __restrict__ MN,
                                                   const int* __restrict__ MNcol, int mode,
                                                   double cb, double cg, int R, int epw,
                                                   int64_t nblocks, int remap,
                                                   const uint32_t* step, int stage_id) {
  constexpr int NF = NP == 3 ? 2 : (NP == 6 ? 3 : 4);
  const int lane = threadIdx.x & (WAVE - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const int r_raw = blockIdx.y * WAVE + lane;
  const bool live = r_raw < R;
  const int r = live ? r_raw : R - 1;
  const uint32_t voff = (uint32_t)r * (uint32_t)sizeof(TS);
  const uint32_t row = (uint32_t)R * (uint32_t)sizeof(TS);
  const int64_t elen = (int64_t)NP * R;
  const bool use_base = ub != nullptr;
  const uint32_t smix = step_mix(step, stage_id);
  const BlockIter it = block_iter(nblocks, remap);
  for (int64_t b = it.first; b < it.end; b += it.stride) {
    const int64_t e0 = (b * (blockDim.x / WAVE) + w) * (int64_t)epw;
    const int64_t e1 = e0 + epw < E ? e0 + epw : E;
    for (int64_t e = e0; e < e1; ++e) {
      const int4 m = elem[e];
      const int o = m.w & 1;
      const int mt = meta[e];
      const int fm = mt & 7;
      const bool ext = (mt >> 3) & 1;
      const __amdgpu_buffer_rsrc_t ro = rows_at(out + e * elen);
      // axon element: u stays zero (k = 0, no q-flux); only the operator
      // apply (mode 0) writes its zero derivative
      if (!ext) {
        if (mode == 0 && live) {
#pragma unroll
          for (int i = 0; i < NP; ++i) st_row(ro, voff, i * row, (TS)0);
        }
        continue;
      }
      // every load first: own q, the neighbours' q on the shared faces,
      // the stage input and the RK base
      const __amdgpu_buffer_rsrc_t rq = rows_at(q + 2 * e * elen);
      TS qx[NP], qy[NP], su[NP], sb[NP];
#pragma unroll
      for (int j = 0; j < NP; ++j) {
        qx[j] = ld_row<TS>(rq, voff, j * row);
        qy[j] = ld_row<TS>(rq, voff, (NP + j) * row);
      }
      TS fx[3][NF], fy[3][NF];
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        const int nb = f == 0 ? m.x : (f == 1 ? m.y : m.z);
        // a face off the q-flux reads the element's own rows (unused)
        const __amdgpu_buffer_rsrc_t rn = rows_at(((fm >> f) & 1) ? q + 2 * (int64_t)nb * elen
                                                                   : q + 2 * e * elen);
        const int* cf = MNcol + (o * 3 + f) * NF;
#pragma unroll
        for (int k = 0; k < NF; ++k) {
          fx[f][k] = ld_row<TS>(rn, voff, (uint32_t)cf[k] * row);
          fy[f][k] = ld_row<TS>(rn, voff, (uint32_t)(NP + cf[k]) * row);
        }
      }
      if (mode != 0) {
        const __amdgpu_buffer_rsrc_t ru = rows_at(us + e * elen);
#pragma unroll
        for (int j = 0; j < NP; ++j) su[j] = ld_row<TS>(ru, voff, j * row);
        if (use_base) {
          const __amdgpu_buffer_rsrc_t rb = rows_at(ub + e * elen);
#pragma unroll
          for (int j = 0; j < NP; ++j) sb[j] = ld_row<TS, DGD_CPOL_BASE>(rb, voff, j * row);
        }
      }
      double acc[NP];
      {
        const double* Dx = MD + ((o * 8 + fm) * 2 + 0) * NP * NP;
        const double* Dy = MD + ((o * 8 + fm) * 2 + 1) * NP * NP;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          double a = 0.0;
#pragma unroll
          for (int j = 0; j < NP; ++j)
            a = fma(Dx[i * NP + j], (double)qx[j], fma(Dy[i * NP + j], (double)qy[j], a));
          acc[i] = a;
        }
      }
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        if (!((fm >> f) & 1)) continue;
        const double* Nx = MN + ((o * 3 + f) * 2 + 0) * NP * NF;
        const double* Ny = MN + ((o * 3 + f) * 2 + 1) * NP * NF;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          double a = acc[i];
#pragma unroll
          for (int k = 0; k < NF; ++k)
            a = fma(Nx[i * NF + k], (double)fx[f][k], fma(Ny[i * NF + k], (double)fy[f][k], a));
          acc[i] = a;
        }
      }
      if (!live) continue;
      const uint32_t hsr = state_salt(m.w, r, smix);
      if (mode == 0) {
#pragma unroll
        for (int i = 0; i < NP; ++i) st_row(ro, voff, i * row, (TS)(cg * acc[i]));
      } else if (use_base) {
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          const double u = (double)su[i], b0 = (double)sb[i];
          st_row<DGD_CPOL_OUT>(ro, voff, i * row,
                               to_state((TS*)nullptr, b0 + cb * (u - b0) + cg * acc[i], hsr, i));
        }
      } else {
#pragma unroll
        for (int i = 0; i < NP; ++i)
          st_row<DGD_CPOL_OUT>(ro, voff, i * row,
                               to_state((TS*)nullptr, (double)su[i] + cg * acc[i], hsr, i));
      }
    }
  }
}

// P3 stage on matrix cores (FP32 state, R a multiple of 16).  For element K
// of class (o, mask) the contraction over the stacked stencil
//   L(u)_K = [S_{o,mask} | N_{o,0} | N_{o,1} | N_{o,2}] (u_stencil - c)
// (rows 10..15 of the stacked matrix A are zero; a missing face has zero
// columns) is a (16 x 40) x (40 x 16) product per block of 16 right-hand
// sides, in one of two forms:
//  * FP32 (BF false): ten v_mfma_f32_16x16x4_f32 steps (K = 40 = 10 x 4
//    exactly).  Lane l of step s holds A[m = l % 16][k = 4 s + l / 16] and
//    B[k = 4 s + l / 16][n = l % 16].
//  * BF16 hi/lo split (BF true): two v_mfma_f32_16x16x32_bf16 steps h, each
//    over 20 stencil rows padded to 32: lane l of step h holds eight values,
//    slot j < 5 of stencil row k = 20 h + 5 (l / 16) + j and slots 5..7 zero,
//    for row m = l % 16 of A and column n = l % 16 of B (the operand layout
//    only has to give a lane's slot j the same k in A and in B, which the
//    instruction does).  A is split on the host into A_hi + A_mid + A_lo,
//    all BF16 (24 significant bits together); each value x = u - c is split
//    here into x_hi = bf16(x) and x_lo = bf16(x - x_hi) (error below
//    2^-17 |x|), and the step accumulates
//    A_lo x_hi + A_mid x_hi + A_hi x_lo + A_hi x_hi in FP32.  What is left
//    out (A_mid x_lo, A_lo x_lo, the rounding of x_lo) depends on the
//    rounding residues of the state, which vary from element to element;
//    the operator's own remainder would not: a fixed relative error e in
//    the stencil breaks its consistency on linear fields, a source of
//    relative size e l / h on a field varying over a length l, so A keeps
//    its third term (with two, e = 2^-18 moved Sigma by ~5e-5).  Eight
//    matrix instructions per block of 16 right-hand sides instead of ten
//    at twice the cost each.
// Either way lane l receives D[m = 4 (l / 16) + i][n = l % 16], i < 4.
//
// A wave covers 64 right-hand sides of an element (blockIdx.y selects which
// 64).  Lane (q, n) = (l / 16, l % 16) loads the four consecutive columns
// 4n .. 4n+3 of each of its ten stencil rows as one 16-byte load, so the
// wave's loads are whole 256-byte rows; the four 16-column blocks are
// t = 0..3 with block t holding columns {4n + t}: the t-th component of
// every lane's load is exactly that block's B operand, and the four blocks'
// results for a row are again four consecutive columns, stored as one
// 16-byte store.
//
// Rounded products lose mass systematically over 10^6 steps, so each
// column's result is corrected by a constant so that its mass w^T L(u)
// equals the FP64 sum of the face fluxes, Phi = C_{o,mask} . u_stencil, with
// the flux coefficients C = w^T [S | N...] (w = reference mass-matrix row
// sums).  Atab (FP32): [16 classes][10 steps][64 lanes] float; (BF16):
// [16 classes][2 steps][hi, mid, lo][64 lanes][8] bf16; Ctab: [16][40] double;
// Wtab: [2][16] double (row weights, zero beyond 10); inv_wsum = 1 / sum w.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));

// two FP32 values rounded to nearest-even BF16, packed (a in the low half)
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
  const f32x2_t v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}

// BF16 hi/lo operands of five values x[0..4] (slots 5..7 zero): x_hi is x
// rounded to BF16 and x_lo the rounded remainder x - x_hi, which FP32 holds
// exactly.
__device__ __forceinline__ void split_bf16x5(const float (&x)[5], bf16x8_t* hi, bf16x8_t* lo) {
  const uint32_t h01 = pack_bf16(x[0], x[1]), h23 = pack_bf16(x[2], x[3]),
                 h4 = pack_bf16(x[4], 0.f);
  const float r0 = x[0] - __uint_as_float(h01 << 16);
  const float r1 = x[1] - __uint_as_float(h01 & 0xffff0000u);
  const float r2 = x[2] - __uint_as_float(h23 << 16);
  const float r3 = x[3] - __uint_as_float(h23 & 0xffff0000u);
  const float r4 = x[4] - __uint_as_float(h4 << 16);
  typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
  const u32x4_t vh = {h01, h23, h4, 0u};
  const u32x4_t vl = {pack_bf16(r0, r1), pack_bf16(r2, r3), pack_bf16(r4, 0.f), 0u};
  *hi = __builtin_bit_cast(bf16x8_t, vh);
  *lo = __builtin_bit_cast(bf16x8_t, vl);
}

template <bool BF>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_stage_p3_mfma(const float* __restrict__ us, const float* ub,
                                                       float* out, const int4* __restrict__ elem,
                                                       int64_t E, const void* __restrict__ Atab,
                                                       const double* __restrict__ Ctab,
                                                       const double* __restrict__ Wtab,
                                                       double inv_wsum, int mode, double cb,
                                                       double cg, int R, int epw, int64_t nblocks,
                                                       int remap, const uint32_t* step,
                                                       int stage_id) {
  typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
  const int lane = threadIdx.x & (WAVE - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const int q = lane >> 4, n = lane & 15;
  const bool use_base = ub != nullptr;
  // this lane's four columns; R % 16 == 0, so they are all in range or all
  // out (then a valid column is read and nothing is stored)
  const int c_raw = blockIdx.y * WAVE + 4 * n;
  const bool col_live = c_raw < R;
  const uint32_t col = (uint32_t)(col_live ? c_raw : 0);
  const uint32_t smix = step_mix(step, stage_id);
  const BlockIter it = block_iter(nblocks, remap);
  for (int64_t b = it.first; b < it.end; b += it.stride) {
    const int64_t e0 = (b * (blockDim.x / WAVE) + w) * (int64_t)epw;
    const int64_t e1 = e0 + epw < E ? e0 + epw : E;
    for (int64_t e = e0; e < e1; ++e) {
      const int4 m = elem[e];
      const int o = m.w & 1;
      const int mask = (m.w >> 1) & 7;
      const int cls = o * 8 + mask;
      const uint32_t self = (uint32_t)e * 10u * (uint32_t)R;
      // every load first: pivot row, the ten operand rows of this lane (the
      // host guarantees E * 10 * R < 2^31), the own rows this lane writes
      // (u and base), the class's operator entries
      f32x4 cpv = *(const f32x4*)(us + self + col);
      f32x4 v[10];
      double cf[10];
#pragma unroll
      for (int s = 0; s < 10; ++s) {
        const int k = BF ? 20 * (s / 5) + 5 * q + s % 5 : 4 * s + q;
        const int blk = k / 10, j = k % 10;
        int eb = (int)e;
        if (blk == 1 && m.x >= 0) eb = m.x;
        if (blk == 2 && m.y >= 0) eb = m.y;
        if (blk == 3 && m.z >= 0) eb = m.z;
        v[s] = *(const f32x4*)(us + ((uint32_t)eb * 10u + (uint32_t)j) * (uint32_t)R + col);
        cf[s] = Ctab[cls * 40 + k];
      }
      float a[10];
      if constexpr (!BF) {
#pragma unroll
        for (int s = 0; s < 10; ++s) a[s] = ((const float*)Atab)[(cls * 10 + s) * WAVE + lane];
      }
      // After the products lane (q, n) holds rows 4q .. 4q+3 of its four
      // columns: 16 values, of which 16, 16, 8 and 0 are real rows (< 10)
      // for q = 0..3.  The combine and rounding are rebalanced to ten values
      // per lane, three row pieces each: lanes q = 3 take rows 3 and 7 and
      // row 2's last two columns, lanes q = 2 row 6's last two columns
      // (cross-lane moves by 32 and 48 lanes; n is kept):
      //   q   piece A (4 cols)  piece B (4 cols)  piece C (2 cols from tC)
      //   0   row 0             row 1             row 2, tC = 0
      //   1   row 4             row 5             row 6, tC = 0
      //   2   row 8             row 9             row 6, tC = 2
      //   3   row 3             row 7             row 2, tC = 2
      const int rA = q == 3 ? 3 : 4 * q, rB = q == 3 ? 7 : 4 * q + 1;
      const int rC = (q == 0 || q == 3) ? 2 : 6, tC = q < 2 ? 0 : 2;
      const uint32_t iA = self + (uint32_t)rA * (uint32_t)R + col;
      const uint32_t iB = self + (uint32_t)rB * (uint32_t)R + col;
      const uint32_t iC = self + (uint32_t)rC * (uint32_t)R + col + (uint32_t)tC;
      f32x4 uA, uB, bA, bB;
      f32x2_t uC, bC;
      if (mode != 0) {
        uA = *(const f32x4*)(us + iA);
        uB = *(const f32x4*)(us + iB);
        uC = *(const f32x2_t*)(us + iC);
        bA = use_base ? *(const f32x4*)(ub + iA) : uA;
        bB = use_base ? *(const f32x4*)(ub + iB) : uB;
        bC = use_base ? *(const f32x2_t*)(ub + iC) : uC;
      }
      double wr[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) wr[i] = Wtab[o * 16 + 4 * q + i];
      f32x4 acc[4];
      double alpha[4];
      if constexpr (BF) {
        // step h outermost, so only one step's three operator terms are live
        const bf16x8_t* At = (const bf16x8_t*)Atab;
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const bf16x8_t ahi = At[((cls * 2 + h) * 3 + 0) * WAVE + lane];
          const bf16x8_t amid = At[((cls * 2 + h) * 3 + 1) * WAVE + lane];
          const bf16x8_t alo = At[((cls * 2 + h) * 3 + 2) * WAVE + lane];
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            float x[5];
#pragma unroll
            for (int j = 0; j < 5; ++j) x[j] = v[5 * h + j][t] - cpv[t];
            bf16x8_t xh, xl;
            split_bf16x5(x, &xh, &xl);
            f32x4 d = acc[t];
            d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, xh, d, 0, 0, 0);
            d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(amid, xh, d, 0, 0, 0);
            d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, xl, d, 0, 0, 0);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, xh, d, 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        double phi = 0.0;
        f32x4 d = acc[t];
        if constexpr (BF) {
#pragma unroll
          for (int s = 0; s < 10; ++s) phi = fma(cf[s], (double)v[s][t], phi);
        } else {
          d = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int s = 0; s < 10; ++s) {
            d = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], v[s][t] - cpv[t], d, 0, 0, 0);
            phi = fma(cf[s], (double)v[s][t], phi);
          }
        }
        double dl = phi;
#pragma unroll
        for (int i = 0; i < 4; ++i) dl = fma(-wr[i], (double)d[i], dl);
        dl += __shfl_xor(dl, 16);
        dl += __shfl_xor(dl, 32);
        acc[t] = d;
        alpha[t] = dl * inv_wsum;
      }
      // the moves (every lane takes part; only q = 2, 3 keep what arrives)
      f32x4 vA, vB;
      f32x2_t vC;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float m48 = __shfl_xor(acc[t][3], 48), m32 = __shfl_xor(acc[t][3], 32);
        vA[t] = q == 3 ? m48 : acc[t][0];
        vB[t] = q == 3 ? m32 : acc[t][1];
      }
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const float m48 = __shfl_xor(acc[2 + k][2], 48);
        vC[k] = q < 2 ? acc[k][2] : m48;
      }
      if (!col_live) continue;
      auto finish = [&](float a_val, int t, int row, float uu, float bb) -> float {
        const double val = (double)a_val + alpha[t];
        if (mode == 0) return (float)(cg * val);
        const double u = (double)uu, b0 = (double)bb;
        return round_stochastic(b0 + cb * (u - b0) + cg * val,
                                sr_node(state_salt(m.w, (int)col + t, smix), row));
      };
      f32x4 oA, oB;
      f32x2_t oC;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        oA[t] = finish(vA[t], t, rA, mode != 0 ? uA[t] : 0.f, mode != 0 ? bA[t] : 0.f);
        oB[t] = finish(vB[t], t, rB, mode != 0 ? uB[t] : 0.f, mode != 0 ? bB[t] : 0.f);
      }
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const double al = tC == 0 ? alpha[k] : alpha[2 + k];
        const double val = (double)vC[k] + al;
        if (mode == 0) {
          oC[k] = (float)(cg * val);
        } else {
          const double u = (double)uC[k], b0 = (double)bC[k];
          oC[k] = round_stochastic(b0 + cb * (u - b0) + cg * val,
                                   sr_node(state_salt(m.w, (int)col + tC + k, smix), rC));
        }
      }
      *(f32x4*)(out + iA) = oA;
      *(f32x4*)(out + iB) = oB;
      *(f32x2_t*)(out + iC) = oC;
    }
  }
}

// Packed stage for few right-hand sides (R <= 64 / G): each wave carries G
// elements side by side, lane l on element (group base + l / (64 / G)) and
// right-hand side l % (64 / G), so no lane idles when R = 16 (G = 4) or
// R = 32 (G = 2).  Face masks then differ across the wave, so the operator
// is used in the split form
//   S_{o,mask} = S_{o,7} - sum_{f not in mask} F_{o,f},
// F_{o,f} = -M^-1 (self-face block of face f): every matrix stays
// wave-uniform (SGPR operands) given the orientation.  Per face, a lane
// accumulates N_{o,f}(u_f - c) if it has the face and -F_{o,f}(u - c) if
// not, by zeroing the other product's vector: a product with an exact zero
// vector leaves the accumulator unchanged (it never holds -0), so a lane
// computes the same bits whatever the masks of the other elements of its
// wave.  A face's N product runs only if some lane's element has the face
// and its F product only if some lane's element lacks it: runs stepped on
// class-sorted element tables (one face mask per wave) do one of the two
// per face, like a single element.  Waves whose elements mix the
// two orientations (rare: meshes are ordered in orientation groups of four)
// run once per orientation under a lane mask.  Modes and combine as in
// k_stage (0 apply, 1 SSP-RK3 stage).  ABS: the operator has absorbing box
// blocks (Bm non-NULL); without them the box code is not compiled in.
template <typename TS, int NP, int G, bool ABS, int MODE>
__global__ void __launch_bounds__(256) k_stage_packed(const TS* __restrict__ us, const TS* ub,
                                                      TS* out, const int4* __restrict__ elem,
                                                      int64_t E, const double* __restrict__ S,
                                                      const double* __restrict__ Fm,
                                                      const double* __restrict__ Nm, int mode,
                                                      double cb, double cg, int R, int epw,
                                                      int64_t nblocks, int remap,
                                                      const uint32_t* step, int stage_id,
                                                      const double* __restrict__ Bm) {
  constexpr int RL = WAVE / G;
  const int lane = threadIdx.x & (WAVE - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const int g = lane / RL;
  const int r_raw = lane % RL;
  const bool live_r = r_raw < R;
  const int r = live_r ? r_raw : R - 1;
  const bool use_base = ub != nullptr;
  const uint32_t smix = MODE == 1 ? step_mix(step, stage_id) : 0u;
  const BlockIter it = block_iter(nblocks, remap);
  for (int64_t b = it.first; b < it.end; b += it.stride) {
    const int64_t q0 = (b * (blockDim.x / WAVE) + w) * (int64_t)epw;
    for (int k = 0; k < epw; ++k) {
      const int64_t eg = (q0 + k) * G;          // first element of the group
      if (eg >= E) break;
      const int64_t e_raw = eg + g;
      const bool live = live_r && e_raw < E;
      const int64_t e = e_raw < E ? e_raw : E - 1;
      const int4 m = elem[e];
      const int o = m.w & 1;
      const int mask = (m.w >> 1) & 7;
      // wave-uniform facts: orientation of lane 0, whether any lane differs,
      // whether any element misses a face
      const int o0 = __builtin_amdgcn_readfirstlane(o);
      const bool mixed = __ballot(o != o0) != 0;
      // per face: whether some lane's element has it, and whether some
      // lane's lacks it (from P2 up; with class-sorted element tables a wave
      // holds one face mask, so only one of the two products below runs per
      // face).  At P1 the products are cheap and the plain test is faster:
      // N products always, F products when any element misses a face.
      constexpr bool PER_FACE = NP > 3;
      const bool partial = __ballot(mask != 7) != 0;
      bool has_any[3], lacks_any[3];
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        has_any[f] = PER_FACE ? __ballot((mask >> f) & 1) != 0 : true;
        lacks_any[f] = PER_FACE ? __ballot(!((mask >> f) & 1)) != 0 : partial;
      }
      const bool box0 = ABS && m.x == -2, box1 = ABS && m.y == -2;
      const bool any_box = ABS && __ballot(box0 || box1) != 0;
      // one element and right-hand side per lane with orientation oo (uniform)
      auto body = [&](const int oo) {
        const int64_t self = (e * NP) * (int64_t)R + r;
        const int64_t n0 = (m.x >= 0 ? (int64_t)m.x * NP * R + r : self);
        const int64_t n1 = (m.y >= 0 ? (int64_t)m.y * NP * R + r : self);
        const int64_t n2 = (m.z >= 0 ? (int64_t)m.z * NP * R + r : self);
        TS su[NP], s0[NP], s1[NP], s2[NP], sb[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) {
          su[j] = us[self + (int64_t)j * R];
          s0[j] = us[n0 + (int64_t)j * R];
          s1[j] = us[n1 + (int64_t)j * R];
          s2[j] = us[n2 + (int64_t)j * R];
        }
        if (use_base) {
#pragma unroll
          for (int j = 0; j < NP; ++j) sb[j] = __builtin_nontemporal_load(ub + self + (int64_t)j * R);
        }
        const double c = (double)su[0];
        double d[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) d[j] = (double)su[j] - c;
        double acc[NP];
        {
          const double* Se = S + (oo * 8 + 7) * NP * NP;
#pragma unroll
          for (int i = 0; i < NP; ++i) {
            double a = 0.0;
#pragma unroll
            for (int j = 0; j < NP; ++j) a = fma(Se[i * NP + j], d[j], a);
            acc[i] = a;
          }
        }
#define DGD_PFACE(F, SV)                                                                     \
        {                                                                                    \
          const bool has = !partial || ((mask >> F) & 1);                                    \
          if (has_any[F]) {                                                                  \
            const double* Nf = Nm + (oo * 3 + F) * NP * NP;                                  \
            double dn[NP];                                                                   \
            _Pragma("unroll") for (int j = 0; j < NP; ++j)                                   \
              dn[j] = has ? (double)SV[j] - c : 0.0;                                         \
            _Pragma("unroll") for (int i = 0; i < NP; ++i) {                                 \
              double a = acc[i];                                                             \
              _Pragma("unroll") for (int j = 0; j < NP; ++j) a = fma(Nf[i * NP + j], dn[j], a); \
              acc[i] = a;                                                                    \
            }                                                                                \
          }                                                                                  \
          if (lacks_any[F]) {                                                                \
            const double* Ff = Fm + (oo * 3 + F) * NP * NP;                                  \
            double dm[NP];                                                                   \
            _Pragma("unroll") for (int j = 0; j < NP; ++j) dm[j] = has ? 0.0 : d[j];         \
            _Pragma("unroll") for (int i = 0; i < NP; ++i) {                                 \
              double a = acc[i];                                                             \
              _Pragma("unroll") for (int j = 0; j < NP; ++j) a = fma(-Ff[i * NP + j], dm[j], a); \
              acc[i] = a;                                                                    \
            }                                                                                \
          }                                                                                  \
        }
        DGD_PFACE(0, s0)
        DGD_PFACE(1, s1)
        DGD_PFACE(2, s2)
#undef DGD_PFACE
        // absorbing box faces: lanes without one multiply exact zeros
        if (any_box) {
#pragma unroll
          for (int f = 0; f < 2; ++f) {
            const bool on = f == 0 ? box0 : box1;
            const double* Bf = Bm + (oo * 3 + f) * NP * NP;
            double ub_[NP];
#pragma unroll
            for (int j = 0; j < NP; ++j) ub_[j] = on ? (double)su[j] : 0.0;
#pragma unroll
            for (int i = 0; i < NP; ++i) {
              double a = acc[i];
#pragma unroll
              for (int j = 0; j < NP; ++j) a = fma(Bf[i * NP + j], ub_[j], a);
              acc[i] = a;
            }
          }
        }
        if (!live) return;
        const uint32_t hsr = state_salt(m.w, r, smix);
        if constexpr (MODE == 0) {
#pragma unroll
          for (int i = 0; i < NP; ++i) out[self + (int64_t)i * R] = (TS)(cg * acc[i]);
        } else if (use_base) {
#pragma unroll
          for (int i = 0; i < NP; ++i) {
            const double b0 = (double)sb[i];
            store_state_nt(out, self + (int64_t)i * R, b0 + cb * ((double)su[i] - b0) + cg * acc[i],
                        hsr, i);
          }
        } else {
#pragma unroll
          for (int i = 0; i < NP; ++i)
            store_state_nt(out, self + (int64_t)i * R, (double)su[i] + cg * acc[i],
                        hsr, i);
        }
      };
      if (!mixed) {
        body(o0);
      } else if (o == 0) {
        body(0);
      } else {
        body(1);
      }
    }
  }
}

// Reduction kernels share one shape: 4 waves per workgroup, each wave walks
// `epw` consecutive elements, lanes on right-hand sides; per-block partials
// part[b][r][6] are summed later in a fixed order (deterministic).

// Partial moments with element-local offsets d = c_K - x0 in FP64 (c_K the
// cell centre from integer indices).  x0 is [G][R][2].
template <typename T, int NP>
__global__ void __launch_bounds__(256) k_moments(const T* __restrict__ u,
                                                 const int4* __restrict__ elem, int64_t E,
                                                 const double* __restrict__ W,
                                                 const double* __restrict__ x0,
                                                 const int* __restrict__ blk_geom, double h, int R,
                                                 int epw, int64_t nblocks,
                                                 double* __restrict__ part) {
  __shared__ double red[4][WAVE][6];
  const int lane = threadIdx.x & (WAVE - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const BlockIter it = block_iter(nblocks, 1);
  for (int64_t b = it.first; b < it.end; b += it.stride) {
    const int g = blk_geom ? blk_geom[b] : 0;
    const int64_t e0 = (b * (blockDim.x / WAVE) + w) * (int64_t)epw;
    const int64_t e1 = e0 + epw < E ? e0 + epw : E;
    for (int r0 = 0; r0 < R; r0 += WAVE) {
      const int r = r0 + lane;
      double a0 = 0, ax = 0, ay = 0, axx = 0, axy = 0, ayy = 0;
      if (r < R) {
        const double px = x0[((int64_t)g * R + r) * 2], py = x0[((int64_t)g * R + r) * 2 + 1];
        for (int64_t e = e0; e < e1; ++e) {
          const int4 m = elem[e];
          const int o = m.w & 1;
          const int ci = (m.w >> 4) & 0x3fff;
          const int cj = (m.w >> 18) & 0x3fff;
          const double* Wo = W + o * 6 * NP;
          double i0 = 0, ix = 0, iy = 0, ixx = 0, ixy = 0, iyy = 0;
          const int64_t base = (e * NP) * (int64_t)R + r;
#pragma unroll
          for (int j = 0; j < NP; ++j) {
            const double v = (double)u[base + (int64_t)j * R];
            i0 += Wo[0 * NP + j] * v;
            ix += Wo[1 * NP + j] * v;
            iy += Wo[2 * NP + j] * v;
            ixx += Wo[3 * NP + j] * v;
            ixy += Wo[4 * NP + j] * v;
            iyy += Wo[5 * NP + j] * v;
          }
          const double dx = (ci + 0.5) * h - px;
          const double dy = (cj + 0.5) * h - py;
          a0 += i0;
          ax += ix + dx * i0;
          ay += iy + dy * i0;
          axx += ixx + 2.0 * dx * ix + dx * dx * i0;
          axy += ixy + dx * iy + dy * ix + dx * dy * i0;
          ayy += iyy + 2.0 * dy * iy + dy * dy * i0;
        }
      }
      red[w][lane][0] = a0;
      red[w][lane][1] = ax;
      red[w][lane][2] = ay;
      red[w][lane][3] = axx;
      red[w][lane][4] = axy;
      red[w][lane][5] = ayy;
      __syncthreads();
      if (w == 0 && r < R) {
        for (int c = 0; c < 6; ++c) {
          double s = red[0][lane][c];
          for (int k = 1; k < (int)(blockDim.x / WAVE); ++k) s += red[k][lane][c];
          part[(b * R + r) * 6 + c] = s;
        }
      }
      __syncthreads();
    }
  }
}

// Partial q-space signal of the propagator (one geometry): for element K
// and right-hand side r,
//   exp(i q.(c_K - x0_r)) * sum_j Wq[q][o][j] u_K[j][r],
// Wq the element integrals of the nodal basis times exp(i q.(x - c_K))
// (c_K the cell centre, h^2 included), summed over the block's elements
// into part[b][r][q][2] = (re, im).  The phase is computed in FP64 from
// integer cell indices.  QC wave vectors per launch slice (blockIdx.z).
// Wq: [nq][2][NP][2]; qv: [nq][2]; x0: [R][2].
template <typename T, int NP, int QC>
__global__ void __launch_bounds__(256) k_signal(const T* __restrict__ u,
                                                const int4* __restrict__ elem, int64_t E,
                                                const double* __restrict__ Wq,
                                                const double* __restrict__ qv, int nq,
                                                const double* __restrict__ x0, double h, int R,
                                                int epw, int64_t nblocks,
                                                double* __restrict__ part) {
  __shared__ double red[4][WAVE][2 * QC];
  const int lane = threadIdx.x & (WAVE - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const int r = blockIdx.y * WAVE + lane;
  const int q0 = blockIdx.z * QC;
  const BlockIter it = block_iter(nblocks, 1);
  for (int64_t b = it.first; b < it.end; b += it.stride) {
    const int64_t e0 = (b * (blockDim.x / WAVE) + w) * (int64_t)epw;
    const int64_t e1 = e0 + epw < E ? e0 + epw : E;
    double are[QC], aim[QC];
#pragma unroll
    for (int k = 0; k < QC; ++k) are[k] = aim[k] = 0.0;
    if (r < R) {
      const double px = x0[(int64_t)r * 2], py = x0[(int64_t)r * 2 + 1];
      for (int64_t e = e0; e < e1; ++e) {
        const int4 m = elem[e];
        const int o = m.w & 1;
        const int ci = (m.w >> 4) & 0x3fff;
        const int cj = (m.w >> 18) & 0x3fff;
        double uv[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) uv[j] = (double)u[(e * NP + j) * (int64_t)R + r];
        const double dx = (ci + 0.5) * h - px;
        const double dy = (cj + 0.5) * h - py;
#pragma unroll
        for (int k = 0; k < QC; ++k) {
          const int qi = q0 + k;
          if (qi >= nq) break;
          const double* Wk = Wq + ((int64_t)qi * 2 + o) * NP * 2;
          double wr = 0.0, wi = 0.0;
#pragma unroll
          for (int j = 0; j < NP; ++j) {
            wr = fma(Wk[2 * j], uv[j], wr);
            wi = fma(Wk[2 * j + 1], uv[j], wi);
          }
          double sn, cs;
          sincos(qv[2 * qi] * dx + qv[2 * qi + 1] * dy, &sn, &cs);
          are[k] += cs * wr - sn * wi;
          aim[k] += sn * wr + cs * wi;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < QC; ++k) {
      red[w][lane][2 * k] = are[k];
      red[w][lane][2 * k + 1] = aim[k];
    }
    __syncthreads();
    if (w == 0 && r < R) {
      for (int k = 0; k < QC && q0 + k < nq; ++k)
        for (int c = 0; c < 2; ++c) {
          double sum = red[0][lane][2 * k + c];
          for (int v = 1; v < (int)(blockDim.x / WAVE); ++v) sum += red[v][lane][2 * k + c];
          part[((b * R + r) * (int64_t)nq + q0 + k) * 2 + c] = sum;
        }
    }
    __syncthreads();
  }
}

// out[g][r][c] = sum of part[b][r][c] (c < W) over the blocks b of geometry g.  One
// 64-lane workgroup per output value: each lane sums a strided subset of the
// blocks in order, then a fixed-order tree over the 64 lanes.
__global__ void __launch_bounds__(64) k_reduce_seg(const double* __restrict__ part,
                                                   const int* __restrict__ blk_start, int G, int R,
                                                   int W, double* __restrict__ out) {
  const int t = blockIdx.x;            // (g * R + r) * W + c
  if (t >= G * R * W) return;
  const int g = t / (R * W);
  const int rc = t % (R * W);
  const int b0 = blk_start[g], b1 = blk_start[g + 1];
  double s = 0;
  for (int b = b0 + (int)threadIdx.x; b < b1; b += 64) s += part[(int64_t)b * R * W + rc];
  __shared__ double sh[64];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int k = 32; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[t] = sh[0];
}

__device__ inline bool near_cell(int ci, int cj, double h, double px, double py, double lim) {
  const double xc = (ci + 0.5) * h, yc = (cj + 0.5) * h;
  double dx = fabs(xc - px) - 0.5 * h;
  double dy = fabs(yc - py) - 0.5 * h;
  dx = dx > 0 ? dx : 0;
  dy = dy > 0 ? dy : 0;
  return dx * dx + dy * dy <= lim * lim;
}

// quad layout: [o][q][3 + NP] = (x, y, w, phi_0 .. phi_{NP-1}), cell-local.
template <int NP>
__global__ void __launch_bounds__(256) k_ic_mass(const int4* __restrict__ elem, int64_t E,
                                                 const double* __restrict__ quad, int nq,
                                                 const double* __restrict__ x0,
                                                 const int* __restrict__ blk_geom, double sigma0,
                                                 double h, double cutoff, int R, int epw,
                                                 int64_t nblocks, double* __restrict__ part) {
  __shared__ double red[4][WAVE];
  const int lane = threadIdx.x & (WAVE - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const double inv2s2 = 1.0 / (2.0 * sigma0 * sigma0);
  const double lim = cutoff * sigma0;
  const BlockIter it = block_iter(nblocks, 1);
  for (int64_t b = it.first; b < it.end; b += it.stride) {
    const int g = blk_geom ? blk_geom[b] : 0;
    const int64_t e0 = (b * (blockDim.x / WAVE) + w) * (int64_t)epw;
    const int64_t e1 = e0 + epw < E ? e0 + epw : E;
    for (int r0 = 0; r0 < R; r0 += WAVE) {
      const int r = r0 + lane;
      double acc = 0;
      if (r < R) {
        const double px = x0[((int64_t)g * R + r) * 2], py = x0[((int64_t)g * R + r) * 2 + 1];
        for (int64_t e = e0; e < e1; ++e) {
          const int4 m = elem[e];
          const int o = m.w & 1;
          const int ci = (m.w >> 4) & 0x3fff;
          const int cj = (m.w >> 18) & 0x3fff;
          if (ci == kPadCell && cj == kPadCell) continue;   // batch padding
          if (!near_cell(ci, cj, h, px, py, lim)) continue;
          const double* Q = quad + (int64_t)o * nq * (3 + NP);
          double s = 0;
          for (int q = 0; q < nq; ++q) {
            const double X = (ci + Q[q * (3 + NP)]) * h - px;
            const double Y = (cj + Q[q * (3 + NP) + 1]) * h - py;
            s += Q[q * (3 + NP) + 2] * exp(-(X * X + Y * Y) * inv2s2);
          }
          acc += s * h * h;
        }
      }
      red[w][lane] = acc;
      __syncthreads();
      if (w == 0 && r < R) {
        double s = red[0][lane];
        for (int k = 1; k < (int)(blockDim.x / WAVE); ++k) s += red[k][lane];
        part[(b * R + r) * 6 + 0] = s;
        for (int c = 1; c < 6; ++c) part[(b * R + r) * 6 + c] = 0.0;
      }
      __syncthreads();
    }
  }
}

// u = M^-1 (sum_q w_q g(x_q) phi(x_q)) / mass, written for every element
// (zero beyond the cutoff).  mass is [G][R][6] (slot 0).
template <typename T, int NP>
__global__ void __launch_bounds__(256) k_ic_project(const int4* __restrict__ elem, int64_t E,
                                                    const double* __restrict__ quad, int nq,
                                                    const double* __restrict__ Minv,
                                                    const double* __restrict__ x0,
                                                    const int* __restrict__ blk_geom,
                                                    const double* __restrict__ mass, double sigma0,
                                                    double h, double cutoff, int R, int epw,
                                                    int64_t nblocks, T* __restrict__ u) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const double inv2s2 = 1.0 / (2.0 * sigma0 * sigma0);
  const double lim = cutoff * sigma0;
  const BlockIter it = block_iter(nblocks, 1);
  for (int64_t b = it.first; b < it.end; b += it.stride) {
    const int g = blk_geom ? blk_geom[b] : 0;
    const int64_t e0 = (b * (blockDim.x / WAVE) + w) * (int64_t)epw;
    const int64_t e1 = e0 + epw < E ? e0 + epw : E;
    for (int64_t e = e0; e < e1; ++e) {
      const int4 m = elem[e];
      const int o = m.w & 1;
      const int ci = (m.w >> 4) & 0x3fff;
      const int cj = (m.w >> 18) & 0x3fff;
      const double* Q = quad + (int64_t)o * nq * (3 + NP);
      const double* Mi = Minv + o * NP * NP;
      for (int r = lane; r < R; r += WAVE) {
        const double px = x0[((int64_t)g * R + r) * 2], py = x0[((int64_t)g * R + r) * 2 + 1];
        double c[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) c[j] = 0;
        if (!(ci == kPadCell && cj == kPadCell) && near_cell(ci, cj, h, px, py, lim)) {
          double bq[NP];
#pragma unroll
          for (int j = 0; j < NP; ++j) bq[j] = 0;
          for (int q = 0; q < nq; ++q) {
            const double* Qq = Q + q * (3 + NP);
            const double X = (ci + Qq[0]) * h - px;
            const double Y = (cj + Qq[1]) * h - py;
            const double gq = Qq[2] * exp(-(X * X + Y * Y) * inv2s2);
#pragma unroll
            for (int j = 0; j < NP; ++j) bq[j] += gq * Qq[3 + j];
          }
          const double s = 1.0 / mass[((int64_t)g * R + r) * 6];
#pragma unroll
          for (int i = 0; i < NP; ++i) {
            double a = 0;
#pragma unroll
            for (int j = 0; j < NP; ++j) a += Mi[i * NP + j] * bq[j];
            c[i] = a * s;
          }
        }
        const int64_t base = (e * NP) * (int64_t)R + r;
#pragma unroll
        for (int i = 0; i < NP; ++i) u[base + (int64_t)i * R] = (T)c[i];
      }
    }
  }
}

template <int NP>
__global__ void __launch_bounds__(256) k_dot_mass(const double* __restrict__ x,
                                                  const double* __restrict__ y,
                                                  const int4* __restrict__ elem, int64_t E,
                                                  const double* __restrict__ Mass, int R, int epw,
                                                  int64_t nblocks, double* __restrict__ part) {
  __shared__ double red[4][WAVE];
  const int lane = threadIdx.x & (WAVE - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const BlockIter it = block_iter(nblocks, 1);
  for (int64_t b = it.first; b < it.end; b += it.stride) {
    const int64_t e0 = (b * (blockDim.x / WAVE) + w) * (int64_t)epw;
    const int64_t e1 = e0 + epw < E ? e0 + epw : E;
    for (int r0 = 0; r0 < R; r0 += WAVE) {
      const int r = r0 + lane;
      double acc = 0;
      if (r < R) {
        for (int64_t e = e0; e < e1; ++e) {
          const int o = elem[e].w & 1;
          const double* M = Mass + o * NP * NP;
          const int64_t base = (e * NP) * (int64_t)R + r;
          double xv[NP], yv[NP];
#pragma unroll
          for (int j = 0; j < NP; ++j) {
            xv[j] = x[base + (int64_t)j * R];
            yv[j] = y[base + (int64_t)j * R];
          }
#pragma unroll
          for (int i = 0; i < NP; ++i) {
            double a = 0;
#pragma unroll
            for (int j = 0; j < NP; ++j) a += M[i * NP + j] * yv[j];
            acc += xv[i] * a;
          }
        }
      }
      red[w][lane] = acc;
      __syncthreads();
      if (w == 0 && r < R) {
        double s = red[0][lane];
        for (int k = 1; k < (int)(blockDim.x / WAVE); ++k) s += red[k][lane];
        part[(b * R + r) * 6 + 0] = s;
        for (int c = 1; c < 6; ++c) part[(b * R + r) * 6 + c] = 0.0;
      }
      __syncthreads();
    }
  }
}

// y = a x + b y (b == 0 never reads y)
__global__ void k_axpby(double* __restrict__ y, const double* __restrict__ x, double a, double b,
                        int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = b == 0.0 ? a * x[i] : a * x[i] + b * y[i];
}

template <typename T>
__global__ void k_fill_random(T* x, int64_t n, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // splitmix64 of (seed, i)
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  x[i] = (T)((double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0);
}

template <typename T, int NP>
void stage_t(const void* us, const void* ub, void* out, const int4* elem, int64_t E, const void* S,
             const void* N, int mode, double cb, double cg, int R, const Shape& sh,
             const uint32_t* step, int stage_id, const void* B, hipStream_t st) {
  const unsigned chunks = (unsigned)((R + 63) / 64);
  const dim3 grid((unsigned)sh.grid, chunks), block(64 * sh.waves);
#define DGD_STAGE_LAUNCH(MD, SP, BS, AB)                                                         \
  hipLaunchKernelGGL((k_stage<T, NP, MD, SP, BS, AB>), grid, block, 0, st, (const T*)us,         \
                     (const T*)ub, (T*)out, elem, E, (const double*)S, (const double*)N, mode, cb, \
                     cg, R, sh.epw, sh.blocks, sh.remap ? 1 : 0, step, stage_id, (const double*)B)
  const bool ab = B != nullptr;
  if constexpr (NP == 10) {
    if (mode == 0) {
      if (ab) DGD_STAGE_LAUNCH(0, true, false, true); else DGD_STAGE_LAUNCH(0, true, false, false);
    } else if (ub) {
      if (ab) DGD_STAGE_LAUNCH(1, true, true, true); else DGD_STAGE_LAUNCH(1, true, true, false);
    } else {
      if (ab) DGD_STAGE_LAUNCH(1, true, false, true); else DGD_STAGE_LAUNCH(1, true, false, false);
    }
  } else {
    if (mode == 0) DGD_STAGE_LAUNCH(0, false, false, false); else DGD_STAGE_LAUNCH(1, false, false, false);
  }
#undef DGD_STAGE_LAUNCH
}

// Advance a run's step counter (one lane, a vector store).
// Projected point masses: thread k * np + i writes coefficient i of the
// (geometry, start point) k into its element; the state is zero elsewhere.
// pe[k] is the element (row of the concatenated table), col[k] the column.
template <typename T>
__global__ void k_ic_point(const int64_t* __restrict__ pe, const int* __restrict__ col,
                           const double* __restrict__ vals, int n, int np, int R,
                           T* __restrict__ u) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * np) return;
  const int64_t k = t / np;
  const int i = (int)(t - k * np);
  u[(pe[k] * np + i) * (int64_t)R + col[k]] = (T)vals[t];
}

__global__ void k_step_bump(uint32_t* step) {
  if (threadIdx.x == 0) step[0] = step[0] + 1u;
}

}  // namespace

Shape element_shape(int64_t E, int epw, int waves, bool xcd_remap, int64_t max_grid) {
  Shape s;
  s.epw = epw;
  s.waves = waves;
  s.remap = xcd_remap;
  const int64_t per_block = (int64_t)s.waves * epw;
  s.blocks = (E + per_block - 1) / per_block;
  if (s.blocks < 1) s.blocks = 1;
  s.grid = s.blocks;
  if (max_grid > 0 && s.grid > max_grid) s.grid = max_grid;   // persistent
  if (s.remap) s.grid = (s.grid + 7) / 8 * 8;
  return s;
}

#define DGD_DISPATCH_NP(np, ...)                              \
  switch (np) {                                               \
    case 3: { constexpr int NP = 3; __VA_ARGS__; break; }     \
    case 6: { constexpr int NP = 6; __VA_ARGS__; break; }     \
    case 10: { constexpr int NP = 10; __VA_ARGS__; break; }   \
    default: break;                                           \
  }

void launch_stage(int prec, int np, const void* us, const void* ub, void* out, const int4* elem,
                  int64_t E, const void* S, const void* N, int mode, double cb, double cg, int R,
                  const Shape& sh, hipStream_t st, const uint32_t* step, int stage_id,
                  const void* B) {
  if (prec == 0) {
    DGD_DISPATCH_NP(np, stage_t<double, NP>(us, ub, out, elem, E, S, N, mode, cb, cg, R, sh, step,
                                            stage_id, B, st));
  } else {
    DGD_DISPATCH_NP(np, stage_t<float, NP>(us, ub, out, elem, E, S, N, mode, cb, cg, R, sh, step,
                                           stage_id, B, st));
  }
}

void launch_step_bump(uint32_t* step, hipStream_t st) {
  hipLaunchKernelGGL(k_step_bump, dim3(1), dim3(64), 0, st, step);
}

template <typename T, int NP>
void mixed_stage_t(const void* us, const void* ub, void* out, void* q, const int4* elem,
                   const uint8_t* meta, int64_t E, const void* MG, const void* MD, const void* MN,
                   const int* MNcol, int mode, double cb, double cg, int R, const Shape& sh, const uint32_t* step,
                   int stage_id, hipStream_t st) {
  const unsigned chunks = (unsigned)((R + 63) / 64);
  const dim3 grid((unsigned)sh.grid, chunks), block(64 * sh.waves);
  hipLaunchKernelGGL((k_mixed_grad<T, NP>), grid, block, 0, st, (const T*)us, (T*)q, elem, meta, E,
                     (const double*)MG, (const double*)MN, MNcol, R, sh.epw, sh.blocks,
                     sh.remap ? 1 : 0);
  hipLaunchKernelGGL((k_mixed_div<T, NP>), grid, block, 0, st, (const T*)q, (const T*)us,
                     (const T*)ub, (T*)out, elem, meta, E, (const double*)MD, (const double*)MN,
                     MNcol, mode, cb, cg, R, sh.epw, sh.blocks, sh.remap ? 1 : 0, step, stage_id);
}

void launch_mixed_stage(int prec, int np, const void* us, const void* ub, void* out, void* q,
                        const int4* elem, const uint8_t* meta, int64_t E, const void* MG,
                        const void* MD, const void* MN, const int* MNcol, int mode, double cb,
                        double cg, int R, const Shape& sh, hipStream_t st, const uint32_t* step,
                        int stage_id) {
  if (prec == 0) {
    DGD_DISPATCH_NP(np, mixed_stage_t<double, NP>(us, ub, out, q, elem, meta, E, MG, MD, MN, MNcol,
                                                  mode, cb, cg, R, sh, step, stage_id, st));
  } else {
    DGD_DISPATCH_NP(np, mixed_stage_t<float, NP>(us, ub, out, q, elem, meta, E, MG, MD, MN, MNcol,
                                                 mode, cb, cg, R, sh, step, stage_id, st));
  }
}

void launch_ic_point(int prec, const int64_t* pe, const int* col, const double* vals, int n, int np,
                     int R, void* u, hipStream_t st) {
  const int64_t threads = (int64_t)n * np;
  const unsigned grid = (unsigned)((threads + 255) / 256);
  if (prec == 0)
    hipLaunchKernelGGL(k_ic_point<double>, dim3(grid), dim3(256), 0, st, pe, col, vals, n, np, R,
                       (double*)u);
  else
    hipLaunchKernelGGL(k_ic_point<float>, dim3(grid), dim3(256), 0, st, pe, col, vals, n, np, R,
                       (float*)u);
}

void launch_stage_packed(int prec, int np, int G, const void* us, const void* ub, void* out,
                         const int4* elem, int64_t E, const void* S, const void* F, const void* N,
                         int mode, double cb, double cg, int R, const Shape& sh, hipStream_t st,
                         const uint32_t* step, int stage_id, const void* B) {
#define DGD_PACKED_LAUNCH1(T, GG, AB, MD)                                                       \
  DGD_DISPATCH_NP(np, hipLaunchKernelGGL((k_stage_packed<T, NP, GG, AB, MD>), dim3((unsigned)sh.grid), \
                                         dim3(64 * sh.waves), 0, st, (const T*)us, (const T*)ub, \
                                         (T*)out, elem, E, (const double*)S, (const double*)F,   \
                                         (const double*)N, mode, cb, cg, R, sh.epw, sh.blocks,   \
                                         sh.remap ? 1 : 0, step, stage_id, (const double*)B))
#define DGD_PACKED_LAUNCH(T, GG)                                                                \
  if (mode == 0) {                                                                              \
    if (B) { DGD_PACKED_LAUNCH1(T, GG, true, 0); } else { DGD_PACKED_LAUNCH1(T, GG, false, 0); } \
  } else {                                                                                      \
    if (B) { DGD_PACKED_LAUNCH1(T, GG, true, 1); } else { DGD_PACKED_LAUNCH1(T, GG, false, 1); } \
  }
  if (prec == 0 && G == 4) {
    DGD_PACKED_LAUNCH(double, 4);
  } else if (prec == 0) {
    DGD_PACKED_LAUNCH(double, 2);
  } else if (G == 4) {
    DGD_PACKED_LAUNCH(float, 4);
  } else {
    DGD_PACKED_LAUNCH(float, 2);
  }
#undef DGD_PACKED_LAUNCH
#undef DGD_PACKED_LAUNCH1
}

void launch_stage_p3_mfma(bool bf16x3, const void* us, const void* ub, void* out,
                          const int4* elem, int64_t E, const void* Atab, const double* Ctab,
                          const double* Wtab, double wsum, int mode, double cb, double cg, int R,
                          const Shape& sh, hipStream_t st, const uint32_t* step, int stage_id) {
  const dim3 grid((unsigned)sh.grid, (unsigned)((R + WAVE - 1) / WAVE));
  if (bf16x3)
    hipLaunchKernelGGL(k_stage_p3_mfma<true>, grid, dim3(64 * sh.waves), 0, st, (const float*)us,
                       (const float*)ub, (float*)out, elem, E, Atab, Ctab, Wtab, 1.0 / wsum, mode,
                       cb, cg, R, sh.epw, sh.blocks, sh.remap ? 1 : 0, step, stage_id);
  else
    hipLaunchKernelGGL(k_stage_p3_mfma<false>, grid, dim3(64 * sh.waves), 0, st, (const float*)us,
                       (const float*)ub, (float*)out, elem, E, Atab, Ctab, Wtab, 1.0 / wsum, mode,
                       cb, cg, R, sh.epw, sh.blocks, sh.remap ? 1 : 0, step, stage_id);
}

void launch_cheb(int np, const double* tcur, const double* tprev, double* tnext, double* res,
                 const int4* elem, int64_t E, const void* S, const void* N, double cg, double ck,
                 int R, const Shape& sh, hipStream_t st, const void* B) {
  const unsigned chunks = (unsigned)((R + 63) / 64);
  if (B) {
    DGD_DISPATCH_NP(np, hipLaunchKernelGGL((k_stage<double, NP, 2, true, true, true>),
                                           dim3((unsigned)sh.grid, chunks), dim3(64 * sh.waves), 0, st,
                                           tcur, tprev, tnext, elem, E, (const double*)S,
                                           (const double*)N, 2, 0.0, cg, R, sh.epw, sh.blocks,
                                           sh.remap ? 1 : 0, nullptr, 0, (const double*)B, res, ck));
  } else {
    DGD_DISPATCH_NP(np, hipLaunchKernelGGL((k_stage<double, NP, 2, true, true, false>),
                                           dim3((unsigned)sh.grid, chunks), dim3(64 * sh.waves), 0, st,
                                           tcur, tprev, tnext, elem, E, (const double*)S,
                                           (const double*)N, 2, 0.0, cg, R, sh.epw, sh.blocks,
                                           sh.remap ? 1 : 0, nullptr, 0, (const double*)B, res, ck));
  }
}

void launch_axpby(double* y, const double* x, double a, double b, int64_t n, hipStream_t st) {
  k_axpby<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(y, x, a, b, n);
}

void launch_moments(int prec, int np, const void* u, const int4* elem, int64_t E, const double* W,
                    const double* x0, const int* blk_geom, double h, int R, const Shape& sh,
                    double* part, hipStream_t st) {
  const dim3 grid((unsigned)sh.grid), block(64 * sh.waves);
  if (prec == 0) {
    DGD_DISPATCH_NP(np, k_moments<double, NP><<<grid, block, 0, st>>>(
                            (const double*)u, elem, E, W, x0, blk_geom, h, R, sh.epw, sh.blocks,
                            part));
  } else {
    DGD_DISPATCH_NP(np, k_moments<float, NP><<<grid, block, 0, st>>>(
                            (const float*)u, elem, E, W, x0, blk_geom, h, R, sh.epw, sh.blocks,
                            part));
  }
}

void launch_reduce(const double* part, const int* blk_start, int G, int R, double* out,
                   hipStream_t st) {
  k_reduce_seg<<<dim3((unsigned)(G * R * 6)), dim3(64), 0, st>>>(part, blk_start, G, R, 6, out);
}

void launch_signal(int prec, int np, const void* u, const int4* elem, int64_t E, const double* Wq,
                   const double* qv, int nq, const double* x0, double h, int R, const Shape& sh,
                   double* part, hipStream_t st) {
  constexpr int QC = 8;
  const dim3 grid((unsigned)sh.grid, (unsigned)((R + WAVE - 1) / WAVE), (unsigned)((nq + QC - 1) / QC));
  if (prec == 0) {
    DGD_DISPATCH_NP(np, hipLaunchKernelGGL((k_signal<double, NP, QC>), grid, dim3(64 * sh.waves), 0,
                                           st, (const double*)u, elem, E, Wq, qv, nq, x0, h, R,
                                           sh.epw, sh.blocks, part));
  } else {
    DGD_DISPATCH_NP(np, hipLaunchKernelGGL((k_signal<float, NP, QC>), grid, dim3(64 * sh.waves), 0,
                                           st, (const float*)u, elem, E, Wq, qv, nq, x0, h, R,
                                           sh.epw, sh.blocks, part));
  }
}

void launch_reduce_width(const double* part, const int* blk_start, int G, int R, int W,
                         double* out, hipStream_t st) {
  k_reduce_seg<<<dim3((unsigned)(G * R * W)), dim3(64), 0, st>>>(part, blk_start, G, R, W, out);
}

void launch_ic_mass(int np, const int4* elem, int64_t E, const double* quad, int nq,
                    const double* x0, const int* blk_geom, double sigma0, double h, double cutoff,
                    int R, const Shape& sh, double* part, hipStream_t st) {
  DGD_DISPATCH_NP(np, k_ic_mass<NP><<<dim3((unsigned)sh.grid), dim3(64 * sh.waves), 0, st>>>(
                          elem, E, quad, nq, x0, blk_geom, sigma0, h, cutoff, R, sh.epw,
                          sh.blocks, part));
}

void launch_ic_project(int prec, int np, const int4* elem, int64_t E, const double* quad, int nq,
                       const double* Minv, const double* x0, const int* blk_geom,
                       const double* mass, double sigma0, double h, double cutoff, int R,
                       const Shape& sh, void* u, hipStream_t st) {
  const dim3 grid((unsigned)sh.grid), block(64 * sh.waves);
  if (prec == 0) {
    DGD_DISPATCH_NP(np, k_ic_project<double, NP><<<grid, block, 0, st>>>(
                            elem, E, quad, nq, Minv, x0, blk_geom, mass, sigma0, h, cutoff, R,
                            sh.epw, sh.blocks, (double*)u));
  } else {
    DGD_DISPATCH_NP(np, k_ic_project<float, NP><<<grid, block, 0, st>>>(
                            elem, E, quad, nq, Minv, x0, blk_geom, mass, sigma0, h, cutoff, R,
                            sh.epw, sh.blocks, (float*)u));
  }
}

void launch_dot_mass(int np, const double* x, const double* y, const int4* elem, int64_t E,
                     const double* Mass, int R, const Shape& sh, double* part, hipStream_t st) {
  DGD_DISPATCH_NP(np, k_dot_mass<NP><<<dim3((unsigned)sh.grid), dim3(64 * sh.waves), 0, st>>>(
                          x, y, elem, E, Mass, R, sh.epw, sh.blocks, part));
}

void launch_fill_random(double* x, int64_t n, uint64_t seed, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_random<double>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n,
                     seed);
}

void launch_fill_random_f32(float* x, int64_t n, uint64_t seed, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_random<float>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n,
                     seed);
}

}  // namespace dgd
