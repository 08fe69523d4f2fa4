// Host-side launch wrappers of the HIP kernels (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dgd {

// Launch shape shared by the element kernels: workgroups of `waves` 64-wide
// waves, each wave walking `epw` consecutive elements with its lanes on
// right-hand sides.  `blocks` logical blocks cover the elements; `grid`
// workgroups are launched (fewer than `blocks` makes the kernel persistent).
// With `remap`, each of the eight XCDs sweeps one contiguous band of blocks.
struct Shape {
  int epw = 1;
  int waves = 4;        // <= 4: the reduction kernels use 4-wave LDS arrays
  bool remap = true;
  int64_t blocks = 0;
  int64_t grid = 0;
};
Shape element_shape(int64_t E, int epw, int waves = 4, bool xcd_remap = true, int64_t max_grid = 0);

// One SSP-RK3 stage (mode 1) or a plain operator apply (mode 0):
//   mode 0: out = cg * L(us)
//   mode 1: out = base + cb * (us - base) + cg * L(us), base = ub (or us when ub is NULL)
// with L(us)_K = S_{o,mask}(us_K - c) + sum_f N_{o,f}(us_f - c), c = us_K[node 0]
// per right-hand side; S, N are FP64.  `ub` may equal `out`.
// step (NULL: 0) is the run's device step counter and stage_id (0..2) the
// stage within the step: both enter the salt of the stochastic rounding of
// FP32 stores (modes 1, 2).  B (NULL: zero-flux box) is FP64 [2][3][np][np],
// the blocks of faces on an absorbing box (neighbour code -2, faces 0, 1).
void launch_stage(int prec, int np, const void* us, const void* ub, void* out, const int4* elem,
                  int64_t E, const void* S, const void* N, int mode, double cb, double cg, int R,
                  const Shape& sh, hipStream_t st, const uint32_t* step = nullptr, int stage_id = 0,
                  const void* B = nullptr);
// step[0] += 1 (a one-lane kernel, so graph replays advance the counter).
void launch_step_bump(uint32_t* step, hipStream_t st);

// Packed stage for R <= 64 / G right-hand sides (G = 4: R <= 16, G = 2:
// R <= 32): G elements per wave.  Same modes 0 and 1 as launch_stage; F is
// FP64 [2][3][np][np], the self-face blocks with S_{o,mask} = S_{o,7} -
// sum_{f not in mask} F_{o,f}.  The shape counts groups of G elements.
void launch_stage_packed(int prec, int np, int G, const void* us, const void* ub, void* out,
                         const int4* elem, int64_t E, const void* S, const void* F, const void* N,
                         int mode, double cb, double cg, int R, const Shape& sh, hipStream_t st,
                         const uint32_t* step = nullptr, int stage_id = 0, const void* B = nullptr);

// P3 stage on matrix cores (FP32 state, R % 16 == 0; each wave walks epw
// elements for 64 right-hand sides, grid.y covers the rest), same modes and
// coefficients as launch_stage, with a per-element FP64 mass correction.
// bf16x3: BF16 hi/lo split products (Atab in the BF16 lane order), else FP32
// products (Atab in the FP32 lane order).
void launch_stage_p3_mfma(bool bf16x3, const void* us, const void* ub, void* out,
                          const int4* elem, int64_t E, const void* Atab, const double* Ctab,
                          const double* Wtab, double wsum, int mode, double cb, double cg, int R,
                          const Shape& sh, hipStream_t st, const uint32_t* step = nullptr,
                          int stage_id = 0);

// One step of the Chebyshev recurrence for exp(t L) (FP64 state):
//   tnext = 2 (tcur + cg L(tcur)) - tprev,   res += ck * tnext.
void launch_cheb(int np, const double* tcur, const double* tprev, double* tnext, double* res,
                 const int4* elem, int64_t E, const void* S, const void* N, double cg, double ck,
                 int R, const Shape& sh, hipStream_t st, const void* B = nullptr);
// y = a x + b y over n values (b == 0: y is only written).
void launch_axpby(double* y, const double* x, double a, double b, int64_t n, hipStream_t st);

// FP64 moment partial sums per logical block: part[b][r][6].  x0 is
// [G][R][2]; blk_geom (NULL when G = 1) gives the geometry of each block.
void launch_moments(int prec, int np, const void* u, const int4* elem, int64_t E, const double* W,
                    const double* x0, const int* blk_geom, double h, int R, const Shape& sh,
                    double* part, hipStream_t st);

// out[g][r][c] = sum over the blocks of geometry g (blk_start[g] ..
// blk_start[g+1]) of part[b][r][c], in a fixed order.
void launch_reduce(const double* part, const int* blk_start, int G, int R, double* out,
                   hipStream_t st);

// Partial q-space signal per block: part[b][r][q][2] = (re, im) of the
// block's elements' sum of exp(i q.(c_K - x0_r)) sum_j Wq[q][o][j] u_K[j][r]
// (one geometry; Wq [nq][2][np][2], qv [nq][2], x0 [R][2]).
void launch_signal(int prec, int np, const void* u, const int4* elem, int64_t E, const double* Wq,
                   const double* qv, int nq, const double* x0, double h, int R, const Shape& sh,
                   double* part, hipStream_t st);
// launch_reduce over W values per (geometry, right-hand side).
void launch_reduce_width(const double* part, const int* blk_start, int G, int R, int W,
                         double* out, hipStream_t st);

// Initial data.  The mass pass writes part[b][r][0] = sum of h^2 w_q g(x_q)
// over the block's elements; the project pass writes
// u = M^-1 (sum_q w_q g phi) / mass[g][r].
void launch_ic_mass(int np, const int4* elem, int64_t E, const double* quad, int nq,
                    const double* x0, const int* blk_geom, double sigma0, double h, double cutoff,
                    int R, const Shape& sh, double* part, hipStream_t st);
void launch_ic_project(int prec, int np, const int4* elem, int64_t E, const double* quad, int nq,
                       const double* Minv, const double* x0, const int* blk_geom,
                       const double* mass, double sigma0, double h, double cutoff, int R,
                       const Shape& sh, void* u, hipStream_t st);

// One RK stage of the mixed form: q = grad pass into q ([E][2][np][R], the
// state type), then the divergence pass with the stage combine of
// launch_stage (modes 0 and 1).  meta [E]: face mask of the q-flux | 8 for
// an extracellular element.  MG, MD: FP64 [2][8][2][np][np]; MN: FP64
// [2][3][2][np][p+1], the neighbour blocks on the face-node columns MNcol
// (int32 [2][3][p+1]).
void launch_mixed_stage(int prec, int np, const void* us, const void* ub, void* out, void* q,
                        const int4* elem, const uint8_t* meta, int64_t E, const void* MG,
                        const void* MD, const void* MN, const int* MNcol, int mode, double cb,
                        double cg, int R, const Shape& sh, hipStream_t st,
                        const uint32_t* step = nullptr, int stage_id = 0);

// Point-mass initial data: u[(pe[k] np + i) R + col[k]] = vals[k np + i]
// for k < n (the rest of u is cleared by the caller).
void launch_ic_point(int prec, const int64_t* pe, const int* col, const double* vals, int n, int np,
                     int R, void* u, hipStream_t st);

// part[b][r][0] = sum over the block's elements of x_K^T Mhat y_K (FP64).
void launch_dot_mass(int np, const double* x, const double* y, const int4* elem, int64_t E,
                     const double* Mass, int R, const Shape& sh, double* part, hipStream_t st);

// x[i] = deterministic pseudo-random value in [-1, 1) from (seed, i).
void launch_fill_random(double* x, int64_t n, uint64_t seed, hipStream_t st);
void launch_fill_random_f32(float* x, int64_t n, uint64_t seed, hipStream_t st);

}  // namespace dgd
