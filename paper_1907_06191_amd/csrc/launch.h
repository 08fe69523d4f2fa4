// Host-side launch wrappers of the HIP kernels (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dgd {

// Launch shape shared by the element kernels: 256-thread workgroups (four
// 64-wide waves), each wave walking `epw` consecutive elements with its
// lanes on right-hand sides.  Blocks are remapped so that each of the eight
// XCDs sweeps one contiguous band of elements.
struct Shape {
  int epw = 4;          // elements per wave
  int waves = 4;        // waves per workgroup (<= 4: the reductions use 4-wave LDS arrays)
  int64_t blocks = 0;   // logical blocks (negative: identity block mapping, |blocks| blocks)
  int64_t grid = 0;     // launched blocks (multiple of 8 with the XCD remap)
  int64_t nblk() const { return blocks < 0 ? -blocks : blocks; }
};
Shape element_shape(int64_t E, int epw, int waves = 4, bool xcd_remap = true);

// One SSP-RK3 stage (mode 1) or a plain operator apply (mode 0):
//   mode 0: out = cg * L(us)
//   mode 1: out = base + cb * (us - base) + cg * L(us), base = ub (or us when ub is NULL)
// with L(us)_K = S_{o,mask}(us_K - c) + sum_f N_{o,f}(us_f - c), c = us_K[node 0]
// per right-hand side.  `ub` may equal `out`.
void launch_stage(int prec, int np, const void* us, const void* ub, void* out, const int4* elem,
                  int64_t E, const void* S, const void* N, int mode, double cb, double cg, int R,
                  const Shape& sh, hipStream_t st);

// FP64 moment partial sums per block: part[b][r][6].
void launch_moments(int prec, int np, const void* u, const int4* elem, int64_t E, const double* W,
                    const double* x0, double h, int R, const Shape& sh, double* part, hipStream_t st);

// Deterministic sum of partials over blocks: out[r][c] = sum_b part[b][r][c], c < 6.
void launch_reduce(const double* part, int nblk, int R, double* out, hipStream_t st);

// Initial data.  Mass pass writes part[b][r][0] = sum of h^2 w_q g(x_q) over
// the block's elements; project pass writes u = M^-1 (sum_q w_q g phi) / mass.
void launch_ic_mass(int np, const int4* elem, int64_t E, const double* quad, int nq,
                    const double* x0, double sigma0, double h, double cutoff, int R, const Shape& sh,
                    double* part, hipStream_t st);
void launch_ic_project(int prec, int np, const int4* elem, int64_t E, const double* quad, int nq,
                       const double* Minv, const double* x0, const double* mass, double sigma0,
                       double h, double cutoff, int R, const Shape& sh, void* u, hipStream_t st);

// part[b][r][0] = sum over the block's elements of x_K^T Mhat y_K (FP64).
void launch_dot_mass(int np, const double* x, const double* y, const int4* elem, int64_t E,
                     const double* Mass, int R, const Shape& sh, double* part, hipStream_t st);

// x[i] = deterministic pseudo-random value in [-1, 1) from (seed, i).
void launch_fill_random(double* x, int64_t n, uint64_t seed, hipStream_t st);
void launch_scale(double* x, int64_t n, double s, hipStream_t st);

}  // namespace dgd
