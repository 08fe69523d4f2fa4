// Launch-shape autotuner of the stage kernels (internal).
//
// The stage kernels give the same bits for every launch shape (each
// element and right-hand side is computed by one lane, in a fixed order),
// so the shape is a pure performance choice.  The tuner times every shape
// of a small search space on the device and keeps the fastest per key:
// device architecture, element size Np, state precision, kernel (VALU,
// packed VALU or matrix core), number of right-hand sides, and the element
// count rounded down to a power of two.
#pragma once

#include <functional>
#include <string>

#include "dgd_internal.h"
#include "launch.h"

namespace dgd {

struct TuneParams {
  int epw = 1;          // elements per wave
  int waves = 4;        // waves per workgroup (1, 2 or 4)
  int remap = 1;        // XCD-banded block order
  int grid_per_cu = 0;  // > 0: persistent grid of this many workgroups per CU
  double ms = 0;        // measured time of one stage launch
};

std::string tune_key(int np, int prec, const char* kernel, int R, int64_t E);
bool tune_find(const std::string& key, TuneParams* out);
// Shape over `units` work units (elements, or element groups of the packed
// kernel).
Shape tune_shape(const TuneParams& p, int64_t units);

// One launch of the kernel being tuned: out = stage(src, base).
using StageLaunch = std::function<void(const Shape&, const void* src, const void* base, void* out)>;

// Time every candidate shape of `launch` over `units` work units on an
// SSP-RK3 step's pattern of launches (one stage without a base state, two
// reading `base`), using a and b (n_values states of the given precision
// each) as scratch and reading `base` (n_values finite states, left
// unchanged; NULL: a is filled and read as the base).  Stores the fastest
// under `key` and returns it (ms per launch).  Synchronises the stream.
TuneParams tune_stage(const std::string& key, int64_t units, int prec, int64_t n_values, void* a,
                      void* b, const void* base, const StageLaunch& launch, hipStream_t st);

std::string tune_export();
int tune_import(const std::string& text);
void tune_clear();

}  // namespace dgd
