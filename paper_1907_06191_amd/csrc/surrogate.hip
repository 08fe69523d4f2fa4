// Learned surrogate: an occupancy-image CNN + MLP that predicts
// Sigma / (2 D Delta) of the start-point mixture, trained on DG solves, with
// hand-written HIP kernels for every forward and backward step (FP32).
//
// Network (per ensemble member):
//   4 x [conv 3x3 zero-pad 1 -> C channels, + bias, ReLU, 2x2 average pool]
//   64x64x1 -> 32x32xC -> 16x16xC -> 8x8xC -> 4x4xC, flatten (c, y, x),
//   append log Delta, 3 x [dense H + bias, ReLU], dense 3 + bias; MSE loss.
// Parameters: one flat FP32 vector per member, layer order conv1.w, conv1.b,
// ..., conv4.b, fc1.w [H][16C+1], fc1.b, fc2.w, fc2.b, fc3.w, fc3.b,
// head.w [3][H], head.b.  All reductions run in a fixed order, so training
// is bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "dgd_internal.h"

namespace dgd {
namespace {

constexpr int IMG = 64;
constexpr int MAXC = 32;

// ------------------------------------------------------------- kernels ----

__global__ void k_gather(const uint8_t* __restrict__ imgs, const double* __restrict__ logd,
                         const int* __restrict__ idx, int B, float* __restrict__ x,
                         float* __restrict__ ld) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < (int64_t)B * IMG * IMG) {
    const int b = (int)(t / (IMG * IMG));
    const int p = (int)(t % (IMG * IMG));
    x[t] = (float)imgs[(int64_t)idx[b] * IMG * IMG + p];
  }
  if (t < B) ld[t] = (float)logd[idx[t]];
}

// z = conv(x) + bias, a = relu(z).  One workgroup per (image, tile of
// T x T pixels), one thread per pixel computing all Co outputs; input tile
// with halo and all weights staged in LDS.
template <int T>
__global__ void __launch_bounds__(T * T) k_conv_fwd(const float* __restrict__ x,
                                                    const float* __restrict__ w,
                                                    const float* __restrict__ bias,
                                                    float* __restrict__ z, float* __restrict__ a,
                                                    int Ci, int Co, int S) {
  __shared__ float tile[8][T + 2][T + 2];
  __shared__ float ws[MAXC * MAXC * 9];
  const int tiles = S / T;
  const int b = blockIdx.x / (tiles * tiles);
  const int tt = blockIdx.x % (tiles * tiles);
  const int ty0 = (tt / tiles) * T, tx0 = (tt % tiles) * T;
  const int ly = threadIdx.x / T, lx = threadIdx.x % T;
  for (int k = threadIdx.x; k < Co * Ci * 9; k += T * T) ws[k] = w[k];
  float acc[MAXC];
#pragma unroll
  for (int co = 0; co < MAXC; ++co) acc[co] = 0.f;
  for (int c0 = 0; c0 < Ci; c0 += 8) {
    const int nc = min(8, Ci - c0);
    __syncthreads();
    for (int k = threadIdx.x; k < nc * (T + 2) * (T + 2); k += T * T) {
      const int c = k / ((T + 2) * (T + 2));
      const int r = k % ((T + 2) * (T + 2));
      const int yy = ty0 + r / (T + 2) - 1, xx = tx0 + r % (T + 2) - 1;
      tile[c][r / (T + 2)][r % (T + 2)] =
          (yy >= 0 && yy < S && xx >= 0 && xx < S) ? x[(((int64_t)b * Ci + c0 + c) * S + yy) * S + xx] : 0.f;
    }
    __syncthreads();
    for (int c = 0; c < nc; ++c)
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        const float v = tile[c][ly + t / 3][lx + t % 3];
#pragma unroll
        for (int co = 0; co < MAXC; ++co)
          if (co < Co) acc[co] += ws[(co * Ci + c0 + c) * 9 + t] * v;
      }
  }
  const int y = ty0 + ly, xx = tx0 + lx;
#pragma unroll
  for (int co = 0; co < MAXC; ++co)
    if (co < Co) {
      const float v = acc[co] + bias[co];
      const int64_t o = (((int64_t)b * Co + co) * S + y) * S + xx;
      z[o] = v;
      a[o] = v > 0.f ? v : 0.f;
    }
}

// dx = conv^T(dz): dx[b][ci][y][x] = sum_co sum_t w[co][ci][t] dz[b][co][y + 1 - ty][x + 1 - tx].
template <int T>
__global__ void __launch_bounds__(T * T) k_conv_bwd_data(const float* __restrict__ dz,
                                                         const float* __restrict__ w,
                                                         float* __restrict__ dx, int Ci, int Co,
                                                         int S) {
  __shared__ float tile[8][T + 2][T + 2];
  __shared__ float ws[MAXC * MAXC * 9];
  const int tiles = S / T;
  const int b = blockIdx.x / (tiles * tiles);
  const int tt = blockIdx.x % (tiles * tiles);
  const int ty0 = (tt / tiles) * T, tx0 = (tt % tiles) * T;
  const int ly = threadIdx.x / T, lx = threadIdx.x % T;
  for (int k = threadIdx.x; k < Co * Ci * 9; k += T * T) ws[k] = w[k];
  float acc[MAXC];
#pragma unroll
  for (int ci = 0; ci < MAXC; ++ci) acc[ci] = 0.f;
  for (int c0 = 0; c0 < Co; c0 += 8) {
    const int nc = min(8, Co - c0);
    __syncthreads();
    for (int k = threadIdx.x; k < nc * (T + 2) * (T + 2); k += T * T) {
      const int c = k / ((T + 2) * (T + 2));
      const int r = k % ((T + 2) * (T + 2));
      const int yy = ty0 + r / (T + 2) - 1, xx = tx0 + r % (T + 2) - 1;
      tile[c][r / (T + 2)][r % (T + 2)] =
          (yy >= 0 && yy < S && xx >= 0 && xx < S) ? dz[(((int64_t)b * Co + c0 + c) * S + yy) * S + xx] : 0.f;
    }
    __syncthreads();
    for (int c = 0; c < nc; ++c)
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        // dz at (y + 1 - ty, x + 1 - tx) = tile[ly + 2 - ty][lx + 2 - tx]
        const float v = tile[c][ly + 2 - t / 3][lx + 2 - t % 3];
#pragma unroll
        for (int ci = 0; ci < MAXC; ++ci)
          if (ci < Ci) acc[ci] += ws[((c0 + c) * Ci + ci) * 9 + t] * v;
      }
  }
  const int y = ty0 + ly, xx = tx0 + lx;
#pragma unroll
  for (int ci = 0; ci < MAXC; ++ci)
    if (ci < Ci) dx[(((int64_t)b * Ci + ci) * S + y) * S + xx] = acc[ci];
}

// dw[co][ci][t] = sum_b sum_pix dz[b][co][pix] x[b][ci][pix + t - (1,1)];
// db[co] = sum dz (computed by the ci == 0 workgroup).  One 256-thread
// workgroup per (co, ci); fixed-order tree reduction.
__global__ void __launch_bounds__(256) k_conv_bwd_weight(const float* __restrict__ x,
                                                         const float* __restrict__ dz,
                                                         float* __restrict__ dw,
                                                         float* __restrict__ db, int B, int Ci,
                                                         int Co, int S) {
  const int co = blockIdx.x / Ci, ci = blockIdx.x % Ci;
  float acc[10];
#pragma unroll
  for (int t = 0; t < 10; ++t) acc[t] = 0.f;
  const int64_t n = (int64_t)B * S * S;
  for (int64_t k = threadIdx.x; k < n; k += 256) {
    const int b = (int)(k / (S * S));
    const int p = (int)(k % (S * S));
    const int y = p / S, xx = p % S;
    const float g = dz[((int64_t)b * Co + co) * S * S + p];
    const float* xb = x + ((int64_t)b * Ci + ci) * S * S;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int yy = y + t / 3 - 1, xs = xx + t % 3 - 1;
      if (yy >= 0 && yy < S && xs >= 0 && xs < S) acc[t] += g * xb[yy * S + xs];
    }
    acc[9] += g;
  }
  __shared__ float red[10][256];
#pragma unroll
  for (int t = 0; t < 10; ++t) red[t][threadIdx.x] = acc[t];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
#pragma unroll
      for (int t = 0; t < 10; ++t) red[t][threadIdx.x] += red[t][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 9) dw[((int64_t)co * Ci + ci) * 9 + threadIdx.x] = red[threadIdx.x][0];
  if (threadIdx.x == 0 && ci == 0) db[co] = red[9][0];
}

__global__ void k_pool_fwd(const float* __restrict__ a, float* __restrict__ y, int BC, int S) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int So = S / 2;
  if (t >= (int64_t)BC * So * So) return;
  const int64_t bc = t / (So * So);
  const int p = (int)(t % (So * So));
  const int i = p / So, j = p % So;
  const float* s = a + bc * S * S;
  y[t] = 0.25f * (s[(2 * i) * S + 2 * j] + s[(2 * i) * S + 2 * j + 1] + s[(2 * i + 1) * S + 2 * j] +
                  s[(2 * i + 1) * S + 2 * j + 1]);
}

// dz = 0.25 * dy[parent] * (z > 0)
__global__ void k_pool_relu_bwd(const float* __restrict__ dy, const float* __restrict__ z,
                                float* __restrict__ dz, int BC, int S) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)BC * S * S) return;
  const int64_t bc = t / (S * S);
  const int p = (int)(t % (S * S));
  const int y = p / S, x = p % S;
  const int So = S / 2;
  dz[t] = z[t] > 0.f ? 0.25f * dy[bc * So * So + (y / 2) * So + x / 2] : 0.f;
}

// feat[b] = [pooled4[b] (16 C values), log Delta[b]]
__global__ void k_concat(const float* __restrict__ p4, const float* __restrict__ ld, float* __restrict__ feat,
                         int B, int F) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)B * (F + 1)) return;
  const int b = (int)(t / (F + 1)), k = (int)(t % (F + 1));
  feat[t] = k < F ? p4[(int64_t)b * F + k] : ld[b];
}

// dpool4[b][k] = dfeat[b][k] for k < F
__global__ void k_split_feat(const float* __restrict__ dfeat, float* __restrict__ dp4, int B, int F) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)B * F) return;
  const int b = (int)(t / F), k = (int)(t % F);
  dp4[t] = dfeat[(int64_t)b * (F + 1) + k];
}

// C[m][n] = sum_k A(m, k) B(k, n), A(m, k) = A[m*sam + k*sak], B(k, n) = B[k*sbk + n*sbn]
// (every dense layer's forward and backward product), on the matrix cores:
// a workgroup of four waves computes a 64 x 64 tile of C, each wave a
// 32 x 32 quarter as 2 x 2 blocks of v_mfma_f32_16x16x4_f32; K runs in
// chunks of 16 staged through LDS (zero-filled past M, N, K), four MFMA
// k-steps per chunk, in a fixed order.  Operand layout of one MFMA: lane l
// holds A[m = l % 16][k = l / 16] and B[k = l / 16][n = l % 16] and
// receives D[m = 4 (l / 16) + i][n = l % 16], i < 4.
constexpr int GT = 64;    // C tile edge per workgroup
constexpr int GK = 16;    // K chunk
__global__ void __launch_bounds__(256) k_gemm(const float* __restrict__ A, const float* __restrict__ Bm,
                                              float* __restrict__ C, int M, int N, int K,
                                              int64_t sam, int64_t sak, int64_t sbk, int64_t sbn,
                                              int ldc) {
  typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
  __shared__ float As[GT][GK + 1];
  __shared__ float Bs[GK][GT + 1];
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;      // wave's quarter of the tile
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  const int lr = lane & 15, lk = lane >> 4;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += GK) {
    // stage A[m0 .. m0+63][k0 .. k0+15] and B[k0 .. k0+15][n0 .. n0+63]:
    // 1024 values each, four per thread
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = t + 256 * q;
      const int am = idx / GK, ak = idx % GK;
      const int gm = m0 + am, gk = k0 + ak;
      As[am][ak] = (gm < M && gk < K) ? A[gm * sam + gk * sak] : 0.f;
      const int bk = idx / GT, bn = idx % GT;
      const int hk = k0 + bk, hn = n0 + bn;
      Bs[bk][bn] = (hk < K && hn < N) ? Bm[hk * sbk + hn * sbn] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int st = 0; st < GK / 4; ++st) {
      const int kk = 4 * st + lk;
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[wm + 16 * i + lr][kk];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[kk][wn + 16 * j + lr];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * i + 4 * lk + r, n = n0 + wn + 16 * j + lr;
        if (m < M && n < N) C[(int64_t)m * ldc + n] = acc[i][j][r];
      }
}

// z[b][n] += bias[n]; a = relu(z) (relu off: a = z)
__global__ void k_bias_act(float* __restrict__ z, const float* __restrict__ bias, float* __restrict__ a,
                           int B, int N, int relu) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)B * N) return;
  const float v = z[t] + bias[t % N];
  z[t] = v;
  a[t] = (relu && v < 0.f) ? 0.f : v;
}

__global__ void k_relu_bwd(float* __restrict__ d, const float* __restrict__ z, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n && !(z[t] > 0.f)) d[t] = 0.f;
}

// db[n] = sum_b d[b][n] in batch order
__global__ void k_colsum(const float* __restrict__ d, float* __restrict__ db, int B, int N) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int b = 0; b < B; ++b) s += d[(int64_t)b * N + n];
  db[n] = s;
}

// dout = 2 (out - t) / (3 B); per-sample squared error for the loss
__global__ void k_mse(const float* __restrict__ out, const double* __restrict__ targ,
                      const int* __restrict__ idx, int B, float* __restrict__ dout,
                      float* __restrict__ se) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  float s = 0.f;
  for (int k = 0; k < 3; ++k) {
    const float d = out[b * 3 + k] - (float)targ[(int64_t)idx[b] * 3 + k];
    dout[b * 3 + k] = 2.f * d / (3.f * B);
    s += d * d;
  }
  se[b] = s;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float gi = g[t];
  const float mi = b1 * m[t] + (1.f - b1) * gi;
  const float vi = b2 * v[t] + (1.f - b2) * gi * gi;
  m[t] = mi;
  v[t] = vi;
  p[t] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Ensemble mean, spread = max over outputs of (max - min) over members, flag.
__global__ void k_ensemble(const float* __restrict__ outs, int M, int n, float thr,
                           double* __restrict__ mean, double* __restrict__ spread,
                           uint8_t* __restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float sp = 0.f;
  for (int k = 0; k < 3; ++k) {
    float lo = outs[(int64_t)i * 3 + k], hi = lo;
    double s = 0;
    for (int mb = 0; mb < M; ++mb) {
      const float v = outs[((int64_t)mb * n + i) * 3 + k];
      lo = fminf(lo, v);
      hi = fmaxf(hi, v);
      s += v;
    }
    mean[(int64_t)i * 3 + k] = s / M;
    sp = fmaxf(sp, hi - lo);
  }
  spread[i] = sp;
  flag[i] = sp > thr ? 1 : 0;
}

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// ---------------------------------------------------------------- model ----

struct Layout {
  int C, H;
  int64_t off[16];
  int64_t size[16];
  int64_t total;
  void build(int C_, int H_) {
    C = C_;
    H = H_;
    int64_t k = 0;
    int cin = 1;
    for (int L = 0; L < 4; ++L) {
      off[2 * L] = k; size[2 * L] = (int64_t)C * cin * 9; k += size[2 * L];
      off[2 * L + 1] = k; size[2 * L + 1] = C; k += C;
      cin = C;
    }
    int feat = 16 * C + 1;
    for (int L = 0; L < 3; ++L) {
      off[8 + 2 * L] = k; size[8 + 2 * L] = (int64_t)H * feat; k += size[8 + 2 * L];
      off[9 + 2 * L] = k; size[9 + 2 * L] = H; k += H;
      feat = H;
    }
    off[14] = k; size[14] = 3 * (int64_t)H; k += size[14];
    off[15] = k; size[15] = 3; k += 3;
    total = k;
  }
};

// Activations of one batch.
struct Acts {
  int B = 0;
  float *x = nullptr, *ld = nullptr;
  float *z[4] = {}, *a[4] = {}, *p[4] = {};        // conv pre-act, post-act, pooled
  float *feat = nullptr, *dz[4] = {}, *hz[3] = {}, *ha[3] = {}, *out = nullptr;
  float *dout = nullptr, *se = nullptr, *dh = nullptr, *dh2 = nullptr, *dfeat = nullptr, *dp = nullptr;
  float *dc = nullptr, *dc2 = nullptr;
  int* idx = nullptr;
  std::vector<void*> owned;
  void* alloc(size_t bytes) {
    void* d = nullptr;
    DGD_HIP_CHECK(hipMalloc(&d, std::max<size_t>(bytes, 4)));
    owned.push_back(d);
    return d;
  }
  void build(int B_, const Layout& L) {
    B = B_;
    const int C = L.C, H = L.H;
    x = (float*)alloc((size_t)B * IMG * IMG * 4);
    ld = (float*)alloc((size_t)B * 4);
    idx = (int*)alloc((size_t)B * 4);
    int S = IMG;
    for (int l = 0; l < 4; ++l) {
      z[l] = (float*)alloc((size_t)B * C * S * S * 4);
      a[l] = (float*)alloc((size_t)B * C * S * S * 4);
      dz[l] = (float*)alloc((size_t)B * C * S * S * 4);
      p[l] = (float*)alloc((size_t)B * C * (S / 2) * (S / 2) * 4);
      S /= 2;
    }
    feat = (float*)alloc((size_t)B * (16 * C + 1) * 4);
    dfeat = (float*)alloc((size_t)B * (16 * C + 1) * 4);
    for (int l = 0; l < 3; ++l) {
      hz[l] = (float*)alloc((size_t)B * H * 4);
      ha[l] = (float*)alloc((size_t)B * H * 4);
    }
    out = (float*)alloc((size_t)B * 3 * 4);
    dout = (float*)alloc((size_t)B * 3 * 4);
    se = (float*)alloc((size_t)B * 4);
    dh = (float*)alloc((size_t)B * H * 4);
    dh2 = (float*)alloc((size_t)B * H * 4);
    dp = (float*)alloc((size_t)B * C * 32 * 32 * 4);
    dc = (float*)alloc((size_t)B * C * 32 * 32 * 4);
    dc2 = (float*)alloc((size_t)B * C * 32 * 32 * 4);
  }
  void release() {
    for (void* d : owned) (void)hipFree(d);
    owned.clear();
  }
};

void gemm(const float* A, const float* B, float* C, int M, int N, int K, int64_t sam, int64_t sak,
          int64_t sbk, int64_t sbn, int ldc, hipStream_t st) {
  k_gemm<<<dim3((N + GT - 1) / GT, (M + GT - 1) / GT), 256, 0, st>>>(A, B, C, M, N, K, sam, sak, sbk,
                                                                     sbn, ldc);
}

void conv_fwd(const float* x, const float* w, const float* b, float* z, float* a, int B, int Ci,
              int Co, int S, hipStream_t st) {
  if (S >= 16) {
    k_conv_fwd<16><<<B * (S / 16) * (S / 16), 256, 0, st>>>(x, w, b, z, a, Ci, Co, S);
  } else if (S == 8) {
    k_conv_fwd<8><<<B, 64, 0, st>>>(x, w, b, z, a, Ci, Co, S);
  } else {
    k_conv_fwd<4><<<B, 16, 0, st>>>(x, w, b, z, a, Ci, Co, S);
  }
}

void conv_bwd_data(const float* dz, const float* w, float* dx, int B, int Ci, int Co, int S,
                   hipStream_t st) {
  if (S >= 16) {
    k_conv_bwd_data<16><<<B * (S / 16) * (S / 16), 256, 0, st>>>(dz, w, dx, Ci, Co, S);
  } else if (S == 8) {
    k_conv_bwd_data<8><<<B, 64, 0, st>>>(dz, w, dx, Ci, Co, S);
  } else {
    k_conv_bwd_data<4><<<B, 16, 0, st>>>(dz, w, dx, Ci, Co, S);
  }
}

// Forward of one member on a gathered batch (acts.x, acts.ld filled).
void forward(const Layout& L, const float* P, Acts& A, hipStream_t st) {
  const int B = A.B, C = L.C, H = L.H;
  const float* in = A.x;
  int cin = 1, S = IMG;
  for (int l = 0; l < 4; ++l) {
    conv_fwd(in, P + L.off[2 * l], P + L.off[2 * l + 1], A.z[l], A.a[l], B, cin, C, S, st);
    k_pool_fwd<<<nblk((int64_t)B * C * (S / 2) * (S / 2)), 256, 0, st>>>(A.a[l], A.p[l], B * C, S);
    in = A.p[l];
    cin = C;
    S /= 2;
  }
  const int F = 16 * C;
  k_concat<<<nblk((int64_t)B * (F + 1)), 256, 0, st>>>(A.p[3], A.ld, A.feat, B, F);
  const float* h = A.feat;
  int fin = F + 1;
  for (int l = 0; l < 3; ++l) {
    // z[b][n] = sum_k h[b][k] W[n][k]
    gemm(h, P + L.off[8 + 2 * l], A.hz[l], B, H, fin, fin, 1, 1, fin, H, st);
    k_bias_act<<<nblk((int64_t)B * H), 256, 0, st>>>(A.hz[l], P + L.off[9 + 2 * l], A.ha[l], B, H, 1);
    h = A.ha[l];
    fin = H;
  }
  gemm(h, P + L.off[14], A.out, B, 3, H, H, 1, 1, H, 3, st);
  k_bias_act<<<nblk((int64_t)B * 3), 256, 0, st>>>(A.out, P + L.off[15], A.out, B, 3, 0);
}

// Backward from A.dout into the gradient vector G (overwritten).
void backward(const Layout& L, const float* P, float* G, Acts& A, hipStream_t st) {
  const int B = A.B, C = L.C, H = L.H;
  const int F = 16 * C;
  // head
  gemm(A.dout, A.ha[2], G + L.off[14], 3, H, B, 1, 3, H, 1, H, st);   // dW[j][k] = sum_b dout[b][j] h[b][k]
  k_colsum<<<1, 256, 0, st>>>(A.dout, G + L.off[15], B, 3);
  gemm(A.dout, P + L.off[14], A.dh, B, H, 3, 3, 1, H, 1, H, st);      // dh[b][k] = sum_j dout[b][j] W[j][k]
  float* dh = A.dh;
  float* dn = A.dh2;
  for (int l = 2; l >= 0; --l) {
    k_relu_bwd<<<nblk((int64_t)B * H), 256, 0, st>>>(dh, A.hz[l], (int64_t)B * H);
    const float* hin = l > 0 ? A.ha[l - 1] : A.feat;
    const int fin = l > 0 ? H : F + 1;
    gemm(dh, hin, G + L.off[8 + 2 * l], H, fin, B, 1, H, fin, 1, fin, st);
    k_colsum<<<nblk(H), 256, 0, st>>>(dh, G + L.off[9 + 2 * l], B, H);
    float* dst = l > 0 ? dn : A.dfeat;
    gemm(dh, P + L.off[8 + 2 * l], dst, B, fin, H, H, 1, fin, 1, fin, st);
    std::swap(dh, dn);
  }
  k_split_feat<<<nblk((int64_t)B * F), 256, 0, st>>>(A.dfeat, A.dp, B, F);
  // conv layers, from 4x4 back to 64x64
  const float* dpool = A.dp;
  int S = 8;   // spatial size of conv layer 4's pre-pool map
  for (int l = 3; l >= 0; --l) {
    const int cin = l > 0 ? C : 1;
    k_pool_relu_bwd<<<nblk((int64_t)B * C * S * S), 256, 0, st>>>(dpool, A.z[l], A.dz[l], B * C, S);
    const float* xin = l > 0 ? A.p[l - 1] : A.x;
    k_conv_bwd_weight<<<C * cin, 256, 0, st>>>(xin, A.dz[l], G + L.off[2 * l], G + L.off[2 * l + 1], B,
                                                cin, C, S);
    if (l > 0) {
      float* dx = (l % 2) ? A.dc : A.dc2;
      conv_bwd_data(A.dz[l], P + L.off[2 * l], dx, B, cin, C, S, st);
      dpool = dx;
    }
    S *= 2;
  }
}

}  // namespace
}  // namespace dgd

struct dgd_surrogate {
  dgd::Layout L;
  int M = 0;
  std::vector<float*> P, Gd, Mm, Vm;   // per member: params, grads, Adam moments
  std::vector<int64_t> steps;
  hipStream_t st = nullptr;
};

using namespace dgd;

namespace {

template <typename F>
int sguard(F&& f) {
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
  }
}

[[noreturn]] void sfail(int code, const std::string& m) { throw Error{code, m}; }

// Device copies of a dataset.
struct Dataset {
  uint8_t* img = nullptr;
  double* ld = nullptr;
  double* tg = nullptr;
  void upload(const uint8_t* i, const double* l, const double* t, int n) {
    DGD_HIP_CHECK(hipMalloc(&img, (size_t)n * IMG * IMG));
    DGD_HIP_CHECK(hipMemcpy(img, i, (size_t)n * IMG * IMG, hipMemcpyHostToDevice));
    DGD_HIP_CHECK(hipMalloc(&ld, (size_t)n * 8));
    DGD_HIP_CHECK(hipMemcpy(ld, l, (size_t)n * 8, hipMemcpyHostToDevice));
    if (t) {
      DGD_HIP_CHECK(hipMalloc(&tg, (size_t)n * 24));
      DGD_HIP_CHECK(hipMemcpy(tg, t, (size_t)n * 24, hipMemcpyHostToDevice));
    }
  }
  ~Dataset() {
    (void)hipFree(img);
    (void)hipFree(ld);
    (void)hipFree(tg);
  }
};

void check_inputs(const uint8_t* images, const double* logd, int n) {
  if (!images || !logd || n < 1) sfail(DGD_EINVAL, "bad images / log Delta / count");
  for (int64_t k = 0; k < (int64_t)n * IMG * IMG; ++k)
    if (images[k] > 1) sfail(DGD_EINVAL, "images must hold 0 or 1");
  for (int k = 0; k < n; ++k)
    if (!std::isfinite(logd[k])) sfail(DGD_EINVAL, "log Delta must be finite");
}

}  // namespace

extern "C" {

int dgd_surrogate_create(int32_t n_members, int32_t channels, int32_t hidden, uint64_t seed,
                         dgd_surrogate** out) {
  return sguard([&]() -> int {
    if (!out) sfail(DGD_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_members < 1 || n_members > 64) sfail(DGD_EINVAL, "n_members must be in [1, 64]");
    if (channels < 1 || channels > MAXC) sfail(DGD_EINVAL, "channels must be in [1, 32]");
    if (hidden < 1 || hidden > 4096) sfail(DGD_EINVAL, "hidden must be in [1, 4096]");
    auto* s = new dgd_surrogate();
    try {
      s->L.build(channels, hidden);
      s->M = n_members;
      DGD_HIP_CHECK(hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking));
      for (int m = 0; m < n_members; ++m) {
        // He-uniform weights from a per-member seeded generator, zero biases
        std::mt19937_64 rng(seed + 7919ull * (uint64_t)m);
        std::vector<float> p(s->L.total, 0.f);
        for (int k = 0; k < 16; k += 2) {
          const int64_t n = s->L.size[k];
          const int64_t rows = (k < 8) ? s->L.C : (k < 14 ? s->L.H : 3);
          const double lim = std::sqrt(6.0 / (double)(n / rows));
          std::uniform_real_distribution<double> U(-lim, lim);
          for (int64_t i = 0; i < n; ++i) p[s->L.off[k] + i] = (float)U(rng);
        }
        float *P, *G, *Mm, *Vm;
        DGD_HIP_CHECK(hipMalloc(&P, s->L.total * 4));
        DGD_HIP_CHECK(hipMalloc(&G, s->L.total * 4));
        DGD_HIP_CHECK(hipMalloc(&Mm, s->L.total * 4));
        DGD_HIP_CHECK(hipMalloc(&Vm, s->L.total * 4));
        s->P.push_back(P);
        s->Gd.push_back(G);
        s->Mm.push_back(Mm);
        s->Vm.push_back(Vm);
        s->steps.push_back(0);
        DGD_HIP_CHECK(hipMemcpy(P, p.data(), s->L.total * 4, hipMemcpyHostToDevice));
        DGD_HIP_CHECK(hipMemset(Mm, 0, s->L.total * 4));
        DGD_HIP_CHECK(hipMemset(Vm, 0, s->L.total * 4));
      }
    } catch (...) {
      dgd_surrogate_destroy(s);
      throw;
    }
    *out = s;
    return DGD_OK;
  });
}

int dgd_surrogate_n_params(const dgd_surrogate* s, int64_t* n) {
  return sguard([&]() -> int {
    if (!s || !n) sfail(DGD_EINVAL, "NULL argument");
    *n = s->L.total;
    return DGD_OK;
  });
}

int dgd_surrogate_get_params(const dgd_surrogate* s, int32_t member, float* host_out) {
  return sguard([&]() -> int {
    if (!s || !host_out || member < 0 || member >= s->M) sfail(DGD_EINVAL, "bad argument");
    DGD_HIP_CHECK(hipMemcpy(host_out, s->P[member], s->L.total * 4, hipMemcpyDeviceToHost));
    return DGD_OK;
  });
}

int dgd_surrogate_set_params(dgd_surrogate* s, int32_t member, const float* host_in) {
  return sguard([&]() -> int {
    if (!s || !host_in || member < 0 || member >= s->M) sfail(DGD_EINVAL, "bad argument");
    DGD_HIP_CHECK(hipMemcpy(s->P[member], host_in, s->L.total * 4, hipMemcpyHostToDevice));
    return DGD_OK;
  });
}

int dgd_surrogate_loss_grad(dgd_surrogate* s, int32_t member, const uint8_t* images,
                            const double* log_deltas, const double* targets, int32_t n,
                            double* loss_out, float* grad_out) {
  return sguard([&]() -> int {
    if (!s || member < 0 || member >= s->M || !targets) sfail(DGD_EINVAL, "bad argument");
    check_inputs(images, log_deltas, n);
    if (n > 4096) sfail(DGD_EINVAL, "at most 4096 samples per call");
    Dataset ds;
    ds.upload(images, log_deltas, targets, n);
    Acts A;
    try {
      A.build(n, s->L);
      std::vector<int> idx(n);
      for (int k = 0; k < n; ++k) idx[k] = k;
      DGD_HIP_CHECK(hipMemcpyAsync(A.idx, idx.data(), n * 4, hipMemcpyHostToDevice, s->st));
      k_gather<<<nblk((int64_t)n * IMG * IMG), 256, 0, s->st>>>(ds.img, ds.ld, A.idx, n, A.x, A.ld);
      forward(s->L, s->P[member], A, s->st);
      k_mse<<<nblk(n), 256, 0, s->st>>>(A.out, ds.tg, A.idx, n, A.dout, A.se);
      backward(s->L, s->P[member], s->Gd[member], A, s->st);
      DGD_HIP_CHECK(hipGetLastError());
      std::vector<float> se(n);
      DGD_HIP_CHECK(hipMemcpyAsync(se.data(), A.se, n * 4, hipMemcpyDeviceToHost, s->st));
      if (grad_out)
        DGD_HIP_CHECK(hipMemcpyAsync(grad_out, s->Gd[member], s->L.total * 4, hipMemcpyDeviceToHost, s->st));
      DGD_HIP_CHECK(hipStreamSynchronize(s->st));
      double l = 0;
      for (float v : se) l += v;
      if (loss_out) *loss_out = l / (3.0 * n);
    } catch (...) {
      A.release();
      throw;
    }
    A.release();
    return DGD_OK;
  });
}

int dgd_surrogate_train(dgd_surrogate* s, const uint8_t* images, const double* log_deltas,
                        const double* targets, int32_t n, int32_t epochs, int32_t batch, double lr,
                        uint64_t shuffle_seed, double* epoch_loss_out) {
  return sguard([&]() -> int {
    if (!s || !targets || epochs < 0 || batch < 1 || batch > 4096 || !(lr > 0))
      sfail(DGD_EINVAL, "bad argument");
    check_inputs(images, log_deltas, n);
    Dataset ds;
    ds.upload(images, log_deltas, targets, n);
    const int B = std::min<int>(batch, n);
    Acts A;
    try {
      A.build(B, s->L);
      for (int m = 0; m < s->M; ++m) {
        std::mt19937_64 rng(shuffle_seed + 104729ull * (uint64_t)m);
        std::vector<int> perm(n);
        for (int e = 0; e < epochs; ++e) {
          for (int k = 0; k < n; ++k) perm[k] = k;
          std::shuffle(perm.begin(), perm.end(), rng);
          double esum = 0;
          int64_t ecount = 0;
          std::vector<float> se(B);
          for (int b0 = 0; b0 + B <= n; b0 += B) {   // full batches only
            DGD_HIP_CHECK(hipMemcpyAsync(A.idx, perm.data() + b0, B * 4, hipMemcpyHostToDevice, s->st));
            k_gather<<<nblk((int64_t)B * IMG * IMG), 256, 0, s->st>>>(ds.img, ds.ld, A.idx, B, A.x, A.ld);
            forward(s->L, s->P[m], A, s->st);
            k_mse<<<nblk(B), 256, 0, s->st>>>(A.out, ds.tg, A.idx, B, A.dout, A.se);
            backward(s->L, s->P[m], s->Gd[m], A, s->st);
            const int64_t t = ++s->steps[m];
            const float b1 = 0.9f, b2 = 0.999f;
            k_adam<<<nblk(s->L.total), 256, 0, s->st>>>(s->P[m], s->Gd[m], s->Mm[m], s->Vm[m], s->L.total,
                                                        (float)lr, b1, b2, 1e-8f,
                                                        (float)(1.0 - std::pow(0.9, (double)t)),
                                                        (float)(1.0 - std::pow(0.999, (double)t)));
            DGD_HIP_CHECK(hipMemcpyAsync(se.data(), A.se, B * 4, hipMemcpyDeviceToHost, s->st));
            DGD_HIP_CHECK(hipStreamSynchronize(s->st));
            for (float v : se) esum += v;
            ecount += B;
          }
          DGD_HIP_CHECK(hipGetLastError());
          if (epoch_loss_out) epoch_loss_out[(int64_t)m * epochs + e] = esum / (3.0 * std::max<int64_t>(ecount, 1));
        }
      }
    } catch (...) {
      A.release();
      throw;
    }
    A.release();
    return DGD_OK;
  });
}

int dgd_surrogate_predict(dgd_surrogate* s, const uint8_t* images, const double* log_deltas, int32_t n,
                          double threshold, double* mean_out, double* spread_out, uint8_t* fallback_out) {
  return sguard([&]() -> int {
    if (!s || !mean_out) sfail(DGD_EINVAL, "bad argument");
    check_inputs(images, log_deltas, n);
    Dataset ds;
    ds.upload(images, log_deltas, nullptr, n);
    const int B = std::min<int>(4096, n);
    Acts A;
    float* outs = nullptr;
    double *dmean = nullptr, *dspread = nullptr;
    uint8_t* dflag = nullptr;
    auto cleanup = [&]() {
      A.release();
      (void)hipFree(outs);
      (void)hipFree(dmean);
      (void)hipFree(dspread);
      (void)hipFree(dflag);
    };
    try {
      A.build(B, s->L);
      DGD_HIP_CHECK(hipMalloc(&outs, (size_t)s->M * n * 3 * 4));
      DGD_HIP_CHECK(hipMalloc(&dmean, (size_t)n * 24));
      DGD_HIP_CHECK(hipMalloc(&dspread, (size_t)n * 8));
      DGD_HIP_CHECK(hipMalloc(&dflag, (size_t)n));
      std::vector<int> idx(B);
      for (int b0 = 0; b0 < n; b0 += B) {
        const int nb = std::min(B, n - b0);
        for (int k = 0; k < nb; ++k) idx[k] = b0 + k;
        for (int k = nb; k < B; ++k) idx[k] = b0;   // pad the last batch
        DGD_HIP_CHECK(hipMemcpyAsync(A.idx, idx.data(), B * 4, hipMemcpyHostToDevice, s->st));
        k_gather<<<nblk((int64_t)B * IMG * IMG), 256, 0, s->st>>>(ds.img, ds.ld, A.idx, B, A.x, A.ld);
        for (int m = 0; m < s->M; ++m) {
          forward(s->L, s->P[m], A, s->st);
          DGD_HIP_CHECK(hipMemcpyAsync(outs + ((int64_t)m * n + b0) * 3, A.out, (size_t)nb * 12,
                                       hipMemcpyDeviceToDevice, s->st));
        }
        DGD_HIP_CHECK(hipStreamSynchronize(s->st));   // idx is reused
      }
      k_ensemble<<<nblk(n), 256, 0, s->st>>>(outs, s->M, n, (float)threshold, dmean, dspread, dflag);
      DGD_HIP_CHECK(hipGetLastError());
      DGD_HIP_CHECK(hipMemcpyAsync(mean_out, dmean, (size_t)n * 24, hipMemcpyDeviceToHost, s->st));
      std::vector<double> sp(n);
      std::vector<uint8_t> fl(n);
      DGD_HIP_CHECK(hipMemcpyAsync(sp.data(), dspread, (size_t)n * 8, hipMemcpyDeviceToHost, s->st));
      DGD_HIP_CHECK(hipMemcpyAsync(fl.data(), dflag, (size_t)n, hipMemcpyDeviceToHost, s->st));
      DGD_HIP_CHECK(hipStreamSynchronize(s->st));
      if (spread_out) std::memcpy(spread_out, sp.data(), (size_t)n * 8);
      if (fallback_out) std::memcpy(fallback_out, fl.data(), (size_t)n);
    } catch (...) {
      cleanup();
      throw;
    }
    cleanup();
    return DGD_OK;
  });
}

void dgd_surrogate_destroy(dgd_surrogate* s) {
  if (!s) return;
  for (auto* p : s->P) (void)hipFree(p);
  for (auto* p : s->Gd) (void)hipFree(p);
  for (auto* p : s->Mm) (void)hipFree(p);
  for (auto* p : s->Vm) (void)hipFree(p);
  if (s->st) (void)hipStreamDestroy(s->st);
  delete s;
}

}  // extern "C"
