// Training of the outflow MLP 27 -> 64 -> 64 -> 3 on gfx950 (C ABI of
// include/lbm_train.h).
//
// Sec. 3.1, Eq. 17: the network is fitted by the mean squared error of the
// reconstructed unknown populations.  One optimiser step is two launches:
//
//   k_train_tile    one workgroup per 64 samples: gather and standardise the
//                   rows, forward pass (MFMA 16x16x32 BF16, FP32 tanh), loss,
//                   backward pass (MFMA for every product contracted over
//                   units or over samples), per-tile FP32 gradient sums;
//   k_train_update  32 parameters per workgroup: FP64 sum of the tile gradients
//                   in a fixed order (eight tile groups, each in tile order),
//                   Adam on the FP32 master weight, refresh of
//                   the BF16 copies the next forward pass reads.
//
// LDS holds every activation twice, row-major [sample][unit] (A operand of
// the next layer) and transposed [unit][sample] (operands of the
// weight-gradient products, which contract over samples), so every MFMA
// operand is 8 consecutive BF16 per lane.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/lbm_train.h"
#include "d2q9_dev.hpp"
#include "lbm_internal.hpp"
#include "mlp_dev.hpp"

namespace lbm {
namespace {

constexpr int kNP = 6147;
constexpr int kOffW1 = 0, kOffB1 = 64 * 27, kOffW2 = kOffB1 + 64, kOffB2 = kOffW2 + 64 * 64,
              kOffW3 = kOffB2 + 64, kOffB3 = kOffW3 + 3 * 64;
static_assert(kOffB3 + 3 == kNP, "parameter count");
constexpr int kTS = 64;                 // samples per workgroup
constexpr int kP = 72;                  // LDS pitch (BF16) of 64-wide rows
constexpr int kPartStride = kNP + 1;    // gradient sums + loss sum per tile
constexpr int kStatCols = 30;           // 27 inputs + 3 targets
constexpr int kStatBlocks = 256;
constexpr int kUpdBlocks = (kNP + 1 + 31) / 32;   // 32 parameters (and the loss) per workgroup

struct TrainState {
  float w[kNP], m[kNP], v[kNP];   // FP32 masters and Adam moments
  uint16_t w1b[64 * 32];          // BF16 [out][in], in padded to 32
  uint16_t w2b[64 * 64];          // BF16 [out][in]
  uint16_t w2t[64 * 64];          // BF16 [in][out]
  uint16_t w3b[16 * 64];          // BF16 [out][in], out padded to 16
  float mu[32], inv_sd[32];       // input standardisation (27 used)
  float mu_out[4], inv_sd_out[4]; // target standardisation (3 used)
  double loss;
  double mean[kStatCols], sd[kStatCols];
};

struct TrainArgs {
  TrainState* st;
  const float* x;
  const float* t;
  int64_t n;
  const int32_t* rows;   // explicit rows, or null: draw them
  uint64_t seed;
  int64_t step;
  int batch;
  float* part;           // [tiles][kPartStride]
  float gscale;          // d(loss)/d(o) factor 2 / (3 batch)
};

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__host__ __device__ inline int32_t sample_row(uint64_t seed, int64_t step, int batch, int j,
                                              int64_t n) {
  const uint64_t r = splitmix64_at(seed, uint64_t(step) * uint64_t(batch) + uint64_t(j) + 1ull);
  return int32_t(((r >> 32) * uint64_t(n)) >> 32);
}

// C tile = A[m0:m0+16, 0:K] * B[0:K, n0:n0+16] with A row-major (pitch pa)
// and B given transposed (BT row n holds column n of B, pitch pb).  Lane l
// gets C[m0 + 4 (l/16) + i][n0 + l%16], i = 0..3.
__device__ __forceinline__ f32x4_t mm_tile(const uint16_t* A, int pa, int m0, const uint16_t* BT,
                                           int pb, int n0, int K) {
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 32)
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(load8(A + (m0 + r) * pa + k0 + 8 * g),
                                                  load8(BT + (n0 + r) * pb + k0 + 8 * g), acc,
                                                  0, 0, 0);
  return acc;
}

struct alignas(16) TrainLds {
  uint16_t X[kTS * 32];       // standardised inputs [sample][feature]
  uint16_t XT[32 * kP];       // [feature][sample]
  uint16_t H1[kTS * kP], H1T[64 * kP], H2[kTS * kP], H2T[64 * kP];
  float D1[kTS * 64], D2[kTS * 64];   // tanh' = 1 - h^2
  float O[kTS * 4], Y[kTS * 4];       // outputs (then dL/do) and targets
  uint16_t DOT[16 * kP];              // (dL/do)^T, rows 3..15 zero
  uint16_t DZ2[kTS * kP], DZ2T[64 * kP], DZ1T[64 * kP];
  float DZ[kTS * 65];                 // FP32 dL/dz of layer 2, then layer 1
  float red[4];
  int32_t rows[kTS];
};

__device__ __forceinline__ void store4_bf16(uint16_t* p, const uint16_t h[4]) {
  uint2 v;
  v.x = uint32_t(h[0]) | (uint32_t(h[1]) << 16);
  v.y = uint32_t(h[2]) | (uint32_t(h[3]) << 16);
  *reinterpret_cast<uint2*>(p) = v;
}

// Forward hidden layer on this wave's 16 samples: H = tanh(A W^T + b).
__device__ __forceinline__ void fwd_hidden(const uint16_t* A, int pa, const uint16_t* W, int kin,
                                           const float* bias, uint16_t* H, uint16_t* HT,
                                           float* D, int m0) {
  const int lane = threadIdx.x & 63, r16 = lane & 15, grp = lane >> 4;
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const f32x4_t c = mm_tile(A, pa, m0, W, kin, 16 * nt, kin);
    const int u = 16 * nt + r16;
    const float b = bias[u];
    uint16_t hb[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int s = m0 + 4 * grp + i;
      const float h = tanhf(c[i] + b);
      D[s * 64 + u] = 1.f - h * h;
      hb[i] = f32_to_bf16(h);
      H[s * kP + u] = hb[i];
    }
    store4_bf16(&HT[u * kP + m0 + 4 * grp], hb);
  }
}

__global__ void __launch_bounds__(kBlock) k_train_tile(const TrainArgs a) {
  __shared__ TrainLds L;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r16 = lane & 15, grp = lane >> 4;
  const int m0 = 16 * wave;                       // this wave's samples
  const TrainState* __restrict__ st = a.st;
  float* __restrict__ part = a.part + int64_t(blockIdx.x) * kPartStride;

  if (tid < kTS) {
    const int j = blockIdx.x * kTS + tid;
    L.rows[tid] = a.rows ? a.rows[j] : sample_row(a.seed, a.step, a.batch, j, a.n);
  }
  for (int i = tid; i < 13 * kP; i += kBlock) L.DOT[3 * kP + i] = 0;
  __syncthreads();

  // 1. standardised inputs (BF16, both layouts) and targets (FP32)
  for (int i = tid; i < kTS * 32; i += kBlock) {
    const int s = i >> 5, f = i & 31;
    uint16_t z = 0;
    if (f < 27) z = f32_to_bf16((a.x[int64_t(L.rows[s]) * 27 + f] - st->mu[f]) * st->inv_sd[f]);
    L.X[s * 32 + f] = z;
    L.XT[f * kP + s] = z;
  }
  if (tid < kTS * 3) {
    const int s = tid / 3, k = tid - 3 * s;
    L.Y[s * 4 + k] = (a.t[int64_t(L.rows[s]) * 3 + k] - st->mu_out[k]) * st->inv_sd_out[k];
  }
  __syncthreads();

  // 2. forward
  fwd_hidden(L.X, 32, st->w1b, 32, st->w + kOffB1, L.H1, L.H1T, L.D1, m0);
  __syncthreads();
  fwd_hidden(L.H1, kP, st->w2b, 64, st->w + kOffB2, L.H2, L.H2T, L.D2, m0);
  __syncthreads();
  {
    const f32x4_t c = mm_tile(L.H2, kP, m0, st->w3b, 64, 0, 64);
    if (r16 < 3) {
#pragma unroll
      for (int i = 0; i < 4; ++i) L.O[(m0 + 4 * grp + i) * 4 + r16] = c[i] + st->w[kOffB3 + r16];
    }
  }
  __syncthreads();

  // 3. loss and dL/do
  float e2 = 0.f;
  if (tid < kTS * 3) {
    const int s = tid / 3, k = tid - 3 * s;
    const float e = L.O[s * 4 + k] - L.Y[s * 4 + k];
    e2 = e * e;
    const float d = a.gscale * e;
    L.O[s * 4 + k] = d;
    L.DOT[k * kP + s] = f32_to_bf16(d);
  }
  e2 = wave_sum_f(e2);
  if (lane == 0) L.red[wave] = e2;
  __syncthreads();
  if (tid == 0) part[kNP] = ((L.red[0] + L.red[1]) + L.red[2]) + L.red[3];

  // 4. layer 3: dW3 = (dL/do)^T H2, db3, and dL/dz2 = (dL/do W3) * tanh'
  {
    const f32x4_t c = mm_tile(L.DOT, kP, 0, L.H2T, kP, 16 * wave, 64);
    const int u = 16 * wave + r16;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int o = 4 * grp + i;
      if (o < 3) part[kOffW3 + o * 64 + u] = c[i];
    }
  }
  if (tid < 3) {
    float sb = 0.f;
    for (int s = 0; s < kTS; ++s) sb += L.O[s * 4 + tid];
    part[kOffB3 + tid] = sb;
  }
  {
    const int s = tid >> 2, j0 = (tid & 3) * 16;
    const float d0 = L.O[s * 4 + 0], d1 = L.O[s * 4 + 1], d2 = L.O[s * 4 + 2];
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
      const int j = j0 + jj;
      const float dh = d0 * st->w[kOffW3 + j] + d1 * st->w[kOffW3 + 64 + j] +
                       d2 * st->w[kOffW3 + 128 + j];
      const float dz = dh * L.D2[s * 64 + j];
      L.DZ[s * 65 + j] = dz;
      const uint16_t b = f32_to_bf16(dz);
      L.DZ2[s * kP + j] = b;
      L.DZ2T[j * kP + s] = b;
    }
  }
  __syncthreads();

  // 5. layer 2: dW2 = dz2^T H1, db2, then dL/dh1 = dz2 W2
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const f32x4_t c = mm_tile(L.DZ2T, kP, m0, L.H1T, kP, 16 * nt, 64);
#pragma unroll
    for (int i = 0; i < 4; ++i) part[kOffW2 + (m0 + 4 * grp + i) * 64 + 16 * nt + r16] = c[i];
  }
  if (tid < 64) {
    float sb = 0.f;
    for (int s = 0; s < kTS; ++s) sb += L.DZ[s * 65 + tid];
    part[kOffB2 + tid] = sb;
  }
  __syncthreads();
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const f32x4_t c = mm_tile(L.DZ2, kP, m0, st->w2t, 64, 16 * nt, 64);
    const int u = 16 * nt + r16;
    uint16_t hb[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int s = m0 + 4 * grp + i;
      const float dz = c[i] * L.D1[s * 64 + u];
      L.DZ[s * 65 + u] = dz;
      hb[i] = f32_to_bf16(dz);
    }
    store4_bf16(&L.DZ1T[u * kP + m0 + 4 * grp], hb);
  }
  __syncthreads();

  // 6. layer 1: dW1 = dz1^T X, db1
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    const f32x4_t c = mm_tile(L.DZ1T, kP, m0, L.XT, kP, 16 * nt, 64);
    const int f = 16 * nt + r16;
    if (f < 27) {
#pragma unroll
      for (int i = 0; i < 4; ++i) part[kOffW1 + (m0 + 4 * grp + i) * 27 + f] = c[i];
    }
  }
  if (tid < 64) {
    float sb = 0.f;
    for (int s = 0; s < kTS; ++s) sb += L.DZ[s * 65 + tid];
    part[kOffB1 + tid] = sb;
  }
}

__device__ __forceinline__ void refresh_bf16(TrainState* st, int p) {
  const uint16_t b = f32_to_bf16(st->w[p]);
  if (p < kOffB1) {
    const int j = p / 27, f = p - 27 * j;
    st->w1b[j * 32 + f] = b;
  } else if (p >= kOffW2 && p < kOffB2) {
    const int q = p - kOffW2, j = q >> 6, i = q & 63;
    st->w2b[j * 64 + i] = b;
    st->w2t[i * 64 + j] = b;
  } else if (p >= kOffW3 && p < kOffB3) {
    st->w3b[p - kOffW3] = b;
  }
}

struct UpdateArgs {
  TrainState* st;
  const float* part;
  int tiles;
  float* grad;        // gradient mode: write the summed gradient here, no update
  float lr, beta1, beta2, eps, c1, c2;   // c1 = 1/(1-beta1^t), c2 = 1/(1-beta2^t)
  double loss_scale;  // 1 / (3 batch)
};

// 32 parameters per workgroup (index kNP is the loss), eight groups of tiles
// per parameter: thread (i, k) sums tiles k, k + 8, ... of parameter i in
// FP64 with its loads issued together, and the eight sums are added in
// group order (a fixed order; one thread per parameter walking all tiles in
// turn took 20.3 us per step, a chain of dependent loads).
constexpr int kUpdParams = 32, kUpdGroups = kBlock / kUpdParams;
__global__ void __launch_bounds__(kBlock) k_train_update(const UpdateArgs a) {
  __shared__ double red[kUpdGroups][kUpdParams];
  const int i = threadIdx.x % kUpdParams, k = threadIdx.x / kUpdParams;
  const int p = blockIdx.x * kUpdParams + i;
  double s = 0.0;
  if (p <= kNP) {
    for (int t0 = k; t0 < a.tiles; t0 += 8 * kUpdGroups) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int t = t0 + u * kUpdGroups;
        v[u] = t < a.tiles ? a.part[int64_t(t) * kPartStride + p] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) s += double(v[u]);
    }
  }
  red[k][i] = s;
  __syncthreads();
  if (k != 0 || p > kNP) return;
  double g = 0.0;
  for (int j = 0; j < kUpdGroups; ++j) g += red[j][i];
  if (p == kNP) {
    a.st->loss = g * a.loss_scale;
    return;
  }
  const float gf = float(g);
  if (a.grad) {
    a.grad[p] = gf;
  } else {
    TrainState* st = a.st;
    const float m = a.beta1 * st->m[p] + (1.f - a.beta1) * gf;
    const float v = a.beta2 * st->v[p] + (1.f - a.beta2) * gf * gf;
    st->m[p] = m;
    st->v[p] = v;
    st->w[p] -= a.lr * (m * a.c1) / (sqrtf(v * a.c2) + a.eps);
    refresh_bf16(st, p);
  }
}

// Column statistics of the data (mean, standard deviation), FP64, fixed order.
__global__ void __launch_bounds__(kBlock) k_stats_partial(const float* x, const float* t, int64_t n,
                                                          double* part) {
  __shared__ double red[8][32][2];
  const int c = threadIdx.x & 31, ro = threadIdx.x >> 5;
  const int64_t per = (n + kStatBlocks - 1) / kStatBlocks;
  const int64_t r0 = blockIdx.x * per, r1 = r0 + per < n ? r0 + per : n;
  double s = 0.0, s2 = 0.0;
  if (c < kStatCols) {
    for (int64_t r = r0 + ro; r < r1; r += 8) {
      const double v = c < 27 ? double(x[r * 27 + c]) : double(t[r * 3 + (c - 27)]);
      s += v;
      s2 += v * v;
    }
  }
  red[ro][c][0] = s;
  red[ro][c][1] = s2;
  __syncthreads();
  if (threadIdx.x < kStatCols) {
    double a = 0.0, b = 0.0;
    for (int k = 0; k < 8; ++k) {
      a += red[k][threadIdx.x][0];
      b += red[k][threadIdx.x][1];
    }
    part[(blockIdx.x * kStatCols + threadIdx.x) * 2] = a;
    part[(blockIdx.x * kStatCols + threadIdx.x) * 2 + 1] = b;
  }
}

__global__ void __launch_bounds__(kBlock) k_stats_final(TrainState* st, const double* part,
                                                        int64_t n) {
  const int c = threadIdx.x;
  if (c >= kStatCols) return;
  double s = 0.0, s2 = 0.0;
  for (int b = 0; b < kStatBlocks; ++b) {
    s += part[(b * kStatCols + c) * 2];
    s2 += part[(b * kStatCols + c) * 2 + 1];
  }
  const double mean = s / double(n);
  const double var = fmax(s2 / double(n) - mean * mean, 0.0);
  double sd = sqrt(var);
  if (!(sd > 1e-12)) sd = 1.0;          // constant column: leave it unscaled
  st->mean[c] = mean;
  st->sd[c] = sd;
  // FP32 mean and sd, reciprocal in FP32: the same maps the inference path
  // builds from the exported weights
  if (c < 27) {
    st->mu[c] = float(mean);
    st->inv_sd[c] = 1.0f / float(sd);
  } else {
    st->mu_out[c - 27] = float(mean);
    st->inv_sd_out[c - 27] = 1.0f / float(sd);
  }
}

__global__ void k_sample_rows(int32_t* rows, uint64_t seed, int64_t step, int batch, int64_t n) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j < batch) rows[j] = sample_row(seed, step, batch, j, n);
}

uint16_t host_bf16(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return 0x7FC0;
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace
}  // namespace lbm

using namespace lbm;

struct lbm_trainer {
  lbm_train_params p;
  hipStream_t stream;
  TrainState* st;
  float* part;
  double* stat_part;
  float* grad;
  int32_t* rows;
  const float* x;
  const float* t;
  int64_t n;
  int64_t steps;   // optimiser steps taken
  bool weights;
};

#define TRY_HIP(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return set_error(LBM_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

namespace {
struct TrainLayout {
  size_t st, part, stat, grad, rows, total;
};
TrainLayout train_layout(const lbm_train_params& p) {
  TrainLayout L{};
  size_t o = 0;
  auto take = [&](size_t b) {
    size_t at = o;
    o = align256(o + b);
    return at;
  };
  const int tiles = std::max(p.batch, 64) / kTS;
  L.st = take(sizeof(TrainState));
  L.part = take(size_t(std::max(tiles, 1024)) * kPartStride * 4);  // >= gradient batches of 65536
  L.stat = take(size_t(kStatBlocks) * kStatCols * 2 * 8);
  L.grad = take(size_t(kNP) * 4);
  L.rows = take(size_t(65536) * 4);
  L.total = o;
  return L;
}

lbm_status check_train_params(const lbm_train_params* p) {
  if (!p) return set_error(LBM_EINVAL, "params is NULL");
  if (p->batch < 64 || p->batch > 65536 || p->batch % 64)
    return set_error(LBM_EINVAL, "batch must be a multiple of 64 in [64, 65536] (got %d)", p->batch);
  if (!(p->lr > 0) || !(p->beta1 >= 0 && p->beta1 < 1) || !(p->beta2 >= 0 && p->beta2 < 1) ||
      !(p->eps > 0))
    return set_error(LBM_EINVAL, "bad Adam parameters");
  return LBM_OK;
}

lbm_status run_tiles(lbm_trainer* tr, const int32_t* rows, int nrows, int64_t step) {
  TrainArgs a{};
  a.st = tr->st;
  a.x = tr->x;
  a.t = tr->t;
  a.n = tr->n;
  a.rows = rows;
  a.seed = tr->p.seed;
  a.step = step;
  a.batch = nrows;
  a.part = tr->part;
  a.gscale = float(2.0 / (3.0 * nrows));
  hipLaunchKernelGGL(k_train_tile, dim3(nrows / kTS), dim3(kBlock), 0, tr->stream, a);
  TRY_HIP(hipGetLastError());
  return LBM_OK;
}
// ---- the entry point that allocates nothing -------------------------------
// lbm_mlp_gradient_noalloc runs the gradient kernels of lbm_train_gradient
// with their state (weights image and standardisation), per-tile partial
// sums and summed gradient in this file-scope device array instead of a
// caller workspace.  Every GPU holds its own copy at its own address, looked
// up once per device with hipGetSymbolAddress; host code uses only that
// address, never the array's name.
constexpr int kNoallocMaxRows = 4096;
constexpr size_t kNoallocState = (sizeof(TrainState) + 255) / 256 * 256;
constexpr size_t kNoallocPart = size_t(kNoallocMaxRows / kTS) * kPartStride * 4;
constexpr size_t kNoallocGrad = size_t(kNP) * 4;
constexpr size_t kNoallocBytes = size_t(2) << 20;    // 2 MiB per GPU
static_assert(kNoallocState + (kNoallocPart + 255) / 256 * 256 + kNoallocGrad <= kNoallocBytes,
              "scratch layout");
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// Device address of the current device's scratch array (looked up once).
lbm_status scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(LBM_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return set_error(LBM_EINVAL, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return set_error(LBM_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return LBM_OK;
}

// Host image of the state a gradient pass reads: FP32 masters, BF16 copies
// and the standardisation maps (one per host thread: calls from several
// threads build their images apart; on one GPU they still share the device
// scratch).
thread_local TrainState g_noalloc_image;

}  // namespace

extern "C" {

size_t lbm_train_workspace_bytes(const lbm_train_params* p) {
  if (check_train_params(p) != LBM_OK) return 0;
  return train_layout(*p).total;
}

lbm_status lbm_train_create(const lbm_train_params* p, void* ws, size_t bytes, lbm_trainer** out) {
  if (!out) return set_error(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  lbm_status st = check_train_params(p);
  if (st) return st;
  if (!ws || reinterpret_cast<uintptr_t>(ws) % 256)
    return set_error(LBM_EINVAL, "workspace must be non-NULL and 256-byte aligned");
  const TrainLayout L = train_layout(*p);
  if (bytes < L.total) return set_error(LBM_ENOSPACE, "workspace has %zu bytes, needs %zu", bytes, L.total);
  lbm_trainer* tr = new lbm_trainer();
  tr->p = *p;
  tr->stream = static_cast<hipStream_t>(p->stream);
  char* base = static_cast<char*>(ws);
  tr->st = reinterpret_cast<TrainState*>(base + L.st);
  tr->part = reinterpret_cast<float*>(base + L.part);
  tr->stat_part = reinterpret_cast<double*>(base + L.stat);
  tr->grad = reinterpret_cast<float*>(base + L.grad);
  tr->rows = reinterpret_cast<int32_t*>(base + L.rows);
  hipError_t e = hipMemsetAsync(tr->st, 0, sizeof(TrainState), tr->stream);
  if (e != hipSuccess) {
    delete tr;
    return set_error(LBM_EHIP, "hipMemsetAsync: %s", hipGetErrorString(e));
  }
  *out = tr;
  return LBM_OK;
}

lbm_status lbm_train_destroy(lbm_trainer* t) {
  if (t) (void)hipStreamSynchronize(t->stream);
  delete t;
  return LBM_OK;
}

lbm_status lbm_train_set_data(lbm_trainer* tr, const float* x, const float* t, int64_t n) {
  if (!tr || !x || !t) return set_error(LBM_EINVAL, "NULL argument");
  if (n < 2 || n >= (int64_t(1) << 31)) return set_error(LBM_EINVAL, "need 2 <= n < 2^31 samples");
  tr->x = x;
  tr->t = t;
  tr->n = n;
  hipLaunchKernelGGL(k_stats_partial, dim3(kStatBlocks), dim3(kBlock), 0, tr->stream, x, t, n,
                     tr->stat_part);
  TRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(kBlock), 0, tr->stream, tr->st, tr->stat_part, n);
  TRY_HIP(hipGetLastError());
  return LBM_OK;
}

lbm_status lbm_train_set_weights(lbm_trainer* tr, const lbm_mlp* w) {
  if (!tr || !w || !w->w1 || !w->b1 || !w->w2 || !w->b2 || !w->w3 || !w->b3)
    return set_error(LBM_EINVAL, "NULL argument");
  if (w->n_in != 27 || w->n_h1 != 64 || w->n_h2 != 64 || w->n_out != 3)
    return set_error(LBM_EINVAL, "network must be 27-64-64-3");
  // masters, zero moments and BF16 copies: the leading part of TrainState
  const size_t head = offsetof(TrainState, mu);
  std::vector<char> buf(head, 0);
  TrainState* h = reinterpret_cast<TrainState*>(buf.data());
  memcpy(h->w + kOffW1, w->w1, 64 * 27 * 4);
  memcpy(h->w + kOffB1, w->b1, 64 * 4);
  memcpy(h->w + kOffW2, w->w2, 64 * 64 * 4);
  memcpy(h->w + kOffB2, w->b2, 64 * 4);
  memcpy(h->w + kOffW3, w->w3, 3 * 64 * 4);
  memcpy(h->w + kOffB3, w->b3, 3 * 4);
  for (int j = 0; j < 64; ++j)
    for (int f = 0; f < 27; ++f) h->w1b[j * 32 + f] = host_bf16(w->w1[j * 27 + f]);
  for (int j = 0; j < 64; ++j)
    for (int i = 0; i < 64; ++i) {
      h->w2b[j * 64 + i] = host_bf16(w->w2[j * 64 + i]);
      h->w2t[i * 64 + j] = host_bf16(w->w2[j * 64 + i]);
    }
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 64; ++i) h->w3b[k * 64 + i] = host_bf16(w->w3[k * 64 + i]);
  TRY_HIP(hipMemcpyAsync(tr->st, h, head, hipMemcpyHostToDevice, tr->stream));
  TRY_HIP(hipStreamSynchronize(tr->stream));
  tr->steps = 0;
  tr->weights = true;
  return LBM_OK;
}

lbm_status lbm_train_step(lbm_trainer* tr, int64_t nsteps) {
  if (!tr) return set_error(LBM_EINVAL, "NULL trainer");
  if (!tr->x || !tr->weights) return set_error(LBM_ESTATE, "set data and weights first");
  if (nsteps < 0) return set_error(LBM_EINVAL, "nsteps < 0");
  for (int64_t s = 0; s < nsteps; ++s) {
    lbm_status st = run_tiles(tr, nullptr, tr->p.batch, tr->steps);
    if (st) return st;
    const double t1 = double(tr->steps + 1);
    UpdateArgs u{};
    u.st = tr->st;
    u.part = tr->part;
    u.tiles = tr->p.batch / kTS;
    u.grad = nullptr;
    u.lr = float(tr->p.lr);
    u.beta1 = float(tr->p.beta1);
    u.beta2 = float(tr->p.beta2);
    u.eps = float(tr->p.eps);
    u.c1 = float(1.0 / (1.0 - std::pow(tr->p.beta1, t1)));
    u.c2 = float(1.0 / (1.0 - std::pow(tr->p.beta2, t1)));
    u.loss_scale = 1.0 / (3.0 * tr->p.batch);
    hipLaunchKernelGGL(k_train_update, dim3(kUpdBlocks), dim3(kBlock), 0, tr->stream, u);
    TRY_HIP(hipGetLastError());
    ++tr->steps;
  }
  return LBM_OK;
}

lbm_status lbm_train_loss(lbm_trainer* tr, double* loss) {
  if (!tr || !loss) return set_error(LBM_EINVAL, "NULL argument");
  TRY_HIP(hipMemcpyAsync(loss, &tr->st->loss, 8, hipMemcpyDeviceToHost, tr->stream));
  TRY_HIP(hipStreamSynchronize(tr->stream));
  return LBM_OK;
}

lbm_status lbm_train_get_weights(lbm_trainer* tr, const lbm_mlp_host* out) {
  if (!tr || !out) return set_error(LBM_EINVAL, "NULL argument");
  std::vector<float> w(kNP);
  std::vector<double> mean(kStatCols), sd(kStatCols);
  TRY_HIP(hipMemcpyAsync(w.data(), tr->st->w, kNP * 4, hipMemcpyDeviceToHost, tr->stream));
  TRY_HIP(hipMemcpyAsync(mean.data(), tr->st->mean, kStatCols * 8, hipMemcpyDeviceToHost, tr->stream));
  TRY_HIP(hipMemcpyAsync(sd.data(), tr->st->sd, kStatCols * 8, hipMemcpyDeviceToHost, tr->stream));
  TRY_HIP(hipStreamSynchronize(tr->stream));
  auto put = [](float* dst, const float* src, int n) {
    if (dst) memcpy(dst, src, size_t(n) * 4);
  };
  put(out->w1, w.data() + kOffW1, 64 * 27);
  put(out->b1, w.data() + kOffB1, 64);
  put(out->w2, w.data() + kOffW2, 64 * 64);
  put(out->b2, w.data() + kOffB2, 64);
  put(out->w3, w.data() + kOffW3, 3 * 64);
  put(out->b3, w.data() + kOffB3, 3);
  for (int c = 0; c < kStatCols; ++c) {
    if (c < 27) {
      if (out->mu_in) out->mu_in[c] = float(mean[c]);
      if (out->sd_in) out->sd_in[c] = float(sd[c]);
    } else {
      if (out->mu_out) out->mu_out[c - 27] = float(mean[c]);
      if (out->sd_out) out->sd_out[c - 27] = float(sd[c]);
    }
  }
  return LBM_OK;
}

lbm_status lbm_train_gradient(lbm_trainer* tr, const int32_t* rows, int32_t n_rows, float* grad,
                              double* loss) {
  if (!tr || !rows || !grad || !loss) return set_error(LBM_EINVAL, "NULL argument");
  if (!tr->x || !tr->weights) return set_error(LBM_ESTATE, "set data and weights first");
  if (n_rows < 64 || n_rows % 64 || n_rows > 65536)
    return set_error(LBM_EINVAL, "n_rows must be a multiple of 64 in [64, 65536]");
  lbm_status st = run_tiles(tr, rows, n_rows, 0);
  if (st) return st;
  UpdateArgs u{};
  u.st = tr->st;
  u.part = tr->part;
  u.tiles = n_rows / kTS;
  u.grad = tr->grad;
  u.loss_scale = 1.0 / (3.0 * n_rows);
  hipLaunchKernelGGL(k_train_update, dim3(kUpdBlocks), dim3(kBlock), 0, tr->stream, u);
  TRY_HIP(hipGetLastError());
  TRY_HIP(hipMemcpyAsync(grad, tr->grad, kNP * 4, hipMemcpyDeviceToHost, tr->stream));
  TRY_HIP(hipMemcpyAsync(loss, &tr->st->loss, 8, hipMemcpyDeviceToHost, tr->stream));
  TRY_HIP(hipStreamSynchronize(tr->stream));
  return LBM_OK;
}

lbm_status lbm_mlp_gradient_noalloc(const lbm_mlp* w, const float* dev_x, const float* dev_t,
                                    const int32_t* dev_rows, int32_t n_rows, float* grad,
                                    double* loss, void* stream) {
  if (!w || !w->w1 || !w->b1 || !w->w2 || !w->b2 || !w->w3 || !w->b3 || !w->mu_in || !w->sd_in ||
      !w->mu_out || !w->sd_out || !dev_x || !dev_t || !dev_rows || !grad || !loss)
    return set_error(LBM_EINVAL, "NULL argument");
  if (w->n_in != 27 || w->n_h1 != 64 || w->n_h2 != 64 || w->n_out != 3)
    return set_error(LBM_EINVAL, "network must be 27-64-64-3");
  if (n_rows < kTS || n_rows % kTS)
    return set_error(LBM_EINVAL, "n_rows must be a positive multiple of 64 (got %d)", n_rows);
  if (n_rows > kNoallocMaxRows)
    return set_error(LBM_EINVAL, "n_rows %d exceeds the %d rows the static scratch buffer holds",
                     n_rows, kNoallocMaxRows);
  for (int c = 0; c < 27; ++c)
    if (!(w->sd_in[c] > 0) || !std::isfinite(w->sd_in[c]))
      return set_error(LBM_EINVAL, "sd_in[%d] must be finite and > 0", c);
  for (int c = 0; c < 3; ++c)
    if (!(w->sd_out[c] > 0) || !std::isfinite(w->sd_out[c]))
      return set_error(LBM_EINVAL, "sd_out[%d] must be finite and > 0", c);
  void* ptr = nullptr;
  lbm_status st = scratch_address(&ptr);
  if (st) return st;
  hipStream_t strm = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ptr);
  TrainState* dst = reinterpret_cast<TrainState*>(base);
  float* part = reinterpret_cast<float*>(base + kNoallocState);
  float* gdev = reinterpret_cast<float*>(base + kNoallocState + (kNoallocPart + 255) / 256 * 256);
  // the image lbm_train_set_weights and lbm_train_set_data leave: masters,
  // zero moments, BF16 copies, FP32 means and reciprocal deviations
  TrainState& h = g_noalloc_image;
  memset(&h, 0, sizeof h);
  memcpy(h.w + kOffW1, w->w1, 64 * 27 * 4);
  memcpy(h.w + kOffB1, w->b1, 64 * 4);
  memcpy(h.w + kOffW2, w->w2, 64 * 64 * 4);
  memcpy(h.w + kOffB2, w->b2, 64 * 4);
  memcpy(h.w + kOffW3, w->w3, 3 * 64 * 4);
  memcpy(h.w + kOffB3, w->b3, 3 * 4);
  for (int j = 0; j < 64; ++j)
    for (int f = 0; f < 27; ++f) h.w1b[j * 32 + f] = host_bf16(w->w1[j * 27 + f]);
  for (int j = 0; j < 64; ++j)
    for (int i = 0; i < 64; ++i) {
      h.w2b[j * 64 + i] = host_bf16(w->w2[j * 64 + i]);
      h.w2t[i * 64 + j] = host_bf16(w->w2[j * 64 + i]);
    }
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 64; ++i) h.w3b[k * 64 + i] = host_bf16(w->w3[k * 64 + i]);
  for (int c = 0; c < 27; ++c) {
    h.mu[c] = w->mu_in[c];
    h.inv_sd[c] = 1.0f / w->sd_in[c];
  }
  for (int c = 0; c < 3; ++c) {
    h.mu_out[c] = w->mu_out[c];
    h.inv_sd_out[c] = 1.0f / w->sd_out[c];
  }
  TRY_HIP(hipMemcpyAsync(dst, &h, offsetof(TrainState, loss), hipMemcpyHostToDevice, strm));
  TrainArgs a{};
  a.st = dst;
  a.x = dev_x;
  a.t = dev_t;
  a.n = 0;                       // rows are given: the sampler is not used
  a.rows = dev_rows;
  a.batch = n_rows;
  a.part = part;
  a.gscale = float(2.0 / (3.0 * n_rows));
  hipLaunchKernelGGL(k_train_tile, dim3(n_rows / kTS), dim3(kBlock), 0, strm, a);
  TRY_HIP(hipGetLastError());
  UpdateArgs u{};
  u.st = dst;
  u.part = part;
  u.tiles = n_rows / kTS;
  u.grad = gdev;
  u.loss_scale = 1.0 / (3.0 * n_rows);
  hipLaunchKernelGGL(k_train_update, dim3(kUpdBlocks), dim3(kBlock), 0, strm, u);
  TRY_HIP(hipGetLastError());
  TRY_HIP(hipMemcpyAsync(grad, gdev, kNP * 4, hipMemcpyDeviceToHost, strm));
  TRY_HIP(hipMemcpyAsync(loss, &dst->loss, 8, hipMemcpyDeviceToHost, strm));
  TRY_HIP(hipStreamSynchronize(strm));
  return LBM_OK;
}

lbm_status lbm_train_sample_rows(lbm_trainer* tr, int64_t step, int32_t* rows) {
  if (!tr || !rows) return set_error(LBM_EINVAL, "NULL argument");
  if (!tr->x) return set_error(LBM_ESTATE, "set data first");
  hipLaunchKernelGGL(k_sample_rows, dim3((tr->p.batch + kBlock - 1) / kBlock), dim3(kBlock), 0,
                     tr->stream, tr->rows, tr->p.seed, step, tr->p.batch, tr->n);
  TRY_HIP(hipGetLastError());
  TRY_HIP(hipMemcpyAsync(rows, tr->rows, size_t(tr->p.batch) * 4, hipMemcpyDeviceToHost, tr->stream));
  TRY_HIP(hipStreamSynchronize(tr->stream));
  return LBM_OK;
}

}  // extern "C"
