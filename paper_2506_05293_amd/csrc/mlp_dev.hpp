// Outflow MLP 27 -> 64 -> 64 -> 3 on 64-row tiles with gfx950 MFMA.
//
// Sec. 3.1: the unknown populations of the outlet node are reconstructed as
// f_i^B(L) = f_i(L-1) + s_i^NN (Eq. 16) from a small fully connected network
// of interior populations.  Here a workgroup of four wave64 evaluates the
// network for 64 rows at once: the standardised inputs X [64][32] (BF16, 27
// features padded to 32) sit in LDS, each wave owns 16 rows, and every layer
// is a chain of v_mfma_f32_16x16x32_bf16 (BF16 operands, FP32 accumulate).
// Hidden activations are tanh in FP32, rounded to BF16 for the next layer.
//
// MFMA 16x16x32 operand layout used here (lane l, group g = l / 16):
//   A (16 x 32): lane holds row l % 16, the 8 k-values of group g;
//   B (32 x 16): lane holds column l % 16, the same 8 k-values;
//   D (16 x 16 FP32): lane holds rows 4 g + 0..3 of column l % 16.
// Only the row/column placement matters; A and B share the k placement.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_internal.hpp"

namespace lbm {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return 0x7FC0;  // NaN
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

__device__ __forceinline__ bf16x8_t load8(const uint16_t* p) {
  const uint4 v = *reinterpret_cast<const uint4*>(p);
  return __builtin_bit_cast(bf16x8_t, v);
}

// LDS used by the network.  x holds the standardised inputs; h holds the
// hidden activations of both layers (each wave reads its 16 rows of layer 1
// into registers before overwriting them with layer 2); o the outputs.
constexpr int kXPitch = 32;
constexpr int kHPitch = 72;   // 64 + 8 BF16 to spread LDS banks
struct alignas(16) MlpX {
  uint16_t x[kNnRows * kXPitch];
};
struct alignas(16) MlpH {
  uint16_t h[kNnRows * kHPitch];
  float o[kNnRows * 4];
};

__device__ __forceinline__ void mlp_hidden_layer(const uint16_t* __restrict__ wmat, int kin,
                                                 const float* __restrict__ bias,
                                                 const bf16x8_t* a, uint16_t* h, int r16,
                                                 int grp, int orow) {
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int n = nt * 16 + r16;
    f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < kin / 32; ++ks) {
      const bf16x8_t b = load8(&wmat[n * kin + ks * 32 + grp * 8]);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ks], b, acc, 0, 0, 0);
    }
    const float bb = bias[n];
#pragma unroll
    for (int i = 0; i < 4; ++i) h[(orow + i) * kHPitch + n] = f32_to_bf16(tanhf(acc[i] + bb));
  }
}

// Evaluate the tile: reads X.x, writes H.o[row][0..2] (standardised outputs
// before the affine map).  Every thread of the 256-thread block calls it,
// after a barrier that publishes X.x; H may alias memory that is dead by
// then.  Ends with a barrier.
__device__ __forceinline__ void mlp_tile(const MlpDev* __restrict__ w, const MlpX& X, MlpH& H) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int r16 = lane & 15;
  const int grp = lane >> 4;
  const int row = wave * 16 + r16;        // A-operand row of this lane
  const int orow = wave * 16 + grp * 4;   // first D row of this lane
  bf16x8_t a[2];

  a[0] = load8(&X.x[row * kXPitch + grp * 8]);
  mlp_hidden_layer(w->w1, 32, w->b1, a, H.h, r16, grp, orow);        // layer 1
  __syncthreads();
  a[0] = load8(&H.h[row * kHPitch + grp * 8]);
  a[1] = load8(&H.h[row * kHPitch + 32 + grp * 8]);
  __syncthreads();                                                    // rows read
  mlp_hidden_layer(w->w2, 64, w->b2, a, H.h, r16, grp, orow);        // layer 2
  __syncthreads();
  a[0] = load8(&H.h[row * kHPitch + grp * 8]);
  a[1] = load8(&H.h[row * kHPitch + 32 + grp * 8]);
  {                                                                   // layer 3
    f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], load8(&w->w3[r16 * 64 + grp * 8]),
                                                  acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], load8(&w->w3[r16 * 64 + 32 + grp * 8]),
                                                  acc, 0, 0, 0);
    if (r16 < 3) {
      const float bb = w->b3[r16];
#pragma unroll
      for (int i = 0; i < 4; ++i) H.o[(orow + i) * 4 + r16] = acc[i] + bb;
    }
  }
  __syncthreads();
}

// Standardise one feature in FP32 and round to BF16.
__device__ __forceinline__ uint16_t feature_bf16(const MlpDev* __restrict__ w, int k, float v) {
  return f32_to_bf16((v - w->mu_in[k]) * w->inv_sd_in[k]);
}

}  // namespace lbm
