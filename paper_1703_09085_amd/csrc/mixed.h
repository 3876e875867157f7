// Reduced-precision contraction helpers for gfx950.
//
// FP32 mode: operands rounded to FP32, products accumulated in FP32.
// Split-BF16x3 mode: every FP32 operand x is split into three BF16 pieces
// x = h + m + l (each the BF16 rounding of what the previous ones leave), and
// a product a b is taken as the six cross terms of total order below 2^-16,
//   h_a h_b + h_a m_b + m_a h_b + h_a l_b + m_a m_b + l_a h_b,
// on the matrix cores (v_mfma_f32_32x32x16_bf16) with FP32 accumulation; the
// dropped terms are below 2^-24 |a| |b|, the FP32 rounding level.
//
// Operand layout of the 32 x 32 x 16 BF16 instruction (lane l of a wave):
// A(row l % 32, k = 8 (l / 32) + j) and B(k = 8 (l / 32) + j, col l % 32) for
// j = 0..7; result register q holds D(8 (q / 4) + 4 (l / 32) + q % 4, l % 32).
#pragma once
#include <hip/hip_runtime.h>

namespace hm {

enum Precision : int { PREC_FP64 = 0, PREC_FP32 = 1, PREC_BF16X3 = 2 };

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ void split3(const float (&x)[8], bf16x8& h, bf16x8& m, bf16x8& l) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const __bf16 hj = (__bf16)x[j];
    const float r1 = x[j] - (float)hj;  // exact
    const __bf16 mj = (__bf16)r1;
    const float r2 = r1 - (float)mj;    // exact
    h[j] = hj;
    m[j] = mj;
    l[j] = (__bf16)r2;
  }
}

// acc += A B for the 32 x 16 and 16 x 32 FP32 operand fragments a, b of this
// lane (layout above), in split-BF16x3; the small terms go first.
__device__ __forceinline__ f32x16 mfma_bf16x3(const float (&a)[8], const float (&b)[8], f32x16 acc) {
  bf16x8 ah, am, al, bh, bm, bl;
  split3(a, ah, am, al);
  split3(b, bh, bm, bl);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bm, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bh, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bm, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
  return acc;
}

__device__ __forceinline__ f32x16 zero_f32x16() {
  f32x16 z;
#pragma unroll
  for (int i = 0; i < 16; ++i) z[i] = 0.f;
  return z;
}

}  // namespace hm
