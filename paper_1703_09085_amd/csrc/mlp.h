// Rank-predictor network: layout of the parameters and the device-side
// inference used by the truncation kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace hm {

constexpr int MLP_IN = 8;   // features
constexpr int MLP_H = 64;   // hidden width (two layers)
constexpr int MLP_OFF_W1 = 0;
constexpr int MLP_OFF_B1 = MLP_OFF_W1 + MLP_H * MLP_IN;
constexpr int MLP_OFF_W2 = MLP_OFF_B1 + MLP_H;
constexpr int MLP_OFF_B2 = MLP_OFF_W2 + MLP_H * MLP_H;
constexpr int MLP_OFF_W3 = MLP_OFF_B2 + MLP_H;
constexpr int MLP_OFF_B3 = MLP_OFF_W3 + MLP_H;
constexpr int MLP_NPARAM = MLP_OFF_B3 + 1;  // 4801

// Working copy of the weights on the device: BF16 matrices (row-major), FP32
// biases.
struct MlpWeights {
  uint16_t* W1;
  float* b1;
  uint16_t* W2;
  float* b2;
  uint16_t* w3;
  float* b3;
};

__device__ __forceinline__ float bf16_as_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// One forward pass (one thread): predicted log2(1 + k) for features x.
__device__ __forceinline__ float mlp_infer(const MlpWeights& p, const float* x) {
  float h1[MLP_H];
#pragma unroll
  for (int j = 0; j < MLP_H; ++j) {
    float a = p.b1[j];
#pragma unroll
    for (int i = 0; i < MLP_IN; ++i) a = fmaf(bf16_as_f32(p.W1[j * MLP_IN + i]), x[i], a);
    h1[j] = a > 0.f ? a : 0.f;
  }
  float y = p.b3[0];
  for (int j = 0; j < MLP_H; ++j) {
    float a = p.b2[j];
#pragma unroll
    for (int i = 0; i < MLP_H; ++i) a = fmaf(bf16_as_f32(p.W2[j * MLP_H + i]), h1[i], a);
    y = fmaf(bf16_as_f32(p.w3[j]), a > 0.f ? a : 0.f, y);
  }
  return y;
}

hipError_t mlp_publish(const float* w, const MlpWeights& p, hipStream_t s);
hipError_t mlp_forward(const MlpWeights& p, const float* X, int64_t B, float* y, hipStream_t s);
int mlp_backward_blocks(int64_t B);
hipError_t mlp_gradient(const MlpWeights& p, const float* X, const float* T, int64_t B, float scale, float* partial,
                        float* grad, float* loss, hipStream_t s);
hipError_t mlp_adam(float* w, float* m, float* v, const float* g, float lr, int step, const MlpWeights& p,
                    hipStream_t s);

}  // namespace hm
