// Rank-predictor network for gfx950: forward, backward and Adam update.
//
// 8 features of a truncation -> predicted log2(1 + k):
//   h1 = relu(W1 x + b1) (64), h2 = relu(W2 h1 + b2) (64), y = w3 . h2 + b3.
// The weights used by the forward and backward passes are BF16 (rounded to
// nearest even from FP32 master weights); every product is accumulated in
// FP32.  Loss: 0.5 mean (y - t)^2.
//
// Parameter vector (FP32 master weights, gradients, Adam moments), 4801
// entries: W1 (64 x 8, row-major) | b1 (64) | W2 (64 x 64, row-major) | b2 (64)
// | w3 (64) | b3 (1).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mlp.h"

namespace hm {

namespace {

constexpr int NB = 128;  // samples per backward workgroup (one thread each)
constexpr int LR = MLP_H + 1;  // LDS row stride of the per-sample vectors

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // NaN stays NaN
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

__device__ void mlp_store(const MlpWeights& p, int i, float wi) {
  if (i < MLP_OFF_B1)
    p.W1[i - MLP_OFF_W1] = f32_to_bf16(wi);
  else if (i < MLP_OFF_W2)
    p.b1[i - MLP_OFF_B1] = wi;
  else if (i < MLP_OFF_B2)
    p.W2[i - MLP_OFF_W2] = f32_to_bf16(wi);
  else if (i < MLP_OFF_W3)
    p.b2[i - MLP_OFF_B2] = wi;
  else if (i < MLP_OFF_B3)
    p.w3[i - MLP_OFF_W3] = f32_to_bf16(wi);
  else
    p.b3[0] = wi;
}

__global__ __launch_bounds__(256) void mlp_forward_kernel(MlpWeights p, const float* __restrict__ X, int64_t B,
                                                          float* __restrict__ y) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= B) return;
  float x[MLP_IN];
#pragma unroll
  for (int i = 0; i < MLP_IN; ++i) x[i] = X[s * MLP_IN + i];
  y[s] = mlp_infer(p, x);
}

// Backward pass of NB samples per workgroup.  Each thread runs the forward
// pass of its sample into LDS rows (pre-activations z1, z2; h1), turns them
// into the backpropagated factors dz2 = dy w3 [z2 > 0] and dz1 = (W2^T dz2)
// [z1 > 0], and then the workgroup forms its weight gradients as sums over its
// samples in a fixed order, written to partial[blockIdx.x].  scale = 1 / (the
// number of samples of the loss).
__global__ __launch_bounds__(NB) void mlp_backward_kernel(MlpWeights p, const float* __restrict__ X,
                                                          const float* __restrict__ T, int64_t B, float scale,
                                                          float* __restrict__ partial, float* __restrict__ loss) {
  __shared__ float sx[NB][MLP_IN];
  __shared__ float sz1[NB * LR];  // z1, then dz1
  __shared__ float sh1[NB * LR];  // h1
  __shared__ float sz2[NB * LR];  // z2, then dz2, then h2
  __shared__ float sdy[NB], sl[NB];
  const int t = threadIdx.x;
  const int64_t s = blockIdx.x * (int64_t)NB + t;
  float* z1 = sz1 + t * LR;
  float* h1 = sh1 + t * LR;
  float* z2 = sz2 + t * LR;
  const bool act = s < B;
  float x[MLP_IN];
#pragma unroll
  for (int i = 0; i < MLP_IN; ++i) {
    x[i] = act ? X[s * MLP_IN + i] : 0.f;
    sx[t][i] = x[i];
  }
  for (int j = 0; j < MLP_H; ++j) {
    float a = p.b1[j];
#pragma unroll
    for (int i = 0; i < MLP_IN; ++i) a = fmaf(bf16_as_f32(p.W1[j * MLP_IN + i]), x[i], a);
    z1[j] = a;
    h1[j] = a > 0.f ? a : 0.f;
  }
  float y = p.b3[0];
  for (int j = 0; j < MLP_H; ++j) {
    float a = p.b2[j];
    for (int i = 0; i < MLP_H; ++i) a = fmaf(bf16_as_f32(p.W2[j * MLP_H + i]), h1[i], a);
    z2[j] = a;
    y = fmaf(bf16_as_f32(p.w3[j]), a > 0.f ? a : 0.f, y);
  }
  const float r = act ? y - T[s] : 0.f;
  const float dy = r * scale;
  sdy[t] = dy;
  sl[t] = 0.5f * r * r;
  for (int j = 0; j < MLP_H; ++j) z2[j] = z2[j] > 0.f ? dy * bf16_as_f32(p.w3[j]) : 0.f;  // dz2
  for (int i = 0; i < MLP_H; ++i) {
    float a = 0.f;
    for (int j = 0; j < MLP_H; ++j) a = fmaf(bf16_as_f32(p.W2[j * MLP_H + i]), z2[j], a);
    z1[i] = z1[i] > 0.f ? a : 0.f;  // dz1
  }
  __syncthreads();
  float* out = partial + (size_t)blockIdx.x * MLP_NPARAM;
  for (int e = t; e < MLP_H * MLP_IN; e += NB) {  // W1
    const int j = e / MLP_IN, i = e % MLP_IN;
    float a = 0.f;
    for (int q = 0; q < NB; ++q) a = fmaf(sz1[q * LR + j], sx[q][i], a);
    out[MLP_OFF_W1 + e] = a;
  }
  for (int e = t; e < MLP_H * MLP_H; e += NB) {  // W2
    const int j = e / MLP_H, i = e % MLP_H;
    float a = 0.f;
    for (int q = 0; q < NB; ++q) a = fmaf(sz2[q * LR + j], sh1[q * LR + i], a);
    out[MLP_OFF_W2 + e] = a;
  }
  for (int j = t; j < MLP_H; j += NB) {  // b1, b2
    float a = 0.f, b = 0.f;
    for (int q = 0; q < NB; ++q) {
      a += sz1[q * LR + j];
      b += sz2[q * LR + j];
    }
    out[MLP_OFF_B1 + j] = a;
    out[MLP_OFF_B2 + j] = b;
  }
  __syncthreads();
  // w3 needs h2 = relu(W2 h1 + b2): recomputed into the z2 row (dz2 is used up)
  for (int j = 0; j < MLP_H; ++j) {
    float a = p.b2[j];
    for (int i = 0; i < MLP_H; ++i) a = fmaf(bf16_as_f32(p.W2[j * MLP_H + i]), h1[i], a);
    z2[j] = a > 0.f ? a : 0.f;
  }
  __syncthreads();
  for (int j = t; j < MLP_H; j += NB) {
    float a = 0.f;
    for (int q = 0; q < NB; ++q) a = fmaf(sdy[q], sz2[q * LR + j], a);
    out[MLP_OFF_W3 + j] = a;
  }
  if (t == 0) {
    float a = 0.f, l = 0.f;
    for (int q = 0; q < NB; ++q) {
      a += sdy[q];
      l += sl[q];
    }
    out[MLP_OFF_B3] = a;
    if (loss) loss[blockIdx.x] = l;
  }
}

// grad[i] = sum over the nblk partial gradient vectors (fixed order)
__global__ void mlp_reduce_kernel(const float* __restrict__ partial, int nblk, float* __restrict__ grad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= MLP_NPARAM) return;
  float a = 0.f;
  for (int b = 0; b < nblk; ++b) a += partial[(size_t)b * MLP_NPARAM + i];
  grad[i] = a;
}

// Adam step on the FP32 master weights, then the working copy
__global__ void mlp_adam_kernel(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                                const float* __restrict__ g, float lr, float b1, float b2, float c1, float c2,
                                MlpWeights p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= MLP_NPARAM) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
  w[i] = wi;
  mlp_store(p, i, wi);
}

__global__ void mlp_publish_kernel(const float* __restrict__ w, MlpWeights p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < MLP_NPARAM) mlp_store(p, i, w[i]);
}

}  // namespace

hipError_t mlp_publish(const float* w, const MlpWeights& p, hipStream_t s) {
  hipLaunchKernelGGL(mlp_publish_kernel, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, w, p);
  return hipGetLastError();
}

hipError_t mlp_forward(const MlpWeights& p, const float* X, int64_t B, float* y, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, p, X, B, y);
  return hipGetLastError();
}

int mlp_backward_blocks(int64_t B) { return (int)((B + NB - 1) / NB); }

hipError_t mlp_gradient(const MlpWeights& p, const float* X, const float* T, int64_t B, float scale, float* partial,
                        float* grad, float* loss, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  const int nblk = mlp_backward_blocks(B);
  hipLaunchKernelGGL(mlp_backward_kernel, dim3(nblk), dim3(NB), 0, s, p, X, T, B, scale, partial, loss);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, partial, nblk, grad);
  return hipGetLastError();
}

hipError_t mlp_adam(float* w, float* m, float* v, const float* g, float lr, int step, const MlpWeights& p,
                    hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f;
  float c1 = 1.f, c2 = 1.f;
  for (int i = 0; i < step; ++i) {
    c1 *= b1;
    c2 *= b2;
  }
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, w, m, v, g, lr, b1, b2,
                     1.f - c1, 1.f - c2, p);
  return hipGetLastError();
}

}  // namespace hm
