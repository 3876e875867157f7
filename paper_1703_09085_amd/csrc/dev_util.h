// Device helpers shared by the truncation kernels: dynamic dimensions and
// cross-lane reductions of doubles through DPP (64-wide wavefronts).
#pragma once
#include <hip/hip_runtime.h>

#include "hm_types.h"

namespace hm {

__device__ __forceinline__ int rdim(const DDim& d) {
  int v = d.stat;
  if (d.dyn) {
    int r = *d.dyn;
    v = r < v ? r : v;
  }
  return v < 0 ? 0 : v;
}

// Cross-lane moves of a double through DPP (two 32-bit halves).  CTRL is the
// DPP control word; lanes of rows excluded by ROWMASK return `old`.
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ double dpp(double v, double old = 0.0) {
  const long long b = __double_as_longlong(v), o = __double_as_longlong(old);
  const int lo = __builtin_amdgcn_update_dpp((int)o, (int)b, CTRL, ROWMASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(b >> 32), CTRL, ROWMASK, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

constexpr int DPP_XOR1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int DPP_XOR2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int DPP_HALF_MIRROR = 0x141;
constexpr int DPP_MIRROR = 0x140;
constexpr int DPP_BCAST15 = 0x142;
constexpr int DPP_BCAST31 = 0x143;

// Sum over each row of 16 lanes, returned in every lane of the row.
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp<DPP_XOR1>(v);
  v += dpp<DPP_XOR2>(v);
  v += dpp<DPP_HALF_MIRROR>(v);
  v += dpp<DPP_MIRROR>(v);
  return v;
}

__device__ __forceinline__ double row16_max(double v) {
  v = fmax(v, dpp<DPP_XOR1>(v));
  v = fmax(v, dpp<DPP_XOR2>(v));
  v = fmax(v, dpp<DPP_HALF_MIRROR>(v));
  v = fmax(v, dpp<DPP_MIRROR>(v));
  return v;
}

__device__ __forceinline__ double lane_read(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes of a wave (all lanes active), returned in every lane.
__device__ __forceinline__ double wave_sum(double v) {
  v = row16_sum(v);
  v += dpp<DPP_BCAST15, 0xa>(v);  // rows 1, 3 += last lane of rows 0, 2
  v += dpp<DPP_BCAST31, 0xc>(v);  // rows 2, 3 += lane 31
  return lane_read(v, 63);
}

__device__ __forceinline__ double wave_max(double v) {
  v = row16_max(v);
  v = fmax(v, dpp<DPP_BCAST15, 0xa>(v, v));
  v = fmax(v, dpp<DPP_BCAST31, 0xc>(v, v));
  return lane_read(v, 63);
}

// Reductions inside aligned groups of g lanes (g a power of two <= 64); the
// lanes of a group are active together.
__device__ __forceinline__ double group_sum(double v, int g) {
  if (g >= 16) {
    v = row16_sum(v);
    if (g >= 32) v += __shfl_xor(v, 16, 64);
    if (g >= 64) v += __shfl_xor(v, 32, 64);
    return v;
  }
  if (g >= 2) v += dpp<DPP_XOR1>(v);
  if (g >= 4) v += dpp<DPP_XOR2>(v);
  if (g >= 8) v += dpp<DPP_HALF_MIRROR>(v);
  return v;
}

__device__ __forceinline__ double group_max(double v, int g) {
  if (g >= 16) {
    v = row16_max(v);
    if (g >= 32) v = fmax(v, __shfl_xor(v, 16, 64));
    if (g >= 64) v = fmax(v, __shfl_xor(v, 32, 64));
    return v;
  }
  if (g >= 2) v = fmax(v, dpp<DPP_XOR1>(v));
  if (g >= 4) v = fmax(v, dpp<DPP_XOR2>(v));
  if (g >= 8) v = fmax(v, dpp<DPP_HALF_MIRROR>(v));
  return v;
}

// A sum of squares is trusted when it is far from underflow and overflow;
// otherwise it is recomputed on values scaled by an exact power of two.
__device__ __forceinline__ bool safe_sq(double s) { return s > 1e-280 && s < 1e280; }

// Sum and max over each aligned group of 4 lanes (quad), returned in every lane
// of the quad; the four lanes combine their values in the same order, so the
// result is bit-identical across the quad.
__device__ __forceinline__ double quad_sum(double v) {
  v += dpp<DPP_XOR1>(v);
  v += dpp<DPP_XOR2>(v);
  return v;
}

__device__ __forceinline__ double quad_max(double v) {
  v = fmax(v, dpp<DPP_XOR1>(v));
  v = fmax(v, dpp<DPP_XOR2>(v));
  return v;
}

}  // namespace hm
