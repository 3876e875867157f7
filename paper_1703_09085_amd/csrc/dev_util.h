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

// The stacked column counts of an item's parts (up to 4), read by lanes
// 0 .. nparts - 1 of the calling wave at once: one memory latency for all the
// parts' rank words instead of one after another.  Part p's count goes to
// k[p] (when k is given) and its first stacked column to coff[p], the part
// itself to part_out[p] (when given; all three in LDS, written by lane p);
// every lane gets the total l and the first and last parts' counts.  The
// whole wave calls it.
struct StackCounts {
  int l, k0, klast;
};
__device__ __forceinline__ StackCounts stacked_counts(const DTruncPart* __restrict__ parts, int part0, int nparts,
                                                     int* k, int* coff, DTruncPart* part_out) {
  const int lane = threadIdx.x & 63;
  int kp = 0;
  if (lane < nparts) {
    const DTruncPart P = parts[part0 + lane];
    if (part_out) part_out[lane] = P;
    kp = rdim(P.k);
  }
  StackCounts s{0, 0, 0};
  int off = 0;
  for (int p = 0; p < nparts; ++p) {
    const int kq = __builtin_amdgcn_readlane(kp, p);
    if (lane == p) off = s.l;
    if (p == 0) s.k0 = kq;
    s.klast = kq;
    s.l += kq;
  }
  if (lane < nparts) {
    if (k) k[lane] = kp;
    coff[lane] = off;
  }
  return s;
}

// A zero that a predicated-off load reads instead of its element, so that
// the loads of a staging pass issue without branches and stay in flight
// together (a load inside a branch is waited for at the branch's end).
static __device__ const double kZeroElem = 0.0;

// scale * *p when ok, else 0, with the load always issued (of a zero when not
// ok): a global (not generic) load counts only against the vector-memory
// counter, so LDS reads that follow do not wait for it, and a product rather
// than a select keeps the compiler from sinking the load into a branch.
__device__ __forceinline__ double load_or_zero(const double* p, bool ok, double scale) {
  const double* src = ok ? p : &kZeroElem;
  const double x = *(const __attribute__((address_space(1))) double*)src;
  return x * (ok ? scale : 1.0);
}

// Element (i, col) of the stacked factors of a truncation: A_s (side 0, row i
// of the block's lim = m rows, the part's alpha applied) or B_s (side 1, row i
// of its lim = n rows).  The column's part comes from the column offsets coff
// (nparts parts); the element is zero outside the part's rows, lim and the
// stacked width l.  Branch-free: the load always issues.
__device__ __forceinline__ double stacked_elem(const DTruncPart* part, const int* coff, int nparts, int side, int i,
                                               int lim, int col, int l) {
  int p = 0;
  p += (nparts > 1 && col >= coff[1]) ? 1 : 0;
  p += (nparts > 2 && col >= coff[2]) ? 1 : 0;
  p += (nparts > 3 && col >= coff[3]) ? 1 : 0;
  const DTruncPart& P = part[p];
  const int cc = col - coff[p];
  const int r = i - (side ? P.col_off : P.row_off);
  const bool ok = col < l && i < lim && r >= 0 && r < (side ? P.cols : P.rows);
  const double* base = side ? P.B : P.A;
  const int ld = side ? P.ldb : P.lda;
  const bool tr = side ? P.tb != 0 : P.ta != 0;
  const size_t off = tr ? (size_t)cc + (size_t)r * (size_t)ld : (size_t)r + (size_t)cc * (size_t)ld;
  return load_or_zero(base + off, ok, side ? 1.0 : P.alpha);
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
