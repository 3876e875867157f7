// Batched variable-size dense kernels for gfx950: GEMM term lists (FP64, FP32 or
// split-BF16x3 on the matrix cores, always added to FP64 storage), FP64 leaf
// LU, triangular solves with leaf factors, and block copies.
//
// The H-matrix by thin-dense products of Fig. addeval are lowered to GEMM work
// items: one item per output row block sums, in a fixed order, every leaf
// contribution to that row block, so the result is deterministic and no
// atomics are needed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "dev_util.h"
#include "hm_types.h"
#include "mixed.h"

namespace hm {

namespace {

constexpr int GT = 64;   // output tile edge
constexpr int GK = 16;   // k chunk
constexpr int GTB = 256; // threads

__device__ __forceinline__ int rd(const DDim& d) {
  int v = d.stat;
  if (d.dyn) {
    int r = *d.dyn;
    v = r < v ? r : v;
  }
  return v < 0 ? 0 : v;
}

// C tile = beta C + sum_t alpha_t op(A_t) op(B_t).
// PREC_FP64: thread (tx, ty) owns rows tx + 16 a, columns ty + 16 b (a, b < 4).
// PREC_FP32: the same in FP32 (operands rounded to FP32, FP32 sums).
// PREC_BF16X3: wave w owns the 32 x 32 quadrant (32 (w % 2), 32 (w / 2)) and
// accumulates it on the matrix cores in split-BF16x3.
// The sum is added to C in FP64 in every mode.
template <int PREC>
__global__ __launch_bounds__(GTB) void gemm_kernel(const DGemm* __restrict__ items,
                                                    const DGemmTerm* __restrict__ terms) {
  using T = typename std::conditional<PREC == PREC_FP64, double, float>::type;
  __shared__ T As[GK][GT + 1];
  __shared__ T Bs[GK][GT + 1];
  const DGemm it = items[blockIdx.x];
  const int m = rd(it.m), n = rd(it.n);
  const int r0 = it.row0, c0 = it.col0;
  const int mt = min(GT, m - r0), nt = min(GT, n - c0);
  if (mt <= 0 || nt <= 0) return;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int lane = tid & 63, wave = tid >> 6;
  T acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0;
  f32x16 macc = zero_f32x16();
  for (int t = 0; t < it.nterms; ++t) {
    const DGemmTerm Tm = terms[it.term0 + t];
    const int k = rd(Tm.k);
    for (int k0 = 0; k0 < k; k0 += GK) {
      const int kc = min(GK, k - k0);
      // load op(A)[r0 + i, k0 + p] and op(B)[k0 + p, c0 + j]
      for (int e = tid; e < GK * GT; e += GTB) {
        int i, p;
        if (Tm.ta) {  // A^T: element (i, p) = A[p + i*lda]; p fastest for coalescing
          p = e % GK;
          i = e / GK;
        } else {
          i = e % GT;
          p = e / GT;
        }
        double v = 0.0;
        if (i < mt && p < kc) {
          const size_t gi = r0 + i, gp = k0 + p;
          v = Tm.ta ? Tm.A[gp + gi * Tm.lda] : Tm.A[gi + gp * Tm.lda];
        }
        As[p][i] = (T)(v * Tm.alpha);
      }
      for (int e = tid; e < GK * GT; e += GTB) {
        int j, p;
        if (Tm.tb) {  // B^T: element (p, j) = B[j + p*ldb]; j fastest
          j = e % GT;
          p = e / GT;
        } else {
          p = e % GK;
          j = e / GK;
        }
        double v = 0.0;
        if (j < nt && p < kc) {
          const size_t gj = c0 + j, gp = k0 + p;
          v = Tm.tb ? Tm.B[gj + gp * Tm.ldb] : Tm.B[gp + gj * Tm.ldb];
        }
        Bs[p][j] = (T)v;
      }
      __syncthreads();
      if constexpr (PREC == PREC_BF16X3) {
        const int rq = 32 * (wave & 1), cq = 32 * (wave >> 1), kg = 8 * (lane >> 5);
        float a[8], b[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          a[j] = As[kg + j][rq + (lane & 31)];
          b[j] = Bs[kg + j][cq + (lane & 31)];
        }
        macc = mfma_bf16x3(a, b, macc);
      } else {
#pragma unroll 4
        for (int p = 0; p < GK; ++p) {
          T a[4], b[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            a[q] = As[p][tx + 16 * q];
            b[q] = Bs[p][ty + 16 * q];
          }
#pragma unroll
          for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) acc[x][y] += a[x] * b[y];
        }
      }
      __syncthreads();
    }
  }
  if constexpr (PREC == PREC_BF16X3) {
    const int rq = 32 * (wave & 1), cq = 32 * (wave >> 1);
    const int j = cq + (lane & 31);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int i = rq + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
      if (i >= mt || j >= nt) continue;
      double* c = it.ctrans ? it.C + (size_t)(c0 + j) + (size_t)(r0 + i) * it.ldc
                            : it.C + (size_t)(r0 + i) + (size_t)(c0 + j) * it.ldc;
      *c = it.beta ? *c + (double)macc[q] : (double)macc[q];
    }
    return;
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int i = tx + 16 * a;
    if (i >= mt) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int j = ty + 16 * b;
      if (j >= nt) continue;
      double* c = it.ctrans ? it.C + (size_t)(c0 + j) + (size_t)(r0 + i) * it.ldc
                            : it.C + (size_t)(r0 + i) + (size_t)(c0 + j) * it.ldc;
      *c = it.beta ? *c + (double)acc[a][b] : (double)acc[a][b];
    }
  }
}

// In-place unpivoted LU of a dense leaf (n <= 128) staged in LDS.
__global__ __launch_bounds__(GTB) void lu_kernel(const DLu* __restrict__ items, int* status) {
  extern __shared__ double S[];
  const DLu it = items[blockIdx.x];
  const int n = it.n, tid = threadIdx.x;
  for (int e = tid; e < n * n; e += GTB) S[e] = it.N[(e % n) + (size_t)(e / n) * it.ld];
  __syncthreads();
  if (it.kind == LEAF_LU) {
    for (int k = 0; k < n; ++k) {
      const double piv = S[k + k * n];
      if (piv == 0.0) {
        if (tid == 0) atomicOr(status, ST_ZERO_PIVOT);
        break;
      }
      for (int i = k + 1 + tid; i < n; i += GTB) S[i + k * n] /= piv;
      __syncthreads();
      const int w = n - k - 1;
      for (int e = tid; e < w * w; e += GTB) {
        const int i = k + 1 + e % w, j = k + 1 + e / w;
        S[i + j * n] -= S[i + k * n] * S[k + j * n];
      }
      __syncthreads();
    }
  } else if (it.kind == LEAF_INVERSE) {
    // Gauss-Jordan without pivoting: step k scales row k by 1/piv, removes
    // column k from the other rows, and turns column k into that of the
    // inverse
    for (int k = 0; k < n; ++k) {
      const double piv = S[k + k * n];
      if (piv == 0.0) {
        if (tid == 0) atomicOr(status, ST_ZERO_PIVOT);
        break;
      }
      const double p = 1.0 / piv;
      for (int j = tid; j < n; j += GTB)
        if (j != k) S[k + j * n] *= p;
      __syncthreads();
      for (int e = tid; e < n * n; e += GTB) {
        const int i = e % n, j = e / n;
        if (i != k && j != k) S[i + j * n] -= S[i + k * n] * S[k + j * n];
      }
      __syncthreads();
      for (int i = tid; i < n; i += GTB) S[i + k * n] = (i == k) ? p : -S[i + k * n] * p;
      __syncthreads();
    }
  } else {
    // Cholesky L L^T, right-looking; a pivot that is not positive marks the
    // leaf as not positive definite
    for (int k = 0; k < n; ++k) {
      const double d = S[k + k * n];
      if (!(d > 0.0)) {
        if (tid == 0) atomicOr(status, ST_ZERO_PIVOT);
        break;
      }
      const double l = sqrt(d);
      __syncthreads();
      if (tid == 0) S[k + k * n] = l;
      for (int i = k + 1 + tid; i < n; i += GTB) S[i + k * n] /= l;
      __syncthreads();
      const int w = n - k - 1;
      for (int e = tid; e < w * w; e += GTB) {
        const int i = k + 1 + e % w, j = k + 1 + e / w;
        if (i >= j) S[i + j * n] -= S[i + k * n] * S[j + k * n];
      }
      __syncthreads();
    }
    for (int e = tid; e < n * n; e += GTB)
      if (e % n < e / n) S[e] = 0.0;
    __syncthreads();
  }
  for (int e = tid; e < n * n; e += GTB) it.N[(e % n) + (size_t)(e / n) * it.ld] = S[e];
}

// Triangular solve with a dense leaf factor T (n x n, n <= 64) on TRSM_COLS
// columns of X, starting at column col0 (column j of op(X) is row j of X when
// xtrans).  T goes to LDS with an odd leading dimension; wave w solves columns
// col0 + 8 w .. + 7, lane i holding row i of each.  Every substitution step
// broadcasts the finished entry p of each column from lane p and updates the
// remaining rows with one FMA each, in the order of increasing p (forward
// solves) or decreasing p (backward solve).
constexpr int TRSM_COLS = 32;
constexpr int TRSM_WCOLS = 8;
constexpr int TRSM_TB = 64 * TRSM_COLS / TRSM_WCOLS;

__global__ __launch_bounds__(TRSM_TB) void trsm_kernel(const DTrsm* __restrict__ items) {
  extern __shared__ double S[];
  const DTrsm it = items[blockIdx.x];
  const int n = it.n, ld = n | 1;
  const int c = rd(it.c);
  for (int e = threadIdx.x; e < n * n; e += TRSM_TB) S[(e % n) + (e / n) * ld] = it.T[(e % n) + (size_t)(e / n) * it.ldt];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j0 = it.col0 + wave * TRSM_WCOLS;
  if (j0 >= c) return;  // no barrier below
  const int nc = min(TRSM_WCOLS, c - j0);
  const bool row = lane < n;
  double x[TRSM_WCOLS];
#pragma unroll
  for (int k = 0; k < TRSM_WCOLS; ++k) {
    const size_t j = j0 + k;
    x[k] = (k < nc && row) ? (it.xtrans ? it.X[j + (size_t)lane * it.ldx] : it.X[lane + j * it.ldx]) : 0.0;
  }
  if (it.kind == TRSM_L_UNIT) {
    // L unit lower (strict lower part of T)
    for (int p = 0; p + 1 < n; ++p) {
      const double t = (row && lane > p) ? S[lane + p * ld] : 0.0;
#pragma unroll
      for (int k = 0; k < TRSM_WCOLS; ++k) {
        const double xp = lane_read(x[k], p);
        if (lane > p) x[k] = fma(-t, xp, x[k]);
      }
    }
  } else {
    // lane p holds 1 / T(p, p): one division per lane instead of one per
    // column and step
    const double rinv = row ? 1.0 / S[lane + lane * ld] : 0.0;
    if (it.kind == TRSM_RT || it.kind == TRSM_LC) {
      // forward with a lower factor: R^T, (R^T)(i, p) = T(p, i), or the lower
      // triangle of T itself
      const bool up = it.kind == TRSM_RT;
      for (int p = 0; p < n; ++p) {
        const double rp = lane_read(rinv, p);
        const double t = (row && lane > p) ? (up ? S[p + lane * ld] : S[lane + p * ld]) : 0.0;
#pragma unroll
        for (int k = 0; k < TRSM_WCOLS; ++k) {
          const double xp = lane_read(x[k], p) * rp;
          if (lane == p) x[k] = xp;
          else if (lane > p) x[k] = fma(-t, xp, x[k]);
        }
      }
    } else {
      // R upper, backward
      for (int p = n - 1; p >= 0; --p) {
        const double rp = lane_read(rinv, p);
        const double t = lane < p ? S[lane + p * ld] : 0.0;
#pragma unroll
        for (int k = 0; k < TRSM_WCOLS; ++k) {
          const double xp = lane_read(x[k], p) * rp;
          if (lane == p) x[k] = xp;
          else if (lane < p) x[k] = fma(-t, xp, x[k]);
        }
      }
    }
  }
  if (row) {
#pragma unroll
    for (int k = 0; k < TRSM_WCOLS; ++k) {
      if (k >= nc) break;
      const size_t j = j0 + k;
      if (it.xtrans)
        it.X[j + (size_t)lane * it.ldx] = x[k];
      else
        it.X[lane + j * it.ldx] = x[k];
    }
  }
}

__global__ __launch_bounds__(GTB) void copy_kernel(const DCopy* __restrict__ items) {
  const DCopy it = items[blockIdx.x];
  const int m = rd(it.m), n = rd(it.n);
  for (int e = threadIdx.x; e < m * n; e += GTB) {
    const int i = e % m, j = e / m;
    double v;
    if (it.mode == COPY_ZERO)
      v = 0.0;
    else if (it.mode == COPY_IDENTITY)
      v = (i == j) ? 1.0 : 0.0;
    else
      v = it.alpha * (it.strans ? it.src[j + (size_t)i * it.lds] : it.src[i + (size_t)j * it.lds]);
    it.dst[i + (size_t)j * it.ldd] = v;
  }
  if (threadIdx.x == 0 && it.rank_dst) *it.rank_dst = it.rank_src ? *it.rank_src : 0;
}

__global__ void nan_scan_kernel(const double* __restrict__ p, int64_t n, int* flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = p[i];
    if (!(v == v) || v > 1.7e308 || v < -1.7e308) {
      atomicOr(flag, 1);
      return;
    }
  }
}

}  // namespace

// p[0 .. n) = v (counters and flags reset at the start of a run; a kernel
// rather than a memset, so that the reset can be captured in a graph)
__global__ void fill_u32_kernel(unsigned int* __restrict__ p, int64_t n, unsigned int v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

hipError_t launch_fill_u32(unsigned int* p, int64_t n, unsigned int v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_nan_scan(const double* p, int64_t n, int* flag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(nan_scan_kernel, dim3(blocks), dim3(256), 0, s, p, n, flag);
  return hipGetLastError();
}

hipError_t launch_gemm(const DGemm* items, const DGemmTerm* terms, int count, int prec, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (prec == PREC_FP32)
    hipLaunchKernelGGL(gemm_kernel<PREC_FP32>, dim3(count), dim3(GTB), 0, s, items, terms);
  else if (prec == PREC_BF16X3)
    hipLaunchKernelGGL(gemm_kernel<PREC_BF16X3>, dim3(count), dim3(GTB), 0, s, items, terms);
  else
    hipLaunchKernelGGL(gemm_kernel<PREC_FP64>, dim3(count), dim3(GTB), 0, s, items, terms);
  return hipGetLastError();
}

hipError_t launch_lu(const DLu* items, int count, int nmax, int* status, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(lu_kernel, dim3(count), dim3(GTB), (size_t)nmax * nmax * sizeof(double), s, items,
                     status);
  return hipGetLastError();
}

hipError_t launch_trsm(const DTrsm* items, int count, int nmax, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (nmax > 64) return hipErrorInvalidValue;  // one wave row per leaf row
  const size_t lds = (size_t)nmax * (nmax | 1) * sizeof(double);
  hipLaunchKernelGGL(trsm_kernel, dim3(count), dim3(TRSM_TB), lds, s, items);
  return hipGetLastError();
}

hipError_t launch_copy(const DCopy* items, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_kernel, dim3(count), dim3(GTB), 0, s, items);
  return hipGetLastError();
}

}  // namespace hm
