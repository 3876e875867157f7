// Truncation of small blocks (m, n <= 64) for gfx950 (FP64).
//
// Same operation as the general truncation kernel: the truncated sum
// R = sum_p alpha_p A_p B_p^T of up to four factor pairs (Fig. rkadd and the
// stages of Fig. rkmerge), with the rank chosen by the relative Frobenius rule.
// For blocks of at most 64 x 64 the sum itself is smaller than the stacked
// factors once the stacked rank l exceeds about m / 2, so this kernel works on
// the dense sum:
//   1. K^T = B_s A_s^T (n x m), streamed through LDS in chunks of 16 stacked
//      columns, then scaled by a power of two so that max |K| is in [1, 2)
//   2. Householder QR K^T = Q R (only R is kept); M = R^T has the singular
//      values and left singular vectors of K
//   3. one-sided Jacobi on the columns of M: M W = U S
//   4. rank rule on S
//   5. C = U_k and D = K^T U_k = B_s (A_s^T U_k), recomputed from the stacks
// The result equals the best rank-k approximation of the sum, as in Fig. rkadd,
// to rounding.
//
// One workgroup per item, 4 or 8 threads per column (256 or 512 threads).
// Thread t works on column t / TPC of the current matrix and on its rows
// r = t % TPC + TPC s, held in registers; the lanes of a column combine their
// partial sums with two or three DPP steps, so a column's dot product costs no
// LDS round trip.  Two matrix buffers of 64 x 68 doubles in LDS (about 70 KB)
// allow two 256-thread workgroups per compute unit.
#include <hip/hip_runtime.h>

#include "core.h"
#include "dev_util.h"
#include "hm_types.h"

namespace hm {

namespace {

constexpr int SCH = 16;                // stacked columns staged per chunk
constexpr int SCLD = 18;               // staged rows are row-major with this stride
constexpr int SMALL_LDS = 2 * CBUF * 8 + 2 * CMAX * 8;  // two core buffers + reflector pair

struct SmallShared {
  DTruncPart part[4];
  int k[4];
  int coff[4];
  int l, skip, rank;
  CoreShared core;
};

// Stage stacked columns [c0, c0 + SCH) of A_s (m rows) and B_s (n rows) into
// sA / sB, row-major with stride SCLD; zero outside the parts and the sizes.
template <int NT>
__device__ __forceinline__ void stage_chunk(const SmallShared& sh, int nparts, int m, int n, int l, int c0,
                                            double* __restrict__ sA, double* __restrict__ sB) {
  const int t = threadIdx.x;
  const int i = t & 63;
#pragma unroll
  for (int v = 0; v < SCH * 64 / NT; ++v) {
    const int u = (t >> 6) + (NT / 64) * v;
    const int col = c0 + u;
    double a = 0.0, b = 0.0;
    if (col < l) {
      int p = 0;
      while (p + 1 < nparts && col >= sh.coff[p + 1]) ++p;
      const DTruncPart& P = sh.part[p];
      const int cc = col - sh.coff[p];
      const int ra = i - P.row_off;
      if (i < m && ra >= 0 && ra < P.rows)
        a = P.alpha * (P.ta ? P.A[cc + (size_t)ra * P.lda] : P.A[ra + (size_t)cc * P.lda]);
      const int rb = i - P.col_off;
      if (i < n && rb >= 0 && rb < P.cols) b = P.tb ? P.B[cc + (size_t)rb * P.ldb] : P.B[rb + (size_t)cc * P.ldb];
    }
    sA[i * SCLD + u] = a;
    sB[i * SCLD + u] = b;
  }
}

}  // namespace

// STPC threads per column (4 or 8): 64 STPC threads, CMAX / STPC rows each.
template <int STPC>
__global__ __launch_bounds__(64 * STPC) void trunc_small_kernel(const DTrunc* __restrict__ descs,
                                                                const DTruncPart* __restrict__ parts, int* status,
                                                                double eps, int* size_log) {
  constexpr int STB = 64 * STPC;
  constexpr int SROWS = CMAX / STPC;
  extern __shared__ double smem[];
  __shared__ SmallShared sh;
  double* const buf0 = smem;
  double* const buf1 = smem + CBUF;
  double* const vbuf = smem + 2 * CBUF;  // two reflectors (double-buffered by step parity)
  const DTrunc d = descs[blockIdx.x];
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int c = t / STPC, rho = t % STPC;
  const int m = d.m, n = d.n;
  if (t < d.nparts) sh.part[t] = parts[d.part0 + t];
  __syncthreads();
  if (t == 0) {
    int l = 0;
    for (int p = 0; p < d.nparts; ++p) {
      const int kp = rdim(sh.part[p].k);
      sh.k[p] = kp;
      sh.coff[p] = l;
      l += kp;
    }
    sh.l = l;
    sh.skip = (d.flags & TRUNC_SKIP_IF_PART0_EMPTY) && sh.k[0] == 0;
  }
  __syncthreads();
  if (sh.skip) return;
  const int l = sh.l;
  if (l == 0) {
    if (t == 0) *d.rank = 0;
    return;
  }
  const long long clk0 = clock64();

  // 1. W = K^T: thread (c, rho) accumulates W(rho + STPC s, c) = K(c, rho + STPC s)
  double w[SROWS];
#pragma unroll
  for (int s = 0; s < SROWS; ++s) w[s] = 0.0;
  double* const sA = buf1;
  double* const sB = buf1 + CMAX * SCLD;
  for (int c0 = 0; c0 < l; c0 += SCH) {
    stage_chunk<STB>(sh, d.nparts, m, n, l, c0, sA, sB);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < SCH; u += 2) {
      const double2 a = *(const double2*)&sA[c * SCLD + u];
#pragma unroll
      for (int s = 0; s < SROWS; ++s) {
        const double2 b = *(const double2*)&sB[(rho + STPC * s) * SCLD + u];
        w[s] = fma(a.x, b.x, w[s]);
        w[s] = fma(a.y, b.y, w[s]);
      }
    }
    __syncthreads();
  }
  // scale by a power of two: max |K| in [1, 2)
  double amax = 0.0;
#pragma unroll
  for (int s = 0; s < SROWS; ++s) amax = fmax(amax, fabs(w[s]));
  amax = wave_max(amax);
  if (lane == 0) sh.core.red[wave] = amax;
  __syncthreads();
  amax = 0.0;
#pragma unroll
  for (int i = 0; i < STB / 64; ++i) amax = fmax(amax, sh.core.red[i]);
  const bool finite = amax <= 1.7976931348623157e308;  // false for NaN and inf
  const bool zero = amax == 0.0;
  if (finite && !zero) {
    const int e = ilogb(amax);
#pragma unroll
    for (int s = 0; s < SROWS; ++s) w[s] = ldexp(w[s], -e);
  }
  const int q = m < n ? m : n;  // singular values of the m x n sum
  const int a = c;              // Jacobi: group a holds column a of M
  double x[SROWS];
#pragma unroll
  for (int s = 0; s < SROWS; ++s) x[s] = 0.0;
  int sweeps = 0;
  long long clk1 = clk0, clk2 = clk0;
  if (finite && !zero) {
    // 2. Householder QR of W (n x m), M = R^T; 3. Jacobi; 4. singular values
    __syncthreads();  // sh.core.red is reused below
    core_qr<STPC>(w, c, rho, n, m, vbuf, sh.core);
    core_to_m<STPC>(w, x, c, rho, n, m, buf0);
    clk1 = clock64();
    sweeps = core_jacobi<STPC>(x, a, rho, q, buf0, buf1, sh.core);
    clk2 = clock64();
    core_order<STPC>(x, a, rho, q, sh.core);
  }
  if (t == 0) {
    int k = 0;
    bool bad = !finite;
    if (finite && !zero) k = rank_rule(sh.core, q, eps, &bad);
    if (bad) {
      atomicOr(status, ST_NONFINITE);
      atomicExch(status + 1, (int)blockIdx.x + 1);
      k = 0;
    }
    if (k > d.cap) {
      atomicOr(status, ST_RANK_OVERFLOW);
      k = d.cap;
    }
    sh.rank = k;
    if (size_log) {
      int* e = size_log + 8 * (size_t)d.log_idx;
      e[0] = m;
      e[1] = n;
      e[2] = l;
      e[3] = k;
      e[4] = sweeps;
      e[5] = (int)((clk1 - clk0) >> 4);
      e[6] = (int)((clk2 - clk1) >> 4);
    }
    atomicAdd((unsigned long long*)(status + 2), 1ULL);
    const unsigned long long bytes = 8ULL * (unsigned long long)(m + n) * (unsigned long long)(l + k);
    atomicAdd((unsigned long long*)(status + 4), bytes);
    atomicAdd((unsigned long long*)(status + 6), bytes);  // this kernel's share
  }
  __syncthreads();
  const int k = sh.rank;
  const long long clk3 = clock64();
  if (k > 0) {
    // 5. U_k into buf0 (column-major, ld CLD): U(:, pos) = M(:, order[pos]) / s
    const int pos = (a < q) ? sh.core.pos_of[a] : CMAX;
    if (pos < k) {
      const double sa = sh.core.sig[a];
#pragma unroll
      for (int s = 0; s < SROWS; ++s) {
        const int i = rho + STPC * s;
        buf0[i + CLD * pos] = (i < m && sa > 0.0) ? x[s] / sa : 0.0;
      }
    }
    __syncthreads();
    // 6. D = K^T U_k = B_s (A_s^T U_k), by chunks of SCH stacked columns:
    //    T = A_chunk^T U_k (SCH x k), then thread (c, rho) adds B_chunk T to
    //    D(rho + STPC s, c) for c < k
    double dacc[SROWS];
#pragma unroll
    for (int s = 0; s < SROWS; ++s) dacc[s] = 0.0;
    double* const sT = buf1 + 2 * CMAX * SCLD;  // T(u, pos) at u + SCH * pos
    for (int c0 = 0; c0 < l; c0 += SCH) {
      stage_chunk<STB>(sh, d.nparts, m, n, l, c0, sA, sB);
      __syncthreads();
#pragma unroll
      for (int v = 0; v < SCH * CMAX / STB; ++v) {
        const int u = t & (SCH - 1), p = t / SCH + (STB / SCH) * v;
        if (p < k) {
          double acc = 0.0;
          for (int i = 0; i < m; ++i) acc = fma(sA[i * SCLD + u], buf0[i + CLD * p], acc);
          sT[u + SCH * p] = acc;
        }
      }
      __syncthreads();
      if (c < k) {
#pragma unroll
        for (int u = 0; u < SCH; u += 2) {
          const double t0 = sT[u + SCH * c], t1 = sT[u + 1 + SCH * c];
#pragma unroll
          for (int s = 0; s < SROWS; ++s) {
            const double2 b = *(const double2*)&sB[(rho + STPC * s) * SCLD + u];
            dacc[s] = fma(b.x, t0, dacc[s]);
            dacc[s] = fma(b.y, t1, dacc[s]);
          }
        }
      }
      __syncthreads();
    }
    // 7. outputs (every read of the stacks is done: they may alias C and D)
    for (int e = t; e < m * k; e += STB) {
      const int i = e % m, p = e / m;
      d.C[i + (size_t)d.ldc * p] = buf0[i + CLD * p];
    }
    if (c < k) {
#pragma unroll
      for (int s = 0; s < SROWS; ++s) {
        const int j = rho + STPC * s;
        if (j < n) d.D[j + (size_t)d.ldd * c] = dacc[s];
      }
    }
  }
  if (t == 0) {
    *d.rank = k;
    if (size_log) size_log[8 * (size_t)d.log_idx + 7] = (int)((clock64() - clk3) >> 4);
  }
}

// tpc: threads per column, 4 (256 threads, two workgroups per CU) or 8 (512
// threads, one workgroup per CU); the result is the same.
hipError_t launch_trunc_small(const DTrunc* descs, const DTruncPart* parts, int count, int* status, double eps,
                              int* size_log, int tpc, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  if (tpc == 8)
    hipLaunchKernelGGL(trunc_small_kernel<8>, dim3(count), dim3(512), SMALL_LDS, stream, descs, parts, status, eps,
                       size_log);
  else
    hipLaunchKernelGGL(trunc_small_kernel<4>, dim3(count), dim3(256), SMALL_LDS, stream, descs, parts, status, eps,
                       size_log);
  return hipGetLastError();
}

}  // namespace hm
