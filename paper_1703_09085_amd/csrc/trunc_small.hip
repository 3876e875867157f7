// Truncation of small blocks (m, n <= 64) for gfx950 (FP64 core; the
// stacked-factor contractions in FP64, FP32 or split-BF16x3).
//
// Same operation as the general truncation kernel: the truncated sum
// R = sum_p alpha_p A_p B_p^T of up to four factor pairs (Fig. rkadd and the
// stages of Fig. rkmerge), with the rank chosen by the relative Frobenius rule.
// For blocks of at most 64 x 64 the sum itself is smaller than the stacked
// factors once the stacked rank l exceeds about m / 2, so this kernel works on
// the dense sum:
//   1. K^T = B_s A_s^T (n x m), streamed through LDS in chunks of 16 stacked
//      columns, then scaled by a power of two so that max |K| is in [1, 2)
//   2. Householder QR with column pivoting K^T P = Q R (only R is kept),
//      stopped once the remaining columns are at the rounding level;
//      M = R^T (rows in the original order, qe columns) has the singular
//      values and left singular vectors of K
//   3. one-sided Jacobi on the qe columns of M: M W = U S
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

#include <type_traits>

#include "core.h"
#include "dev_util.h"
#include "hm_types.h"
#include "mixed.h"
#include "tiny.h"

namespace hm {

namespace {

constexpr int SCH = 16;                // stacked columns staged per chunk
constexpr int SCLD = 18;               // staged rows are row-major with this stride
constexpr int SMALL_LDS = 2 * CBUF * 8 + 2 * CMAX * 8;  // two core buffers + reflector pair
constexpr int SMALL_LDS_PRED = SMALL_LDS + 4 * CMAX * 8;  // + the 4-column sketch of the features
constexpr int FEAT_LOG = 10;  // floats per item of the feature log: 8 features, k^, outcome

struct SmallShared {
  DTruncPart part[4];
  int k[4];
  int coff[4];
  int l, skip, rank, khat, accepted;
  float feat[MLP_IN];
  float h1[MLP_H];
  double kk, r2;
  CoreShared core;
};

// sum over the block of one value per group of STPC lanes (taken from lane 0
// of each group); every thread gets the result
template <int STPC>
__device__ __forceinline__ double block_group_sum(double v, int g, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(g == 0 ? v : 0.0);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < STPC; ++i) s += red[i];
  __syncthreads();
  return s;
}

// Eigenvalues of a symmetric 4 x 4 matrix (cyclic Jacobi, one thread), sorted
// descending.
__device__ __forceinline__ void eig4(double (&a)[4][4], double (&ev)[4]) {
  for (int sweep = 0; sweep < 12; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int p = 0; p < 4; ++p) {
      diag += a[p][p] * a[p][p];
      for (int q = p + 1; q < 4; ++q) off += a[p][q] * a[p][q];
    }
    if (off <= 1e-32 * diag) break;
    for (int p = 0; p < 3; ++p)
      for (int q = p + 1; q < 4; ++q) {
        const double apq = a[p][q];
        if (fabs(apq) <= 1e-300) continue;
        const double th = (a[q][q] - a[p][p]) / (2.0 * apq);
        const double t = copysign(1.0, th) / (fabs(th) + sqrt(th * th + 1.0));
        const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < 4; ++k) {
          const double akp = a[k][p], akq = a[k][q];
          a[k][p] = cs * akp - sn * akq;
          a[k][q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < 4; ++k) {
          const double apk = a[p][k], aqk = a[q][k];
          a[p][k] = cs * apk - sn * aqk;
          a[q][k] = sn * apk + cs * aqk;
        }
      }
  }
  for (int i = 0; i < 4; ++i) ev[i] = a[i][i];
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j)
      if (ev[j] > ev[i]) {
        const double tmp = ev[i];
        ev[i] = ev[j];
        ev[j] = tmp;
      }
}

// Stage stacked columns [c0, c0 + SCH) of A_s (m rows) and B_s (n rows) into
// sA / sB, row-major with stride SCLD; zero outside the parts and the sizes.
template <int NT, typename T>
__device__ __forceinline__ void stage_chunk(const SmallShared& sh, int nparts, int m, int n, int l, int c0,
                                            T* __restrict__ sA, T* __restrict__ sB) {
  const int t = threadIdx.x;
  const int i = t & 63;
#pragma unroll
  for (int v = 0; v < SCH * 64 / NT; ++v) {
    const int u = (t >> 6) + (NT / 64) * v;
    const int col = c0 + u;
    const double a = stacked_elem(sh.part, sh.coff, nparts, 0, i, m, col, l);
    const double b = stacked_elem(sh.part, sh.coff, nparts, 1, i, n, col, l);
    sA[i * SCLD + u] = (T)a;
    sB[i * SCLD + u] = (T)b;
  }
}

}  // namespace

// Rank rule over the qe core singular values plus a residual r2 outside the
// core (one thread): smallest k with r2 + sum_{i>=k} s_i^2 <= eps^2 total,
// values at or below 1e-13 of the largest counting as zero; *bad for a NaN
// or infinite sum.
__device__ __forceinline__ int rank_rule_resid(const CoreShared& cs, int qe, double eps, double total, double r2,
                                               bool* bad) {
  *bad = !(total == total) || total > 1.7e308 || !(r2 == r2);
  if (*bad || !(total > 0.0)) return 0;
  const double thr = eps * eps * total;
  double tail = r2;
  int k = qe;
  for (int j = qe - 1; j >= 0; --j) {
    const double s = cs.sig[cs.order[j]];
    tail += s * s;
    if (tail <= thr) k = j;
  }
  const double fl = 1e-13 * cs.sig[cs.order[0]];
  int nz = 0;
  while (nz < qe && cs.sig[cs.order[nz]] > fl) ++nz;
  return k < nz ? k : nz;
}

// Features of the truncation and the network's rank estimate (sh.khat).  w
// holds W = K^T (scaled), group c row c of K.  Uses buf2 for the sketch and
// wscratch (8 KB of LDS) for the network's second weight matrix.
template <int STPC>
__device__ __forceinline__ void predictor_features(const double (&w)[CMAX / STPC], int c, int g, int m, int n, int l,
                                                   int q, int level, const DPredictor& P, SmallShared& sh,
                                                   double* __restrict__ buf2, double* wscratch, float* feat) {
  constexpr int R = CMAX / STPC;
  const int t = threadIdx.x, lane = t & 63;
  double kk = 0.0;
#pragma unroll
  for (int s = 0; s < R; ++s) kk = fma(w[s], w[s], kk);
  kk = block_group_sum<STPC>(gsum<STPC>(kk), g, sh.core.red);
  // sketch Y4 = K omega(:, 0:4) (row c by group c)
  for (int j = 0; j < 4; ++j) {
    double y = 0.0;
#pragma unroll
    for (int s = 0; s < R; ++s) y = fma(w[s], P.omega[g + STPC * s + CMAX * j], y);
    y = gsum<STPC>(y);
    if (g == 0) buf2[c + CMAX * j] = c < m ? y : 0.0;
  }
  __syncthreads();
  if (t < 64) {
    // 4 x 4 Gram matrix of the sketch by wave reductions (rows >= m are zero)
    double y[4], gm[10];
#pragma unroll
    for (int j = 0; j < 4; ++j) y[j] = buf2[t + CMAX * j];
    int e = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = i; j < 4; ++j) gm[e++] = wave_sum(y[i] * y[j]);
    if (t == 0) {
      double a[4][4];
      e = 0;
      for (int i = 0; i < 4; ++i)
        for (int j = i; j < 4; ++j) {
          a[i][j] = gm[e];
          a[j][i] = gm[e];
          ++e;
        }
      double ev[4];
      eig4(a, ev);
      const double kn = sqrt(kk);
      sh.kk = kk;
      sh.feat[0] = (float)level;
      sh.feat[1] = (float)log2((double)m);
      sh.feat[2] = (float)log2((double)n);
      sh.feat[3] = (float)log2(1.0 + l);
      for (int j = 0; j < 4; ++j) sh.feat[4 + j] = (float)log10(fmax(sqrt(fmax(ev[j], 0.0)) / kn, 1e-30));
      if (feat)
        for (int j = 0; j < MLP_IN; ++j) feat[j] = sh.feat[j];
    }
  }
  __syncthreads();
  if (P.mode == 1) {
    // network: wave 0, lane j computes hidden unit j of each layer; W2 is
    // staged transposed in LDS (buf1 is free here) so that the lanes read
    // consecutive entries
    uint16_t* const sW2 = (uint16_t*)wscratch;
    for (int e = t; e < MLP_H * MLP_H; e += blockDim.x) sW2[(e % MLP_H) * MLP_H + e / MLP_H] = P.w.W2[e];
    if (t < MLP_H) {
      float a = P.w.b1[t];
#pragma unroll
      for (int i = 0; i < MLP_IN; ++i) a = fmaf(bf16_as_f32(P.w.W1[t * MLP_IN + i]), sh.feat[i], a);
      sh.h1[t] = a > 0.f ? a : 0.f;
    }
    __syncthreads();
    if (t < MLP_H) {
      float a = P.w.b2[t];
      for (int i = 0; i < MLP_H; ++i) a = fmaf(bf16_as_f32(sW2[i * MLP_H + t]), sh.h1[i], a);
      const double y = wave_sum((double)(bf16_as_f32(P.w.w3[t]) * (a > 0.f ? a : 0.f))) + (double)P.w.b3[0];
      if (lane == 0) {
        const double kh = ceil(exp2(fmin(y, 7.0)) - 1.0);
        sh.khat = kh < 0.0 ? 0 : (kh > q ? q : (int)kh);
      }
    }
  }
  __syncthreads();
}

// Items per block of the one-wave path (blocks up to 32 x 32): waves 0..3.
constexpr int TINY_PER_BLOCK = 4;
// modes of the ntiny argument below zero (descriptors made on the device)
constexpr int SMALL_PICK = -1;        // the caller's: the two passes below
constexpr int SMALL_TINY_PASS = -2;   // items of at most 32 x 32, one per wave
constexpr int SMALL_BLOCK_PASS = -3;  // the other items, one per block
static_assert(TINY_PER_BLOCK * TINY_LDS <= SMALL_LDS, "the one-wave items fit the block's LDS");

// STPC threads per column (4 or 8): 64 STPC threads, CMAX / STPC rows each.
// The first ntiny items (m, n <= 32) go to the first tiny_blocks blocks, one
// wave each (TINY_PER_BLOCK per block); every later block takes one of the
// other items.  In the tiny pass (ntiny == SMALL_TINY_PASS), tiny_blocks is
// the number of items.
template <int STPC, int PREC>
__global__ __launch_bounds__(64 * STPC) void trunc_small_kernel(const DTrunc* __restrict__ descs,
                                                                const DTruncPart* __restrict__ parts, int* status,
                                                                double eps, int* size_log, const DPredictor* pred,
                                                                float* feat_log, int ntiny, int tiny_blocks) {
  constexpr int STB = 64 * STPC;
  constexpr int SROWS = CMAX / STPC;
  extern __shared__ double smem[];
  __shared__ SmallShared sh;
  double* const buf0 = smem;
  double* const buf1 = smem + CBUF;
  double* const vbuf = smem + 2 * CBUF;  // two reflectors (double-buffered by step parity)
  double* const buf2 = vbuf + 2 * CMAX;  // with a predictor: the 4-column sketch
  // ntiny < 0: the sizes are known on the device only (descriptors made
  // there).  TINY_PASS: each wave takes one item and works on it only if it
  // is at most 32 x 32; BLOCK_PASS: each block takes one item and skips those
  // (the tiny pass's); PICK: each block takes one item, and one of at most
  // 32 x 32 goes to its first wave.  Each item gets the same arithmetic as
  // with ntiny >= 0.
  const bool pick_here = ntiny < 0;
  if (ntiny == SMALL_TINY_PASS) {
    const int wv = (int)(threadIdx.x >> 6);
    const int item = (int)blockIdx.x * TINY_PER_BLOCK + wv;
    if (wv < TINY_PER_BLOCK && item < tiny_blocks) {
      const DTrunc d = descs[item];
      if (d.m <= TINY_MAX && d.n <= TINY_MAX)
        trunc_tiny_item(d, parts, status, eps, size_log,
                        *reinterpret_cast<TinyShared*>(reinterpret_cast<char*>(smem) + (size_t)wv * TINY_LDS), item);
    }
    return;
  }
  if (!pick_here && (int)blockIdx.x < tiny_blocks) {
    const int wv = (int)(threadIdx.x >> 6);
    const int item = (int)blockIdx.x * TINY_PER_BLOCK + wv;
    if (wv < TINY_PER_BLOCK && item < ntiny)
      trunc_tiny_item(descs[item], parts, status, eps, size_log,
                      *reinterpret_cast<TinyShared*>(reinterpret_cast<char*>(smem) + (size_t)wv * TINY_LDS), item);
    return;
  }
  const int idx = pick_here ? (int)blockIdx.x : ntiny + (int)blockIdx.x - tiny_blocks;
  const DTrunc d = descs[idx];
  if ((d.flags & TRUNC_CLASS_CHECK) && (d.m > TRUNC_SMALL_MAX || d.n > TRUNC_SMALL_MAX)) return;  // another kernel's
  if (pick_here && !pred && d.m <= TINY_MAX && d.n <= TINY_MAX) {
    if (ntiny == SMALL_PICK && threadIdx.x < 64)
      trunc_tiny_item(d, parts, status, eps, size_log, *reinterpret_cast<TinyShared*>(smem), idx);
    return;  // BLOCK_PASS: done by the tiny pass
  }
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int c = t / STPC, rho = t % STPC;
  const int m = d.m, n = d.n;
  if (t < 64) {
    const StackCounts sc = stacked_counts(parts, d.part0, d.nparts, sh.k, sh.coff, sh.part);
    if (t == 0) {
      sh.l = sc.l;
      sh.skip = ((d.flags & TRUNC_SKIP_IF_PART0_EMPTY) && sc.k0 == 0) ||
               ((d.flags & TRUNC_SKIP_IF_HEAD_EMPTY) && sc.l == sc.klast);
    }
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
  float* const sAf = (float*)buf1;  // the reduced-precision modes stage FP32
  float* const sBf = sAf + CMAX * SCLD;
  if constexpr (PREC == PREC_FP64) {
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
  } else if constexpr (PREC == PREC_FP32) {
    float wf[SROWS];
#pragma unroll
    for (int s = 0; s < SROWS; ++s) wf[s] = 0.f;
    for (int c0 = 0; c0 < l; c0 += SCH) {
      stage_chunk<STB>(sh, d.nparts, m, n, l, c0, sAf, sBf);
      __syncthreads();
#pragma unroll
      for (int u = 0; u < SCH; u += 2) {
        const float2 a = *(const float2*)&sAf[c * SCLD + u];
#pragma unroll
        for (int s = 0; s < SROWS; ++s) {
          const float2 b = *(const float2*)&sBf[(rho + STPC * s) * SCLD + u];
          wf[s] = fmaf(a.x, b.x, wf[s]);
          wf[s] = fmaf(a.y, b.y, wf[s]);
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int s = 0; s < SROWS; ++s) w[s] = (double)wf[s];
  } else {
    // W = B_s A_s^T on the matrix cores: wave v < 4 forms the 32 x 32
    // quadrant (32 (v % 2), 32 (v / 2)) of W (rows: B_s, columns: A_s),
    // then W goes to the register layout through buf0
    const int rq = 32 * (wave & 1), cq = 32 * (wave >> 1), kg = 8 * (lane >> 5);
    f32x16 acc = zero_f32x16();
    for (int c0 = 0; c0 < l; c0 += SCH) {
      stage_chunk<STB>(sh, d.nparts, m, n, l, c0, sAf, sBf);
      __syncthreads();
      if (wave < 4) {
        float a[8], b[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          a[j] = sBf[(rq + (lane & 31)) * SCLD + kg + j];
          b[j] = sAf[(cq + (lane & 31)) * SCLD + kg + j];
        }
        acc = mfma_bf16x3(a, b, acc);
      }
      __syncthreads();
    }
    if (wave < 4) {
#pragma unroll
      for (int q = 0; q < 16; ++q)
        buf0[rq + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3) + CLD * (cq + (lane & 31))] = (double)acc[q];
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < SROWS; ++s) w[s] = buf0[rho + STPC * s + CLD * c];
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
  // rank predictor: features (logged) and the estimate k^.  With a width
  // wd = k^ + oversampling below q, the pivoted QR first stops after wd steps
  // (the first wd columns of Q are the range finder); the Jacobi on that core
  // and the exact residual |K - Q_wd Q_wd^T K|_F^2 (the remaining column
  // norms of the QR) decide the rank, and the result is kept when the
  // residual alone meets the bound.  Otherwise the same QR continues to the
  // exact stop.
  int outcome = 0;  // 0 exact, 1 range finder kept, 2 fell back
  int wd = 0;
  if (t == 0) sh.khat = -1;
  __syncthreads();
  float* feat = (pred && feat_log) ? feat_log + FEAT_LOG * (size_t)d.log_idx : nullptr;
  if (pred && finite && !zero) {
    __syncthreads();  // sh.core.red is reused
    predictor_features<STPC>(w, c, rho, m, n, l, q, d.level, *pred, sh, buf2, buf1, feat);
    wd = sh.khat + pred->oversample;
    if (!(pred->mode == 1 && sh.khat >= 0 && wd >= 1 && wd < q)) wd = 0;
  }
  int qe = q;  // width of the Jacobi core
  if (finite && !zero) {
    // 2. Householder QR of W (n x m) with column pivoting; M = R(0:qe, :)^T;
    //    3. Jacobi on its qe columns; 4. singular values
    __syncthreads();  // sh.core.red is reused below
    QrcpState st;
    qe = core_qrcp<STPC>(w, c, rho, n, m, vbuf, sh.core, 0, wd > 0 ? wd : CMAX, st);
    if (wd > 0 && st.capped) {
      core_to_m_piv<STPC>(w, x, c, rho, m, qe, st.mine, buf0);
      sweeps = core_jacobi<STPC>(x, a, rho, qe, buf0, buf1, sh.core);
      core_order<STPC>(x, a, rho, qe, sh.core);
      if (t == 0) {
        bool bad = false;
        const int k = rank_rule_resid(sh.core, qe, eps, st.total, st.resid, &bad);
        sh.rank = k;
        sh.accepted = !bad && st.resid <= eps * eps * st.total;
      }
      __syncthreads();
      outcome = sh.accepted ? 1 : 2;
      if (outcome == 2) qe = core_qrcp<STPC>(w, c, rho, n, m, vbuf, sh.core, qe, CMAX, st);
    }
    if (outcome != 1) {
      core_to_m_piv<STPC>(w, x, c, rho, m, qe, st.mine, buf0);
      clk1 = clock64();
      sweeps = core_jacobi<STPC>(x, a, rho, qe, buf0, buf1, sh.core);
      clk2 = clock64();
      core_order<STPC>(x, a, rho, qe, sh.core);
    }
  }
  if (t == 0 && feat) {
    feat[8] = (float)sh.khat;
    feat[9] = (float)outcome;
  }
  if (t == 0) {
    int k = 0;
    bool bad = !finite;
    if (outcome == 1)
      k = sh.rank;
    else if (finite && !zero)
      k = rank_rule(sh.core, qe, eps, &bad);
    if (d.kfix >= 0 && finite && !zero) k = d.kfix < qe ? d.kfix : qe;
    if (outcome == 1) atomicAdd((unsigned long long*)(status + 8), 1ULL);
    if (outcome == 2) atomicAdd((unsigned long long*)(status + 10), 1ULL);
    if (bad) {
      atomicOr(status, ST_NONFINITE);
      atomicExch(status + 1, idx + 1);
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
      e[4] = sweeps < 0 ? sweeps : sweeps | (qe << 16);  // Jacobi sweeps, core width
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
    const int pos = (a < qe) ? sh.core.pos_of[a] : CMAX;
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
    //    (FP32 in the reduced-precision modes)
    using DT = typename std::conditional<PREC == PREC_FP64, double, float>::type;
    using DT2 = typename std::conditional<PREC == PREC_FP64, double2, float2>::type;
    DT* const tA = (DT*)buf1;
    DT* const tB = tA + CMAX * SCLD;
    DT* const sT = tA + 2 * CMAX * SCLD;  // T(u, pos) at u + SCH * pos
    DT dacc[SROWS];
#pragma unroll
    for (int s = 0; s < SROWS; ++s) dacc[s] = 0;
    for (int c0 = 0; c0 < l; c0 += SCH) {
      stage_chunk<STB>(sh, d.nparts, m, n, l, c0, tA, tB);
      __syncthreads();
#pragma unroll
      for (int v = 0; v < SCH * CMAX / STB; ++v) {
        const int u = t & (SCH - 1), p = t / SCH + (STB / SCH) * v;
        if (p < k) {
          DT acc = 0;
          for (int i = 0; i < m; ++i) acc = fma(tA[i * SCLD + u], (DT)buf0[i + CLD * p], acc);
          sT[u + SCH * p] = acc;
        }
      }
      __syncthreads();
      if (c < k) {
#pragma unroll
        for (int u = 0; u < SCH; u += 2) {
          const DT t0 = sT[u + SCH * c], t1 = sT[u + 1 + SCH * c];
#pragma unroll
          for (int s = 0; s < SROWS; ++s) {
            const DT2 b = *(const DT2*)&tB[(rho + STPC * s) * SCLD + u];
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
        if (j < n) d.D[j + (size_t)d.ldd * c] = (double)dacc[s];
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
// pred (device, may be NULL): rank predictor; feat_log (device, may be NULL):
// FEAT_LOG floats per item (features, k^, outcome) when a predictor is given.
// prec: arithmetic of the two stacked-factor contractions (Precision); the
// core SVD and the rank rule are FP64 in every mode.
template <int PREC>
static void launch_small_prec(const DTrunc* descs, const DTruncPart* parts, int count, int* status, double eps,
                              int* size_log, int tpc, const DPredictor* pred, float* feat_log, int ntiny,
                              hipStream_t stream) {
  const int lds = pred ? SMALL_LDS_PRED : SMALL_LDS;
  if (ntiny == SMALL_PICK) {
    // sizes known on the device only: a pass of TINY_PER_BLOCK items per
    // block for those of at most 32 x 32, then a pass of one item per block
    // for the others
    const int tgrid = (count + TINY_PER_BLOCK - 1) / TINY_PER_BLOCK;
    hipLaunchKernelGGL((trunc_small_kernel<4, PREC>), dim3(tgrid), dim3(256), lds, stream, descs, parts, status, eps,
                       size_log, pred, feat_log, SMALL_TINY_PASS, count);
    ntiny = SMALL_BLOCK_PASS;
  }
  const int tb = ntiny > 0 ? (ntiny + TINY_PER_BLOCK - 1) / TINY_PER_BLOCK : 0;
  const int grid = tb + (count - (ntiny > 0 ? ntiny : 0));
  if (tpc == 8)
    hipLaunchKernelGGL((trunc_small_kernel<8, PREC>), dim3(grid), dim3(512), lds, stream, descs, parts, status,
                       eps, size_log, pred, feat_log, ntiny, tb);
  else
    hipLaunchKernelGGL((trunc_small_kernel<4, PREC>), dim3(grid), dim3(256), lds, stream, descs, parts, status,
                       eps, size_log, pred, feat_log, ntiny, tb);
}

// ntiny >= 0: the first ntiny items have m, n <= 32 and run one per wave
// (FP64 contractions whatever prec says); ntiny < 0: the kernel sends each
// item of at most 32 x 32 to a wave itself (descriptors made on the device).
// With a predictor, whose features the one-wave path does not form, every
// item takes the block-wide path.
hipError_t launch_trunc_small(const DTrunc* descs, const DTruncPart* parts, int count, int* status, double eps,
                              int* size_log, int tpc, const DPredictor* pred, float* feat_log, int prec,
                              hipStream_t stream, int ntiny) {
  if (count <= 0) return hipSuccess;
  if (pred) ntiny = 0;
  if (ntiny > count) ntiny = count;
  if (prec == PREC_FP32)
    launch_small_prec<PREC_FP32>(descs, parts, count, status, eps, size_log, tpc, pred, feat_log, ntiny, stream);
  else if (prec == PREC_BF16X3)
    launch_small_prec<PREC_BF16X3>(descs, parts, count, status, eps, size_log, tpc, pred, feat_log, ntiny, stream);
  else
    launch_small_prec<PREC_FP64>(descs, parts, count, status, eps, size_log, tpc, pred, feat_log, ntiny, stream);
  return hipGetLastError();
}

}  // namespace hm
