// One-wavefront truncation of larger blocks whose stacked rank is small
// (l <= 16), FP64, gfx950.
//
// The operation of the other truncation kernels (the truncated sum of up to
// four factor pairs, Fig. rkadd and the stages of Fig. rkmerge, rank by the
// relative Frobenius rule) with the steps of the register-resident kernel:
// Householder QR of both stacks, A_s = Q_A R_A and B_s = Q_B R_B; the core
// K^T = R_B R_A^T through the pivoted QR and one-sided Jacobi of the one-wave
// small path; C = Q_A [U_k; 0] and D = Q_B [R_B R_A^T U_k; 0].  One wave does
// all of it for one item, with no workgroup barrier.  A stack column belongs
// to LPC consecutive lanes (16, 8 or 4 as l <= 4, 8 or 16), each holding the
// rows g + LPC s, s < 32, so a stack may have up to 32 LPC rows; column sums
// are DPP reductions in the lane group, and a step's reflector reaches the
// other columns through the wave's LDS.  The reflectors of A_s wait in LDS
// while those of B_s stay in registers.
//
// The batch entry points (independent truncations, throughput-bound) launch
// it first on their larger items; it marks the items it takes in `done`, and
// the register-resident and general kernels, launched next on the same items,
// skip them (the rank it writes is the column count of one of the item's
// parts, so they cannot decide alone).  With four items in flight per
// compute unit (33 KB of LDS each) instead of one it raises the throughput of
// full batches.
// Plans do not launch it: their launches are latency-bound (a launch lasts as
// long as its slowest item), one wave takes about as long per item as the
// eight waves of the register-resident kernel (a Householder step is a chain
// of dependent operations of about a thousand cycles either way), and a
// kernel ahead of the register-resident one would add its latency to that
// kernel's.
#include <hip/hip_runtime.h>

#include "tiny.h"

namespace hm {

constexpr int THIN_LMAX = 16;  // stacked rank at most
constexpr int THIN_RPL = 32;   // stack rows per lane at most
constexpr int THIN_Q = 2048;   // doubles of one stack's reflectors (rows x l <= 32 LPC x 64 / LPC)
constexpr int THIN_RLD = 16;   // leading dimension of R_A, R_B, T and S in LDS

struct ThinShared {
  TinyShared t;      // parts and the core; R_A (later S = R_B T) in t.sA, R_B in t.sB, T in t.sT
  double q[THIN_Q];  // one stack's reflectors: column j below its diagonal at q + rows * j
  double tau[2 * THIN_LMAX];
  double step_tau;
};
static_assert(TINY_MAX * TSLD >= THIN_RLD * THIN_LMAX, "R factors fit the staging buffers");
static_assert(TSCH * TINY_MAX >= THIN_RLD * THIN_LMAX, "T fits its buffer");
static_assert(TINY_MAX * TMLD >= THIN_RPL * 16, "a step's reflector fits the core buffer");

__device__ __forceinline__ int thin_lpc(int l) { return l <= 4 ? 16 : (l <= 8 ? 8 : 4); }

__device__ __forceinline__ bool thin_fits(int m, int n, int l) {
  const int r = m > n ? m : n;
  return l >= 1 && l <= THIN_LMAX && r <= THIN_RPL * thin_lpc(l);
}

// Householder QR of one stack (rows x l; side 0: A_s with the first part's
// alpha, side 1: B_s), loaded into w (column lane / LPC, rows g + LPC s).
// Afterwards the group of column c holds R(0:c, c) in its rows <= c and the
// reflector of step c below (its row c is an implicit 1), with tau[c].
template <int LPC, int RPL>
__device__ __forceinline__ void thin_qr(ThinShared& sh, int nparts, int side, int rows, int l, double (&w)[RPL],
                                        double* tau) {
  const int lane = threadIdx.x & 63;
  const int c = lane / LPC, g = lane % LPC;
#pragma unroll
  for (int s = 0; s < RPL; ++s) w[s] = stacked_elem(sh.t.part, sh.t.coff, nparts, side, g + LPC * s, rows, c, l);
  const int q = rows < l ? rows : l;
  double* const vb = sh.t.buf;  // the step's reflector, rows 0 .. 32 LPC - 1
  for (int j = 0; j < q; ++j) {
    if (c == j) {
      double s2 = 0.0, al = 0.0;
#pragma unroll
      for (int s = 0; s < RPL; ++s) {
        const int r = g + LPC * s;
        s2 = r > j ? fma(w[s], w[s], s2) : s2;
        al = r == j ? w[s] : al;
      }
      s2 = lsum<LPC>(s2);
      al = lsum<LPC>(al);
      const bool nz = s2 > 0.0;
      const double beta = nz ? -copysign(sqrt_refined(fma(al, al, s2)), al) : al;
      const double tv = nz ? (beta - al) * rcp_refined(beta) : 0.0;
      const double inv = nz ? rcp_refined(al - beta) : 0.0;
#pragma unroll
      for (int s = 0; s < RPL; ++s) {
        const int r = g + LPC * s;
        const double v = r == j ? 1.0 : (r > j ? w[s] * inv : 0.0);
        vb[r] = v;
        w[s] = r == j ? beta : (r > j ? v : w[s]);
      }
      if (g == 0) {
        sh.step_tau = tv;
        tau[j] = tv;
      }
    }
    wave_sync();
    const double tv = sh.step_tau;
    if (c > j && c < l) {
      double v[RPL];
#pragma unroll
      for (int s = 0; s < RPL; ++s) v[s] = vb[g + LPC * s];
      double d0 = 0.0, d1 = 0.0;
#pragma unroll
      for (int s = 0; s < RPL; s += 2) {
        d0 = fma(v[s], w[s], d0);
        d1 = fma(v[s + 1], w[s + 1], d1);
      }
      const double f = tv * lsum<LPC>(d0 + d1);
#pragma unroll
      for (int s = 0; s < RPL; ++s) w[s] = fma(-f, v[s], w[s]);
    }
    wave_sync();
  }
}

// R(i, c) for i <= c, i < q into R[i + THIN_RLD c].
template <int LPC, int RPL>
__device__ __forceinline__ void thin_put_r(const double (&w)[RPL], int l, int q, double* R) {
  const int lane = threadIdx.x & 63;
  const int c = lane / LPC, g = lane % LPC;
  if (c < l) {
#pragma unroll
    for (int s = 0; s * LPC < THIN_RLD; ++s) {
      const int r = g + LPC * s;
      if (r <= c && r < q) R[r + THIN_RLD * c] = w[s];
    }
  }
}

// The reflectors of steps c < q (rows > c) into sh.q.
template <int LPC, int RPL>
__device__ __forceinline__ void thin_put_q(ThinShared& sh, const double (&w)[RPL], int rows, int q) {
  const int lane = threadIdx.x & 63;
  const int c = lane / LPC, g = lane % LPC;
  if (c < q) {
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      const int r = g + LPC * s;
      if (r > c && r < rows) sh.q[r + rows * c] = w[s];
    }
  }
}

// y <- H_0 H_1 ... H_{q-1} y for every column of y (column lane / LPC, rows
// g + LPC s), H_j = I - tau_j v_j v_j^T with v_j from sh.q.
template <int LPC, int RPL>
__device__ __forceinline__ void thin_apply(const ThinShared& sh, int rows, int q, const double* tau,
                                           double (&y)[RPL]) {
  const int g = (threadIdx.x & 63) % LPC;
  for (int j = q - 1; j >= 0; --j) {
    const double tv = tau[j];
    double v[RPL];
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      const int r = g + LPC * s;
      const bool below = r > j && r < rows;
      const double x = sh.q[below ? r + rows * j : 0];
      v[s] = below ? x : (r == j ? 1.0 : 0.0);
    }
    double d0 = 0.0, d1 = 0.0;
#pragma unroll
    for (int s = 0; s < RPL; s += 2) {
      d0 = fma(v[s], y[s], d0);
      d1 = fma(v[s + 1], y[s + 1], d1);
    }
    const double f = tv * lsum<LPC>(d0 + d1);
#pragma unroll
    for (int s = 0; s < RPL; ++s) y[s] = fma(-f, v[s], y[s]);
  }
}

// The core W = K^T = R_B R_A^T (qb x qa) in the layout of the one-wave small
// path (LPCC lanes per column), scaled and factored there.
template <int LPCC>
__device__ __forceinline__ TinyQr thin_core(ThinShared& sh, int l, int qa, int qb) {
  constexpr int R = TINY_MAX / LPCC;
  const int lane = threadIdx.x & 63;
  const int c = lane / LPCC, g = lane % LPCC;
  const double* RA = sh.t.sA;
  const double* RB = sh.t.sB;
  double w[R];
#pragma unroll
  for (int s = 0; s < R; ++s) {
    const int row = g + LPCC * s;
    double acc = 0.0;
    if (c < qa && row < qb) {
      const int p0 = c > row ? c : row;
      for (int p = p0; p < l; ++p) acc = fma(RB[row + THIN_RLD * p], RA[c + THIN_RLD * p], acc);
    }
    w[s] = acc;
  }
  return tiny_scaled_qr<LPCC>(sh.t, w, qa, qb);
}

template <int LPC, int RPL>
__device__ __forceinline__ void thin_item(const DTrunc& d, ThinShared& sh, int nparts, int l, int* status, double eps,
                                          int* size_log, int item) {
  const int lane = threadIdx.x & 63;
  const int c = lane / LPC, g = lane % LPC;
  const int m = d.m, n = d.n;
  const int qa = m < l ? m : l, qb = n < l ? n : l;
  double* const tauA = sh.tau;
  double* const tauB = sh.tau + THIN_LMAX;
  const long long clk0 = clock64();

  // 1. both stacks: R_A, R_B to LDS; the reflectors of A_s to sh.q, those of
  //    B_s stay in w
  double w[RPL];
  thin_qr<LPC, RPL>(sh, nparts, 0, m, l, w, tauA);
  thin_put_r<LPC, RPL>(w, l, qa, sh.t.sA);
  thin_put_q<LPC, RPL>(sh, w, m, qa);
  thin_qr<LPC, RPL>(sh, nparts, 1, n, l, w, tauB);
  thin_put_r<LPC, RPL>(w, l, qb, sh.t.sB);
  wave_sync();
  const long long clk1 = clock64();

  // 2. the core: pivoted QR and Jacobi of K^T = R_B R_A^T, rank rule, U_k
  //    (qa x k) in sh.t.buf
  const TinyQr qr = qa <= 8 ? thin_core<8>(sh, l, qa, qb) : thin_core<4>(sh, l, qa, qb);
  const int qe = qr.qe;
  bool bad = !qr.finite;
  auto rank_of = [&]() {
    int k = 0;
    if (qr.finite && !qr.zero) k = tiny_rank_rule(sh.t, qe, eps, &bad);
    if (d.kfix >= 0 && qr.finite && !qr.zero) k = d.kfix < qe ? d.kfix : qe;
    if (bad) k = 0;
    return k;
  };
  int k = 0, sweeps = 0;
  if (qr.finite && !qr.zero && qe > 0) {
    if (qe <= 8)
      sweeps = tiny_jacobi<8>(sh.t, qa, qe, rank_of, &k);
    else
      sweeps = tiny_jacobi<4>(sh.t, qa, qe, rank_of, &k);
  } else {
    k = rank_of();
  }
  const long long clk2 = clock64();
  if (k > d.cap) {
    if (lane == 0) atomicOr(status, ST_RANK_OVERFLOW);
    k = d.cap;
  }
  if (lane == 0) {
    if (bad) {
      atomicOr(status, ST_NONFINITE);
      atomicExch(status + 1, item + 1);
    }
    if (size_log) {
      int* e = size_log + 8 * (size_t)d.log_idx;
      e[0] = m;
      e[1] = n;
      e[2] = l;
      e[3] = k;
      e[4] = sweeps | (qe << 16);
      e[5] = (int)((clk1 - clk0) >> 4);
      e[6] = (int)((clk2 - clk1) >> 4);
    }
    atomicAdd((unsigned long long*)(status + 2), 1ULL);
    atomicAdd((unsigned long long*)(status + 4), 8ULL * (unsigned long long)(m + n) * (unsigned long long)(l + k));
  }

  if (k > 0) {
    // 3. T = R_A^T U_k (l x k), then S = R_B T (qb x k) over R_A
    double* const T = sh.t.sT;
    const double* RA = sh.t.sA;
    const double* RB = sh.t.sB;
    const double* U = sh.t.buf;
    for (int e = lane; e < l * k; e += 64) {
      const int p = e % l, cc = e / l;
      const int iend = p + 1 < qa ? p + 1 : qa;
      double acc = 0.0;
      for (int i = 0; i < iend; ++i) acc = fma(RA[i + THIN_RLD * p], U[i + TMLD * cc], acc);
      T[p + THIN_RLD * cc] = acc;
    }
    wave_sync();
    double* const S = sh.t.sA;
    for (int e = lane; e < qb * k; e += 64) {
      const int j = e % qb, cc = e / qb;
      double acc = 0.0;
      for (int p = j; p < l; ++p) acc = fma(RB[j + THIN_RLD * p], T[p + THIN_RLD * cc], acc);
      S[j + THIN_RLD * cc] = acc;
    }
    wave_sync();
    // 4. C = Q_A [U_k; 0] (every read of the stacks is done: C and D may
    //    alias them)
    double y[RPL];
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      const int r = g + LPC * s;
      y[s] = (c < k && r < qa) ? U[r + TMLD * c] : 0.0;
    }
    thin_apply<LPC, RPL>(sh, m, qa, tauA, y);
    if (c < k) {
#pragma unroll
      for (int s = 0; s < RPL; ++s) {
        const int r = g + LPC * s;
        if (r < m) d.C[r + (size_t)d.ldc * c] = y[s];
      }
    }
    wave_sync();
    // 5. D = Q_B [S; 0] with the reflectors of B_s moved to sh.q
    thin_put_q<LPC, RPL>(sh, w, n, qb);
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      const int r = g + LPC * s;
      y[s] = (c < k && r < qb) ? S[r + THIN_RLD * c] : 0.0;
    }
    wave_sync();
    thin_apply<LPC, RPL>(sh, n, qb, tauB, y);
    if (c < k) {
#pragma unroll
      for (int s = 0; s < RPL; ++s) {
        const int r = g + LPC * s;
        if (r < n) d.D[r + (size_t)d.ldd * c] = y[s];
      }
    }
  }
  if (lane == 0) {
    *d.rank = k;
    if (size_log) size_log[8 * (size_t)d.log_idx + 7] = (int)((clock64() - clk2) >> 4);
  }
}

__global__ __launch_bounds__(64) void trunc_thin_kernel(const DTrunc* __restrict__ descs,
                                                        const DTruncPart* __restrict__ parts, int* status, double eps,
                                                        int* size_log, int* done, int run_id) {
  __shared__ ThinShared sh;
  const DTrunc d = descs[blockIdx.x];
  if ((d.flags & TRUNC_CLASS_CHECK) && d.m <= TRUNC_SMALL_MAX && d.n <= TRUNC_SMALL_MAX) return;  // small-block kernel's
  const int lane = threadIdx.x;
  const StackCounts sc = stacked_counts(parts, d.part0, d.nparts, sh.t.k, sh.t.coff, sh.t.part);
  wave_sync();
  const int l = sc.l;
  const bool skip = ((d.flags & TRUNC_SKIP_IF_PART0_EMPTY) && sc.k0 == 0) ||
                    ((d.flags & TRUNC_SKIP_IF_HEAD_EMPTY) && l == sc.klast);
  if (skip || !thin_fits(d.m, d.n, l)) return;  // the other kernels' (l == 0 included)
  if (lane == 0) done[blockIdx.x] = run_id;
  const int lpc = thin_lpc(l);
  const bool r16 = (d.m > d.n ? d.m : d.n) <= 16 * lpc;
  const int item = (int)blockIdx.x;
  if (lpc == 16) {
    if (r16)
      thin_item<16, 16>(d, sh, d.nparts, l, status, eps, size_log, item);
    else
      thin_item<16, 32>(d, sh, d.nparts, l, status, eps, size_log, item);
  } else if (lpc == 8) {
    if (r16)
      thin_item<8, 16>(d, sh, d.nparts, l, status, eps, size_log, item);
    else
      thin_item<8, 32>(d, sh, d.nparts, l, status, eps, size_log, item);
  } else {
    if (r16)
      thin_item<4, 16>(d, sh, d.nparts, l, status, eps, size_log, item);
    else
      thin_item<4, 32>(d, sh, d.nparts, l, status, eps, size_log, item);
  }
}

hipError_t launch_trunc_thin(const DTrunc* descs, const DTruncPart* parts, int count, int* status, double eps,
                             int* size_log, int* done, int run_id, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(trunc_thin_kernel, dim3(count), dim3(64), 0, stream, descs, parts, status, eps, size_log, done,
                     run_id);
  return hipGetLastError();
}

}  // namespace hm
