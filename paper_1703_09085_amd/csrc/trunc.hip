// Batched variable-size truncation for gfx950 (FP64).
//
// One workgroup (8 wavefronts of 64 lanes) per work item.  A work item is the
// truncation of a sum of low-rank terms R = sum_p alpha_p A_p B_p^T, which covers
// the truncated addition of Fig. rkadd (two terms: the update and the current
// block) and the stages of rkmerge (Fig. rkmerge: two zero-padded terms).
//
// Algorithm (equal in exact arithmetic to Fig. rkadd, which takes the QR of the
// stacked right factor, forms [alpha A, C] R_B^* and computes its thin SVD):
//   1. gather the stacked factors A_s = [alpha_p A_p] (m x l), B_s = [B_p] (n x l)
//   2. Householder QR of both:  A_s = Q_A R_A,  B_s = Q_B R_B
//   3. core K = R_A R_B^T (q_A x q_B); one-sided Jacobi on its columns gives
//      K V = U S (V itself is never formed)
//   4. rank rule: smallest k with sum_{i>k} s_i^2 <= eps^2 sum_i s_i^2
//   5. C = Q_A [U_k; 0],  D = Q_B [K^T U_k; 0]   (K^T U_k = V_k S_k)
// Both QRs are backward stable, so the singular values agree with the paper's
// order of operations to rounding, and the rank decisions agree except within
// a rounding-sized band around the threshold.
//
// Blocks with l <= 64 whose stacks fit the registers of the workgroup are done
// by the register-resident kernel (trunc_tall.hip), launched first on the same
// items; this kernel skips the items that kernel marked in `done`.
//
// Memory: the stacks, the core and the small vectors live in LDS when their
// actual sizes fit the workgroup's budget, in a global workspace otherwise.
// Ownership inside the workgroup: column c of a tall array belongs to wave
// c % 8 and row r to lane r % 64, so a thread only re-reads global values it
// wrote itself; values produced by other waves are read after a barrier.
#include <hip/hip_runtime.h>

#include "dev_util.h"
#include "hm_types.h"

namespace hm {

constexpr int TB = 512;
constexpr int NWAVE = TB / 64;
// Dynamic LDS of a truncation workgroup (bytes); one workgroup per CU.
constexpr int TRUNC_LDS = 144 * 1024;

// Euclidean norm of x[lo..hi) owned lane-wise (element r by lane r % 64) by one
// wave; all lanes return the same value.
__device__ __forceinline__ double wave_norm(const double* x, int lo, int hi, int lane) {
  const int base = lo & ~63;
  double s = 0.0;
  for (int r = base + lane; r < hi; r += 64)
    if (r >= lo) s += x[r] * x[r];
  s = wave_sum(s);
  if (safe_sq(s)) return sqrt(s);
  double mx = 0.0;
  for (int r = base + lane; r < hi; r += 64)
    if (r >= lo) mx = fmax(mx, fabs(x[r]));
  mx = wave_max(mx);
  if (mx == 0.0 || !(mx <= 1.7e308)) return mx;
  const int e = ilogb(mx);
  double t = 0.0;
  for (int r = base + lane; r < hi; r += 64)
    if (r >= lo) {
      const double v = ldexp(x[r], -e);
      t += v * v;
    }
  t = wave_sum(t);
  return ldexp(sqrt(t), e);
}

// Householder QR of W (rows x cols, leading dimension ldw) in LAPACK geqr2
// convention: R in the upper triangle, reflector j = I - tau_j v_j v_j^T with
// v_j(j) = 1 implicit and v_j(j+1:) stored below the diagonal.  One barrier
// per column: the owner wave of column j builds reflector j while the other
// waves may still apply reflector j - 1 to columns it does not touch.
// vbuf (LDS, 2 x rows) caches the reflector when W is in global memory.
constexpr int CB = 8;  // columns per wave whose reductions are interleaved

template <bool CACHE>
__device__ __forceinline__ void house_qr(double* __restrict__ W, int rows, int cols, int ldw, double* tau,
                                         double* vbuf) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int q = rows < cols ? rows : cols;
  for (int j = 0; j < q; ++j) {
    const int base = j & ~63;
    double* vb = CACHE ? vbuf + (size_t)(j & 1) * rows : nullptr;
    if (wave == (j % NWAVE)) {
      double* x = W + (size_t)j * ldw;
      const double xn = wave_norm(x, j + 1, rows, lane);
      const double xj = (lane == (j & 63)) ? x[j] : 0.0;
      const double alpha = __shfl(xj, j & 63, 64);
      double t = 0.0;
      if (xn > 0.0) {
        const double beta = -copysign(hypot(alpha, xn), alpha);
        t = (beta - alpha) / beta;
        const double den = alpha - beta;
        for (int r = base + lane; r < rows; r += 64) {
          if (r > j) {
            const double v = x[r] / den;
            x[r] = v;
            if (CACHE) vb[r] = v;
          } else if (r == j) {
            x[r] = beta;
          }
        }
      }
      if (lane == 0) tau[j] = t;
    }
    __syncthreads();
    const double tj = tau[j];
    if (tj != 0.0) {
      const double* v = CACHE ? vb : W + (size_t)j * ldw;
      // columns > j owned by this wave, CB at a time: all dot products first,
      // then their (independent) reductions, then the updates
      const int c0 = j + 1 + ((wave - (j + 1) % NWAVE) % NWAVE + NWAVE) % NWAVE;
      for (int cb = c0; cb < cols; cb += CB * NWAVE) {
        double p[CB];
#pragma unroll
        for (int u = 0; u < CB; ++u) p[u] = 0.0;
        for (int r = base + lane; r < rows; r += 64) {
          if (r < j) continue;
          const double vr = (r == j) ? 1.0 : v[r];
#pragma unroll
          for (int u = 0; u < CB; ++u) {
            const int c = cb + u * NWAVE;
            if (c < cols) p[u] += vr * W[r + (size_t)c * ldw];
          }
        }
#pragma unroll
        for (int u = 0; u < CB; ++u) p[u] = wave_sum(p[u]) * tj;
        for (int r = base + lane; r < rows; r += 64) {
          if (r < j) continue;
          const double vr = (r == j) ? 1.0 : v[r];
#pragma unroll
          for (int u = 0; u < CB; ++u) {
            const int c = cb + u * NWAVE;
            if (c < cols) W[r + (size_t)c * ldw] -= p[u] * vr;
          }
        }
      }
    }
  }
  __syncthreads();
}

// Y (rows x ncol, ldy, global) <- Q Y with Q = H_0 ... H_{q-1} stored in W
// (rows x ., ldw) with factors tau.  Column c of Y by wave c % 8.
__device__ __forceinline__ void apply_q(const double* __restrict__ W, int rows, int ldw, int q, const double* tau,
                                        double* __restrict__ Y, int ldy, int ncol) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int j = q - 1; j >= 0; --j) {
    const double tj = tau[j];
    if (tj == 0.0) continue;
    const int base = j & ~63;
    const double* v = W + (size_t)j * ldw;
    for (int cb = wave; cb < ncol; cb += CB * NWAVE) {
      double p[CB];
#pragma unroll
      for (int u = 0; u < CB; ++u) p[u] = 0.0;
      for (int r = base + lane; r < rows; r += 64) {
        if (r < j) continue;
        const double vr = (r == j) ? 1.0 : v[r];
#pragma unroll
        for (int u = 0; u < CB; ++u) {
          const int c = cb + u * NWAVE;
          if (c < ncol) p[u] += vr * Y[r + (size_t)c * ldy];
        }
      }
#pragma unroll
      for (int u = 0; u < CB; ++u) p[u] = wave_sum(p[u]) * tj;
      for (int r = base + lane; r < rows; r += 64) {
        if (r < j) continue;
        const double vr = (r == j) ? 1.0 : v[r];
#pragma unroll
        for (int u = 0; u < CB; ++u) {
          const int c = cb + u * NWAVE;
          if (c < ncol) Y[r + (size_t)c * ldy] -= p[u] * vr;
        }
      }
    }
  }
}

// Column norms of M (p x r, ld ldm); wave w handles columns w, w + 8, ...
__device__ __forceinline__ void col_norms(const double* M, int p, int r, int ldm, double* out) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int j = wave; j < r; j += NWAVE) {
    const double nrm = wave_norm(M + (size_t)j * ldm, 0, p, lane);
    if (lane == 0) out[j] = nrm;
  }
}

// One-sided Jacobi on the columns of M (p x r, ld ldm).  Parallel tournament
// ordering: every round rotates r'/2 disjoint column pairs, one group of g
// lanes per pair.  A pair is left alone when its columns are orthogonal to
// 1e-15 relative, or when the smaller column lies below floor (1e-13 of the
// largest column norm: singular values that small are rounding noise of the
// large ones and cannot be resolved further).
__device__ __forceinline__ int jacobi(double* M, int p, int r, int ldm, int* flag, double floor) {
  const int tid = threadIdx.x;
  if (r < 2) return 0;
  const int rr = r + (r & 1);
  const int npairs = rr / 2;
  int g = TB / npairs;
  if (g > 64) g = 64;
  int gp = 1;
  while (gp * 2 <= g) gp *= 2;
  g = gp;
  const int groups = TB / g;
  const int gl = tid % g;  // lane inside the group
  const double tol = 1e-15;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) *flag = 0;
    __syncthreads();
    for (int t = 0; t < rr - 1; ++t) {
      for (int pi = tid / g; pi < npairs; pi += groups) {
        const int a = (pi == 0) ? 0 : ((pi - 1 + t) % (rr - 1)) + 1;
        const int bpos = rr - 1 - pi;
        const int b = ((bpos - 1 + t) % (rr - 1)) + 1;
        if (a >= r || b >= r) continue;
        double* ma = M + (size_t)a * ldm;
        double* mb = M + (size_t)b * ldm;
        double sa = 0, sb = 0, sc = 0;
        for (int i = gl; i < p; i += g) {
          const double x = ma[i], y = mb[i];
          sa += x * x;
          sb += y * y;
          sc += x * y;
        }
        sa = group_sum(sa, g);
        sb = group_sum(sb, g);
        sc = group_sum(sc, g);
        int e = 0;
        if (!safe_sq(sa) || !safe_sq(sb)) {
          double mx = 0.0;
          for (int i = gl; i < p; i += g) mx = fmax(mx, fmax(fabs(ma[i]), fabs(mb[i])));
          mx = group_max(mx, g);
          if (mx == 0.0) continue;
          e = ilogb(mx);
          sa = sb = sc = 0.0;
          for (int i = gl; i < p; i += g) {
            const double x = ldexp(ma[i], -e), y = ldexp(mb[i], -e);
            sa += x * x;
            sb += y * y;
            sc += x * y;
          }
          sa = group_sum(sa, g);
          sb = group_sum(sb, g);
          sc = group_sum(sc, g);
        }
        if (sc == 0.0 || fabs(sc) <= tol * sqrt(sa) * sqrt(sb)) continue;
        if (ldexp(fmin(sqrt(sa), sqrt(sb)), e) <= floor) continue;
        const double zeta = (sb - sa) / (2.0 * sc);
        const double tt = copysign(1.0, zeta) / (fabs(zeta) + hypot(1.0, zeta));
        const double cs = 1.0 / sqrt(1.0 + tt * tt);
        const double sn = cs * tt;
        if (sn == 0.0) continue;
        for (int i = gl; i < p; i += g) {
          const double x = ma[i], y = mb[i];
          ma[i] = cs * x - sn * y;
          mb[i] = sn * x + cs * y;
        }
        if (gl == 0) *flag = 1;
      }
      __syncthreads();
    }
    const int f = *flag;
    __syncthreads();
    if (!f) return sweep + 1;
  }
  return 40;
}

// Gather of the stacked factors: column c of the A stack (m rows) is
// alpha_p A_p(:, c - c0) placed at rows row_off.., zero elsewhere (likewise B).
__device__ __forceinline__ void gather(const DTrunc& d, const DTruncPart* __restrict__ parts, const int* k,
                                       const int* coff, double* __restrict__ A, double* __restrict__ B) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int p = 0; p < d.nparts; ++p) {
    const DTruncPart P = parts[d.part0 + p];
    const int kp = k[p], c0 = coff[p];
    for (int c = ((wave - c0 % NWAVE) % NWAVE + NWAVE) % NWAVE; c < kp; c += NWAVE) {
      double* a = A + (size_t)(c0 + c) * d.m;
      for (int r = lane; r < d.m; r += 64) {
        const int rr = r - P.row_off;
        double v = 0.0;
        if (rr >= 0 && rr < P.rows) v = P.alpha * (P.ta ? P.A[c + (size_t)rr * P.lda] : P.A[rr + (size_t)c * P.lda]);
        a[r] = v;
      }
      double* b = B + (size_t)(c0 + c) * d.n;
      for (int r = lane; r < d.n; r += 64) {
        const int rr = r - P.col_off;
        double v = 0.0;
        if (rr >= 0 && rr < P.cols) v = P.tb ? P.B[c + (size_t)rr * P.ldb] : P.B[rr + (size_t)c * P.ldb];
        b[r] = v;
      }
    }
  }
}

// Copy a rows x cols block, column c by wave c % 8, row r by lane r % 64.
__device__ __forceinline__ void copy_block(const double* __restrict__ src, double* __restrict__ dst, int rows,
                                           int cols) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int c = wave; c < cols; c += NWAVE)
    for (int r = lane; r < rows; r += 64) dst[r + (size_t)c * rows] = src[r + (size_t)c * rows];
}

struct TruncShared {
  int k[4];
  int coff[4];
  int l;
  int skip;
  int rank;
  int flag;
  long long ws;
  double floor;
};

__global__ __launch_bounds__(TB) void trunc_kernel(const DTrunc* __restrict__ descs,
                                                   const DTruncPart* __restrict__ parts,
                                                   double* __restrict__ pool, long long pool_doubles,
                                                   unsigned long long* counter, int* status, double eps,
                                                   int* size_log, const int* done, int run_id) {
  extern __shared__ double smem[];
  __shared__ TruncShared sh;
  const DTrunc d = descs[blockIdx.x];
  if ((d.flags & TRUNC_CLASS_CHECK) && d.m <= TRUNC_SMALL_MAX && d.n <= TRUNC_SMALL_MAX) return;  // small-block kernel's
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int m = d.m, n = d.n;
  if (tid < 64) {
    const StackCounts sc = stacked_counts(parts, d.part0, d.nparts, sh.k, sh.coff, nullptr);
    if (tid == 0) {
      sh.l = sc.l;
      sh.skip = ((d.flags & TRUNC_SKIP_IF_PART0_EMPTY) && sc.k0 == 0) ||
               ((d.flags & TRUNC_SKIP_IF_HEAD_EMPTY) && sc.l == sc.klast);
    }
  }
  __syncthreads();
  if (sh.skip) return;
  const int l = sh.l;
  if (l == 0) {
    if (tid == 0) *d.rank = 0;
    return;
  }
  if (done && done[blockIdx.x] == run_id) return;  // done by trunc_tall_kernel
  const int qa = m < l ? m : l;
  const int qb = n < l ? n : l;
  const int q = qa < qb ? qa : qb;  // number of singular values of the sum
  const int qm = qa > qb ? qa : qb;
  const int ldk = qm | 1;  // square core buffer, odd leading dimension (fewer LDS bank conflicts)
  // ---- memory plan (doubles) ----
  const long long budget = TRUNC_LDS / 8;
  const long long small = 4LL * l + (l + 1) / 2 + 4;  // tauA, tauB, tauK, sig, order
  const long long core = (long long)ldk * qm;
  const long long stA = (long long)m * l, stB = (long long)n * l;
  const long long vneed = 2LL * (m > n ? m : n);
  const long long t1n = (long long)l * qb;  // R_A^T U_k
  // everything in LDS, or: each stack's QR in LDS (results copied out to the
  // workspace), the core in LDS when it fits, the reflector cache otherwise
  const bool all_lds = small + stA + stB + core <= budget;
  const bool qrA_lds = small + stA <= budget;
  const bool qrB_lds = small + stB <= budget;
  const bool core_lds = small + core <= budget;
  const bool cache_v = small + vneed <= budget;
  if (small > budget) {  // stacked rank beyond any supported size
    if (tid == 0) atomicOr(status, ST_WS_OVERFLOW);
    return;
  }
  if (tid == 0) {
    long long need = (all_lds ? 0 : stA + stB) + (all_lds || core_lds ? 0 : core) + t1n;
    need = (need + 31) & ~31LL;
    const unsigned long long off = atomicAdd(counter, (unsigned long long)need);
    if ((long long)off + need > pool_doubles) {
      atomicOr(status, ST_WS_OVERFLOW);
      sh.ws = -1;
    } else {
      sh.ws = (long long)off;
    }
  }
  __syncthreads();
  if (sh.ws < 0) return;
  double* gws = pool + sh.ws;
  double* tauA = smem;
  double* tauB = tauA + l;
  double* tauK = tauB + l;
  double* sig = tauK + l;
  int* order = (int*)(sig + l);
  double* lfree = smem + small;
  double *WA, *WB, *T1, *M;
  if (all_lds) {
    WA = lfree;
    WB = WA + stA;
    M = WB + stB;
    T1 = gws;
  } else {
    WA = gws;
    WB = WA + stA;
    T1 = WB + stB;
    M = core_lds ? lfree : T1 + t1n;
  }

  const long long clk0 = clock64();
  // 1.-2. gather and QR of both stacks
  gather(d, parts, sh.k, sh.coff, WA, WB);
  __syncthreads();
  if (all_lds) {
    house_qr<false>(lfree, m, l, m, tauA, nullptr);
    house_qr<false>(lfree + stA, n, l, n, tauB, nullptr);
  } else {
    if (qrA_lds) {
      copy_block(WA, lfree, m, l);
      __syncthreads();
      house_qr<false>(lfree, m, l, m, tauA, nullptr);
      copy_block(lfree, WA, m, l);
    } else if (cache_v) {
      house_qr<true>(WA, m, l, m, tauA, lfree);
    } else {
      house_qr<false>(WA, m, l, m, tauA, nullptr);
    }
    __syncthreads();
    if (qrB_lds) {
      copy_block(WB, lfree, n, l);
      __syncthreads();
      house_qr<false>(lfree, n, l, n, tauB, nullptr);
      copy_block(lfree, WB, n, l);
    } else if (cache_v) {
      house_qr<true>(WB, n, l, n, tauB, lfree);
    } else {
      house_qr<false>(WB, n, l, n, tauB, nullptr);
    }
    __syncthreads();
  }

  const long long clk1 = clock64();
  // 3. core: K^T = R_B R_A^T (qb x qa); its QR K^T = Q R gives M = R^T
  //    (qa x q, lower trapezoidal) with the same left singular vectors as K;
  //    one-sided Jacobi on M converges in few sweeps (QR preconditioning)
  for (int e = tid; e < qa * qb; e += TB) {
    const int j = e % qb, i = e / qb;
    const int p0 = i > j ? i : j;
    double s = 0.0;
    for (int pc = p0; pc < l; ++pc) s += WB[j + (size_t)pc * n] * WA[i + (size_t)pc * m];
    M[j + (size_t)i * ldk] = s;
  }
  __syncthreads();
  house_qr<false>(M, qb, qa, ldk, tauK, nullptr);
  // in-place transpose of the triangle: M(i, j) = R(j, i) for j <= i, zero above
  for (int e = tid; e < qa * q; e += TB) {
    const int i = e % qa, j = e / qa;
    if (j < i) {
      M[i + (size_t)j * ldk] = M[j + (size_t)i * ldk];
      M[j + (size_t)i * ldk] = 0.0;
    }
  }
  __syncthreads();
  col_norms(M, qa, q, ldk, sig);
  __syncthreads();
  if (tid == 0) {
    double fm = 0.0;
    for (int j = 0; j < q; ++j) fm = fmax(fm, sig[j]);
    sh.floor = 1e-13 * fm;
  }
  __syncthreads();
  const int sweeps = jacobi(M, qa, q, ldk, &sh.flag, sh.floor);
  __syncthreads();
  const long long clk2 = clock64();
  const int rc = q;
  col_norms(M, qa, rc, ldk, sig);
  __syncthreads();
  // descending order, ties broken by the lower index; a non-finite value ranks
  // last so that `order` is always a permutation
  for (int j = tid; j < rc; j += TB) {
    const double sj = (sig[j] == sig[j]) ? sig[j] : -1.0;
    int pos = 0;
    for (int i = 0; i < rc; ++i) {
      const double si = (sig[i] == sig[i]) ? sig[i] : -1.0;
      pos += (si > sj) || (si == sj && i < j);
    }
    order[pos] = j;
  }
  __syncthreads();
  // 4. rank rule: tail[j] = sum_{i >= j} s_i^2 accumulated from the smallest
  // value upwards; k = smallest j with tail[j] <= eps^2 tail[0]
  if (tid == 0) {
    double total = 0.0;
    for (int i = q - 1; i >= 0; --i) {
      const double s = sig[order[i]];
      total += s * s;
    }
    int k = 0;
    if (total > 0.0) {
      const double thr = eps * eps * total;
      double tail = 0.0;
      k = q;
      for (int j = q - 1; j >= 0; --j) {
        const double s = sig[order[j]];
        tail += s * s;
        if (tail <= thr) k = j;
      }
    }
    // values below 1e-13 of the largest are rounding noise (their columns are
    // not orthogonalised by the Jacobi sweeps) and count as zero
    if (q > 0) {
      const double fl = 1e-13 * sig[order[0]];
      int nz = 0;
      while (nz < q && sig[order[nz]] > fl) ++nz;
      if (k > nz) k = nz;
    }
    if (d.kfix >= 0 && total > 0.0) k = d.kfix < q ? d.kfix : q;
    if (!(total == total) || total > 1.7e308) {
      atomicOr(status, ST_NONFINITE);
      atomicExch(status + 1, (int)blockIdx.x + 1);
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
    atomicAdd((unsigned long long*)(status + 4), 8ULL * (unsigned long long)(m + n) * (unsigned long long)(l + k));
  }
  __syncthreads();
  const int k = sh.rank;

  // 5. U_k = M(:, order) / s (top qa rows of C); T1 = R_A^T U_k (l x k);
  //    D top = R_B T1 = K^T U_k (qb rows); then the reflectors.
  for (int c = wave; c < k; c += NWAVE) {
    const int j = order[c];
    const double s = sig[j];
    double* cc = d.C + (size_t)c * d.ldc;
    for (int r = lane; r < m; r += 64) cc[r] = (r < qa && s > 0.0) ? M[r + (size_t)j * ldk] / s : 0.0;
  }
  for (int e = tid; e < l * k; e += TB) {
    const int p = e % l, c = e / l;
    const int j = order[c];
    const double s = sig[j];
    const int iend = (p + 1 < qa) ? p + 1 : qa;
    double acc = 0.0;
    if (s > 0.0)
      for (int i = 0; i < iend; ++i) acc += WA[i + (size_t)p * m] * (M[i + (size_t)j * ldk] / s);
    T1[p + (size_t)c * l] = acc;
  }
  __syncthreads();
  for (int c = wave; c < k; c += NWAVE) {
    double* dc = d.D + (size_t)c * d.ldd;
    for (int r = lane; r < n; r += 64) {
      double acc = 0.0;
      if (r < qb)
        for (int p = r; p < l; ++p) acc += WB[r + (size_t)p * n] * T1[p + (size_t)c * l];
      dc[r] = acc;
    }
  }
  __syncthreads();
  apply_q(WA, m, m, qa, tauA, d.C, d.ldc, k);
  apply_q(WB, n, n, qb, tauB, d.D, d.ldd, k);
  if (tid == 0) {
    *d.rank = k;
    if (size_log) size_log[8 * (size_t)d.log_idx + 7] = (int)((clock64() - clk2) >> 4);
  }
}

hipError_t launch_trunc(const DTrunc* descs, const DTruncPart* parts, int count, double* pool, int64_t pool_doubles,
                        int* counter, int* status, double eps, int* size_log, const int* done, int run_id,
                        hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(trunc_kernel, dim3(count), dim3(TB), TRUNC_LDS, stream, descs, parts, pool,
                     (long long)pool_doubles, (unsigned long long*)counter, status, eps, size_log, done, run_id);
  return hipGetLastError();
}

}  // namespace hm
