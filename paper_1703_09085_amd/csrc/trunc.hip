// Batched variable-size truncation for gfx950 (FP64).
//
// One workgroup (4 wavefronts of 64 lanes) per work item.  A work item is the
// truncation of a sum of low-rank terms R = sum_p alpha_p A_p B_p^T, which covers
// the truncated addition of Fig. rkadd (two terms: the update and the current
// block) and the stages of rkmerge (Fig. rkmerge: two zero-padded terms).
//
// Algorithm (equal in exact arithmetic to Fig. rkadd, which takes the QR of the
// stacked right factor, forms [alpha A, C] R_B^* and computes its thin SVD):
//   1. gather the stacked factors A_s = [alpha_p A_p] (m x l), B_s = [B_p] (n x l)
//   2. Householder QR of both:  A_s = Q_A R_A,  B_s = Q_B R_B
//   3. core K = R_A R_B^T (q_A x q_B) and its SVD by one-sided Jacobi (FP64)
//   4. rank rule: smallest k with sum_{i>k} s_i^2 <= eps^2 sum_i s_i^2
//   5. C = Q_A U(:, 1:k),  D = Q_B V(:, 1:k) diag(s_1..s_k)
// Both QRs are backward stable, so the singular values agree with the paper's
// order of operations to rounding, and the rank decisions agree except within
// a rounding-sized band around the threshold.
//
// Data ownership inside the workgroup: column c of every tall array belongs to
// wave c % 4 and row r to lane r % 64, so a thread only re-reads global values
// it wrote itself; values produced by other waves are read after a barrier.
#include <hip/hip_runtime.h>

#include "hm_types.h"

namespace hm {

constexpr int TB = 256;
constexpr int NWAVE = TB / 64;

__device__ __forceinline__ int rdim(const DDim& d) {
  int v = d.stat;
  if (d.dyn) {
    int r = *d.dyn;
    v = r < v ? r : v;
  }
  return v < 0 ? 0 : v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Reductions inside aligned groups of g lanes (g a power of two <= 64).
__device__ __forceinline__ double group_sum(double v, int g) {
  for (int off = g >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double group_max(double v, int g) {
  for (int off = g >> 1; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Householder QR of W (rows x cols, ld = rows) in global memory, LAPACK geqr2
// convention: R in the upper triangle, reflector j = I - tau_j v_j v_j^T with
// v_j(j) = 1 implicit and v_j(j+1:) stored below the diagonal.
// vbuf (LDS, >= rows doubles when use_vbuf) caches the current reflector.
// Row r of every column is always touched by lane r % 64 (loops start at the
// 64-aligned row below the diagonal), column c by wave c % 4.
__device__ void house_qr(double* __restrict__ W, int rows, int cols, double* tau, double* vbuf,
                         bool use_vbuf) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int q = rows < cols ? rows : cols;
  for (int j = 0; j < q; ++j) {
    const int base = j & ~63;
    if (wave == (j % NWAVE)) {
      double* x = W + (size_t)j * rows;
      double mx = 0.0;
      for (int r = base + lane; r < rows; r += 64)
        if (r > j) mx = fmax(mx, fabs(x[r]));
      mx = wave_max(mx);
      // scaled by division (a reciprocal of a subnormal maximum overflows)
      double s = 0.0;
      if (mx > 0.0) {
        for (int r = base + lane; r < rows; r += 64)
          if (r > j) {
            const double v = x[r] / mx;
            s += v * v;
          }
      }
      s = wave_sum(s);
      const double xn = mx * sqrt(s);
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
            if (use_vbuf) vbuf[r] = v;
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
      const double* v = W + (size_t)j * rows;
      for (int c = j + 1; c < cols; ++c) {
        if ((c % NWAVE) != wave) continue;
        double* y = W + (size_t)c * rows;
        double p = 0.0;
        for (int r = base + lane; r < rows; r += 64) {
          if (r < j) continue;
          const double vr = (r == j) ? 1.0 : (use_vbuf ? vbuf[r] : v[r]);
          p += vr * y[r];
        }
        const double w = wave_sum(p) * tj;
        for (int r = base + lane; r < rows; r += 64) {
          if (r < j) continue;
          const double vr = (r == j) ? 1.0 : (use_vbuf ? vbuf[r] : v[r]);
          y[r] -= w * vr;
        }
      }
    }
    __syncthreads();
  }
}

// Y (rows x ncol, ldy, global) <- Q Y with Q = H_0 ... H_{q-1} stored in W
// (rows x ., ld = rows) with factors tau.  Same ownership as house_qr.
__device__ void apply_q(const double* __restrict__ W, int rows, int q, const double* tau,
                        double* __restrict__ Y, int ldy, int ncol) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int j = q - 1; j >= 0; --j) {
    const double tj = tau[j];
    if (tj == 0.0) continue;
    const int base = j & ~63;
    const double* v = W + (size_t)j * rows;
    for (int c = wave; c < ncol; c += NWAVE) {
      double* y = Y + (size_t)c * ldy;
      double p = 0.0;
      for (int r = base + lane; r < rows; r += 64)
        if (r >= j) p += ((r == j) ? 1.0 : v[r]) * y[r];
      const double w = wave_sum(p) * tj;
      for (int r = base + lane; r < rows; r += 64)
        if (r >= j) y[r] -= w * ((r == j) ? 1.0 : v[r]);
    }
  }
}

// Column norms of M (p x r, ld p), scaled by the column maximum (division, so
// subnormal columns neither overflow nor underflow).  Wave w handles columns
// w, w + 4, ...; lane 0 writes out[j].
__device__ void col_norms(const double* M, int p, int r, double* out) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int j = wave; j < r; j += NWAVE) {
    const double* col = M + (size_t)j * p;
    double mx = 0.0;
    for (int i = lane; i < p; i += 64) mx = fmax(mx, fabs(col[i]));
    mx = wave_max(mx);
    double s = 0.0;
    if (mx > 0.0)
      for (int i = lane; i < p; i += 64) {
        const double v = col[i] / mx;
        s += v * v;
      }
    s = wave_sum(s);
    if (lane == 0) out[j] = mx * sqrt(s);
  }
}

// One-sided Jacobi on M (p x r, p >= r, column-major, ld = p) with rotations
// accumulated in V (r x r).  Parallel tournament ordering: every round rotates
// r'/2 disjoint column pairs, one group of g lanes per pair.  A pair is left
// alone when its columns are orthogonal to 1e-15 relative, or when the smaller
// column lies below floor (1e-13 of the largest column norm: singular values
// that small are rounding noise of the large ones and cannot be resolved).
__device__ void jacobi(double* M, int p, int r, double* V, int* flag, double floor) {
  const int tid = threadIdx.x;
  for (int i = tid; i < r * r; i += TB) V[i] = ((i % r) == (i / r)) ? 1.0 : 0.0;
  __syncthreads();
  if (r < 2) return;
  const int rr = r + (r & 1);
  const int npairs = rr / 2;
  int g = TB / npairs;
  if (g > 64) g = 64;
  int gp = 1;
  while (gp * 2 <= g) gp *= 2;
  g = gp < 1 ? 1 : gp;
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
        double* ma = M + (size_t)a * p;
        double* mb = M + (size_t)b * p;
        double mx = 0.0;
        for (int i = gl; i < p; i += g) mx = fmax(mx, fmax(fabs(ma[i]), fabs(mb[i])));
        mx = group_max(mx, g);
        if (mx == 0.0) continue;
        double sa = 0, sb = 0, sc = 0;
        for (int i = gl; i < p; i += g) {
          const double x = ma[i] / mx, y = mb[i] / mx;
          sa += x * x;
          sb += y * y;
          sc += x * y;
        }
        sa = group_sum(sa, g);
        sb = group_sum(sb, g);
        sc = group_sum(sc, g);
        if (sc == 0.0 || fabs(sc) <= tol * sqrt(sa) * sqrt(sb)) continue;
        if (fmin(sqrt(sa), sqrt(sb)) * mx <= floor) continue;
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
        double* va = V + (size_t)a * r;
        double* vb = V + (size_t)b * r;
        for (int i = gl; i < r; i += g) {
          const double x = va[i], y = vb[i];
          va[i] = cs * x - sn * y;
          vb[i] = sn * x + cs * y;
        }
        if (gl == 0) *flag = 1;
      }
      __syncthreads();
    }
    const int f = *flag;
    __syncthreads();
    if (!f) break;
  }
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

// Dynamic LDS budget of a truncation workgroup (bytes).  The small arrays, the
// reflector cache and the Jacobi core are placed in LDS when the actual sizes
// fit, in the global workspace otherwise (generic pointers serve both).
constexpr int TRUNC_LDS = 56 * 1024;

__global__ __launch_bounds__(TB) void trunc_kernel(const DTrunc* __restrict__ descs,
                                                   const DTruncPart* __restrict__ parts,
                                                   double* __restrict__ pool, long long pool_doubles,
                                                   unsigned long long* counter, int* status, double eps) {
  extern __shared__ double smem[];
  __shared__ TruncShared sh;
  const DTrunc d = descs[blockIdx.x];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int m = d.m, n = d.n;
  if (tid == 0) {
    int l = 0;
    for (int p = 0; p < d.nparts; ++p) {
      int kp = rdim(parts[d.part0 + p].k);
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
    if (tid == 0) *d.rank = 0;
    return;
  }
  const int qa = m < l ? m : l;
  const int qb = n < l ? n : l;
  const bool tall = qa >= qb;
  const int pp = tall ? qa : qb, rc = tall ? qb : qa;
  // memory plan: small arrays (3 l doubles + l ints), reflector cache
  // (max(m, n)), core (pp rc + rc rc); LDS first, workspace for the rest
  const long long small = 3LL * l + (l + 1) / 2 + 2;
  const long long vneed = m > n ? m : n;
  const long long core = (long long)pp * rc + (long long)rc * rc;
  const long long budget = TRUNC_LDS / 8;
  const bool small_lds = small <= budget;
  const bool core_lds = small_lds && small + core <= budget;
  const bool v_lds = small_lds && small + (core_lds ? core : 0) + vneed <= budget;
  if (tid == 0) {
    long long need = (long long)(m + n) * l + (small_lds ? 0 : small) + (core_lds ? 0 : core);
    need = (need + 31) & ~31LL;
    unsigned long long off = atomicAdd(counter, (unsigned long long)need);
    if ((long long)off + need > pool_doubles) {
      atomicOr(status, ST_WS_OVERFLOW);
      sh.ws = -1;
    } else {
      sh.ws = (long long)off;
    }
  }
  __syncthreads();
  if (sh.ws < 0) return;
  double* WA = pool + sh.ws;
  double* WB = WA + (size_t)m * l;
  double* gnext = WB + (size_t)n * l;
  double* lnext = smem;
  double* smallp;
  if (small_lds) {
    smallp = lnext;
    lnext += small;
  } else {
    smallp = gnext;
    gnext += small;
  }
  double* tauA = smallp;
  double* tauB = tauA + l;
  double* sig = tauB + l;
  int* order = (int*)(sig + l);
  double* M;
  if (core_lds) {
    M = lnext;
    lnext += core;
  } else {
    M = gnext;
    gnext += core;
  }
  double* V = M + (size_t)pp * rc;
  double* vbuf = lnext;

  // 1. gather the stacks (column c by wave c % 4, row r by lane r % 64)
  for (int p = 0; p < d.nparts; ++p) {
    const DTruncPart P = parts[d.part0 + p];
    const int kp = sh.k[p], c0 = sh.coff[p];
    for (int c = 0; c < kp; ++c) {
      const int cc = c0 + c;
      if ((cc % NWAVE) != wave) continue;
      double* a = WA + (size_t)cc * m;
      for (int r = lane; r < m; r += 64) {
        const int rr = r - P.row_off;
        double v = 0.0;
        if (rr >= 0 && rr < P.rows) v = P.alpha * (P.ta ? P.A[c + (size_t)rr * P.lda] : P.A[rr + (size_t)c * P.lda]);
        a[r] = v;
      }
      double* b = WB + (size_t)cc * n;
      for (int r = lane; r < n; r += 64) {
        const int rr = r - P.col_off;
        double v = 0.0;
        if (rr >= 0 && rr < P.cols) v = P.tb ? P.B[c + (size_t)rr * P.ldb] : P.B[rr + (size_t)c * P.ldb];
        b[r] = v;
      }
    }
  }
  __syncthreads();

  // 2. QR of both stacks
  house_qr(WA, m, l, tauA, vbuf, v_lds);
  house_qr(WB, n, l, tauB, vbuf, v_lds);

  // 3. core K = R_A R_B^T (qa x qb), stored in its tall orientation
  for (int e = tid; e < qa * qb; e += TB) {
    const int i = e % qa, j = e / qa;
    const int p0 = i > j ? i : j;
    double s = 0.0;
    for (int pc = p0; pc < l; ++pc) s += WA[i + (size_t)pc * m] * WB[j + (size_t)pc * n];
    if (tall)
      M[i + (size_t)j * pp] = s;
    else
      M[j + (size_t)i * pp] = s;
  }
  __syncthreads();
  col_norms(M, pp, rc, sig);
  __syncthreads();
  if (tid == 0) {
    double fmax_ = 0.0;
    for (int j = 0; j < rc; ++j) fmax_ = fmax(fmax_, sig[j]);
    sh.floor = 1e-13 * fmax_;
  }
  __syncthreads();
  jacobi(M, pp, rc, V, &sh.flag, sh.floor);
  __syncthreads();

  // singular values = column norms of the rotated core
  col_norms(M, pp, rc, sig);
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
  // 4. rank rule on the sorted values: tail[j] = sum_{i >= j} s_i^2 accumulated
  // from the smallest value upwards; k = smallest j with tail[j] <= eps^2 tail[0]
  if (tid == 0) {
    double total = 0.0;
    for (int i = rc - 1; i >= 0; --i) {
      const double s = sig[order[i]];
      total += s * s;
    }
    int k = 0;
    if (total > 0.0) {
      const double thr = eps * eps * total;
      double tail = 0.0;
      k = rc;
      for (int j = rc - 1; j >= 0; --j) {
        const double s = sig[order[j]];
        tail += s * s;
        if (tail <= thr) k = j;
      }
    }
    if (!(total == total) || total > 1.7e308) {
      atomicOr(status, ST_NONFINITE);
      atomicExch(status + 1, (int)blockIdx.x + 1);
    }
    if (k > d.cap) {
      atomicOr(status, ST_RANK_OVERFLOW);
      k = d.cap;
    }
    sh.rank = k;
    atomicAdd((unsigned long long*)(status + 2), 1ULL);
    atomicAdd((unsigned long long*)(status + 4), 8ULL * (unsigned long long)(m + n) * (unsigned long long)(l + k));
  }
  __syncthreads();
  const int k = sh.rank;

  // 5. C = Q_A [U_k; 0], D = Q_B [V_k S_k; 0]
  // tall: U = M columns / s, V = rotations;  wide: U = rotations, V = M columns.
  for (int c = wave; c < k; c += NWAVE) {
    const int j = order[c];
    const double s = sig[j];
    double* cc = d.C + (size_t)c * d.ldc;
    double* dc = d.D + (size_t)c * d.ldd;
    for (int r = lane; r < m; r += 64) {
      double v = 0.0;
      if (r < qa) v = tall ? (s > 0.0 ? M[r + (size_t)j * pp] / s : 0.0) : V[r + (size_t)j * rc];
      cc[r] = v;
    }
    for (int r = lane; r < n; r += 64) {
      double v = 0.0;
      if (r < qb) v = tall ? V[r + (size_t)j * rc] * s : M[r + (size_t)j * pp];
      dc[r] = v;
    }
  }
  __syncthreads();
  apply_q(WA, m, qa, tauA, d.C, d.ldc, k);
  apply_q(WB, n, qb, tauB, d.D, d.ldd, k);
  if (tid == 0) *d.rank = k;
}

hipError_t launch_trunc(const DTrunc* descs, const DTruncPart* parts, int count, double* pool, int64_t pool_doubles,
                        int* counter, int* status, double eps, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(trunc_kernel, dim3(count), dim3(TB), TRUNC_LDS, stream, descs, parts, pool,
                     (long long)pool_doubles, (unsigned long long*)counter, status, eps);
  return hipGetLastError();
}

}  // namespace hm
