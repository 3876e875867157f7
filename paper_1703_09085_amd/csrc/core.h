// Dense-core SVD machinery shared by the truncation kernels (FP64, gfx950).
//
// A "core" is a matrix of at most 64 x 64 held in registers: column c belongs
// to the TPC consecutive threads t with t / TPC == c, and thread t holds rows
// r = t % TPC + TPC s, s = 0 .. 64 / TPC - 1.  Column reductions combine the
// TPC partial sums with DPP (2 or 3 steps), in the same order in every lane,
// so all threads of a column see bit-identical sums.  The block has 64 TPC
// threads (TPC wavefronts).
//
//   core_qrcp      Householder QR of W (nr x nc) with column pivoting,
//                  stopped at the rounding level (or at a given step)
//   core_to_m_piv  M = R^T (nc x qe) through LDS, one column of M per group
//   core_jacobi  one-sided Jacobi on the columns of M (M W = U S)
//   core_order   singular values (column norms) and their descending order
//   rank_rule    relative Frobenius rank rule on the ordered values
#pragma once
#include <hip/hip_runtime.h>

#include "dev_util.h"
#include "hm_types.h"

namespace hm {

constexpr int CMAX = 64;        // largest core dimension
constexpr int CLD = 68;         // leading dimension of the core matrices in LDS
constexpr int CBUF = CMAX * CLD;  // doubles per core buffer

// LDS scratch of the core routines (besides two CBUF buffers and 2 x 64
// doubles for the reflectors).
struct CoreShared {
  double red[8];
  double tau[2];
  double sig[CMAX];
  int order[CMAX];
  int pos_of[CMAX];
  int lastrot;
};

// 1 / sqrt(x) for x in [1, 2]: the hardware estimate and one Newton step
// (error of a few units in the last place)
__device__ __forceinline__ double rsqrt_refined(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x * y;
  const double r = fma(-h, y, 0.5);
  return fma(y, r, y);
}

// 1 / x for a finite normal x whose reciprocal is normal too: the hardware
// estimate and two Newton steps (about one unit in the last place).  Used on
// the scaled cores (largest entry in [1, 2)), where the arguments stay far
// from the ends of the exponent range, to shorten the dependency chain of a
// step; the IEEE division's exact rounding is not needed there.
__device__ __forceinline__ double rcp_refined(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}

// sqrt(x) for a finite normal x > 0 (on the scaled cores, as above): the
// hardware reciprocal square root, two Newton steps on it, then one on the
// root itself (about one unit in the last place)
__device__ __forceinline__ double sqrt_refined(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x * y, y, 1.5);
  y = y * fma(-0.5 * x * y, y, 1.5);
  const double h = x * y;
  return fma(fma(-h, h, x), 0.5 * y, h);
}

template <int TPC>
__device__ __forceinline__ double gsum(double v) {
  static_assert(TPC == 4 || TPC == 8, "4 or 8 threads per column");
  v += dpp<DPP_XOR1>(v);
  v += dpp<DPP_XOR2>(v);
  if (TPC == 8) v += dpp<DPP_HALF_MIRROR>(v);
  return v;
}

// (value, index) of the largest of the 64 values v[0..64) (ties: the lower
// index); every lane of every wave gets the same result.  The values must not
// be NaN.  A DPP maximum, then a ballot of the lanes that hold it.
__device__ __forceinline__ int lds_argmax64(const double* v, double* vmax) {
  const int lane = threadIdx.x & 63;
  const double x = v[lane];
  const double m = wave_max(x);
  const unsigned long long hit = __ballot(x == m);
  *vmax = m;
  return __ffsll((unsigned long long)hit) - 1;
}

// State of a column-pivoted QR carried between calls of core_qrcp.
struct QrcpState {
  int mine = -1;       // this group's pivot step, or -1
  double thr = 0.0;    // stop level: 1e-30 times the largest initial column norm^2
  double total = 0.0;  // |W|_F^2 (the sum of the initial column norms^2)
  double resid = 0.0;  // sum of the remaining column norms^2 where the last call stopped
  bool capped = false; // the last call stopped at jmax, above the stop level
};

// Householder QR of W (nr x nc, both <= 64) with column pivoting, steps
// j0 .. : step j takes the column of largest remaining norm (rows >= j) as
// its pivot.  The factorisation stops once every remaining column is at or
// below 1e-15 of the largest initial column norm (the rest of R is below the
// rounding level of W, at most 8e-15 |W|_F), or at step jmax; a later call
// with j0 = the returned step continues it.  Columns stay with their groups:
// group c holds column c of R = Q^T W (rows <= st.mine of a pivot column, all
// rows < the step count of the others), and st.resid is |W - Q_j R_j|_F^2
// for the first j columns of Q.  cs.sig serves as scratch; vbuf: 2 x 64
// doubles.
template <int TPC>
__device__ __forceinline__ int core_qrcp(double (&w)[CMAX / TPC], int c, int g, int nr, int nc, double* vbuf,
                                         CoreShared& cs, int j0, int jmax, QrcpState& st) {
  constexpr int R = CMAX / TPC;
  const int q = nr < nc ? nr : nc;
  const int lane = threadIdx.x & 63;
  int j = j0;
  for (;; ++j) {
    const int par = j & 1;
    double* vb = vbuf + par * CMAX;
    const bool open = st.mine < 0 && c < nc;
    double n0 = 0.0, n1 = 0.0;
#pragma unroll
    for (int s = 0; s < R; s += 2) {
      const int r = g + TPC * s;
      n0 = r >= j ? fma(w[s], w[s], n0) : n0;
      n1 = r + TPC >= j ? fma(w[s + 1], w[s + 1], n1) : n1;
    }
    const double nn = gsum<TPC>(n0 + n1);
    if (g == 0) cs.sig[c] = open ? nn : -1.0;
    __syncthreads();
    double vmax;
    const int p = lds_argmax64(cs.sig, &vmax);
    if (j == 0) st.thr = 1e-30 * vmax;
    // the same decisions in every thread
    const bool below = !(vmax > st.thr);
    const bool stop = j >= q || j >= jmax || below;
    if (j == 0 || stop) {
      const double sum = wave_sum(fmax(cs.sig[lane], 0.0));  // the same in every wave
      if (j == 0) st.total = sum;
      if (stop) st.resid = sum;
    }
    if (stop) {
      st.capped = !below && j < q;
      break;
    }
    // reflector j from the pivot column (selects rather than branches around
    // the register updates: the compiler then keeps w in place)
    const bool piv = c == p;
    if (__ballot(piv) != 0) {  // only the wave that holds the pivot column
      double s2 = 0.0, s3 = 0.0, al = 0.0;
#pragma unroll
      for (int s = 0; s < R; s += 2) {
        const int r = g + TPC * s;
        s2 = r > j ? fma(w[s], w[s], s2) : s2;
        s3 = r + TPC > j ? fma(w[s + 1], w[s + 1], s3) : s3;
        al = r == j ? w[s] : al;
        al = r + TPC == j ? w[s + 1] : al;
      }
      s2 = gsum<TPC>(s2 + s3);
      al = gsum<TPC>(al);
      const bool nz = s2 > 0.0;
      const double beta = nz ? -copysign(sqrt_refined(fma(al, al, s2)), al) : al;
      const double tv = nz ? (beta - al) * rcp_refined(beta) : 0.0;
      const double inv = nz ? rcp_refined(al - beta) : 0.0;
#pragma unroll
      for (int s = 0; s < R; ++s) {
        const int r = g + TPC * s;
        const double v = r == j ? 1.0 : (r > j ? w[s] * inv : 0.0);
        const double wn = r == j ? beta : (r > j ? v : w[s]);
        w[s] = piv ? wn : w[s];
        if (piv) vb[r] = v;
      }
      if (piv && g == 0) cs.tau[par] = tv;
    }
    st.mine = piv ? j : st.mine;
    __syncthreads();
    // apply it to the other open columns (factor zero elsewhere; a wave
    // without open columns skips it)
    const bool upd = st.mine < 0 && c < nc;
    if (__ballot(upd) != 0) {
      const double tj = cs.tau[par];
      double d0 = 0.0, d1 = 0.0;
#pragma unroll
      for (int s = 0; s < R; s += 2) {
        d0 = fma(vb[g + TPC * s], w[s], d0);
        d1 = fma(vb[g + TPC * (s + 1)], w[s + 1], d1);
      }
      const double dsum = gsum<TPC>(d0 + d1);
      const double f = upd ? tj * dsum : 0.0;
#pragma unroll
      for (int s = 0; s < R; ++s) w[s] = fma(-f, vb[g + TPC * s], w[s]);
    }
  }
  __syncthreads();  // cs.sig is read above and reused by the caller
  return j;
}

// After core_qrcp of W (nr x nc): M = R(0:qe, :)^T (nc x qe) is written to
// buf (column-major, ld CLD; row c of M from group c, so M keeps the row order
// of W's columns) and loaded into x: group a holds column a of M.
template <int TPC>
__device__ __forceinline__ void core_to_m_piv(const double (&w)[CMAX / TPC], double (&x)[CMAX / TPC], int c, int g,
                                              int nc, int qe, int pos, double* __restrict__ buf) {
  constexpr int R = CMAX / TPC;
#pragma unroll
  for (int s = 0; s < R; ++s) {
    const int r = g + TPC * s;
    buf[c + CLD * r] = (r < qe && (pos < 0 || r <= pos) && c < nc) ? w[s] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < R; ++s) x[s] = (c < qe) ? buf[g + TPC * s + CLD * c] : 0.0;
}

// One-sided Jacobi on the q columns of M (group a holds column a in x; buf0
// holds M on entry).  The rounds of a sweep follow the circle method on
// N = q rounded up to even columns: in round r (0 .. N-2) column N-1 pairs
// with column r and every other column a with (2 r - a) mod (N-1), so every
// round is a perfect matching and a sweep visits every pair once; a pair with
// a column >= q (the padding column) is idle.  buf0 / buf1 alternate as the
// source of the partner columns; groups of columns >= q do no work.  A pair
// is not rotated when its columns are orthogonal to 1e-15 relative or when
// the smaller one is below 1e-13 of the largest column norm (rounding noise
// that cannot be resolved further).  Returns the sweeps.
template <int TPC>
__device__ __forceinline__ int core_jacobi(double (&x)[CMAX / TPC], int a, int g, int q, double* buf0,
                                           double* buf1, CoreShared& cs) {
  constexpr int R = CMAX / TPC;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double nn = 0.0;
#pragma unroll
  for (int s = 0; s < R; ++s) nn = fma(x[s], x[s], nn);
  nn = wave_max(gsum<TPC>(nn));
  if (lane == 0) cs.red[wave] = nn;
  if (threadIdx.x == 0) cs.lastrot = -1;
  __syncthreads();
  double cmax = 0.0;
#pragma unroll
  for (int i = 0; i < TPC; ++i) cmax = fmax(cmax, cs.red[i]);
  const double floor2 = 1e-26 * cmax;
  const double tol2 = 1e-30;
  const int N = q + (q & 1), N1 = N - 1;
  const bool active = a < q;
  int round = 0;
  for (int sweep = 0; sweep < 40; ++sweep) {
    for (int r = 0; r < N1; ++r, ++round) {
      const double* cur = (round & 1) ? buf1 : buf0;
      double* nxt = (round & 1) ? buf0 : buf1;
      int b = a == N1 ? r : (a == r ? N1 : 2 * r - a);
      if (b < 0) b += N1;
      else if (b >= N1 && a != r) b -= N1;
      if (active && b < q) {
        double y[R];
#pragma unroll
        for (int s = 0; s < R; ++s) y[s] = cur[g + TPC * s + CLD * b];
        double sxx = 0.0, syy = 0.0, sxy = 0.0;
#pragma unroll
        for (int s = 0; s < R; ++s) {
          sxx = fma(x[s], x[s], sxx);
          syy = fma(y[s], y[s], syy);
          sxy = fma(x[s], y[s], sxy);
        }
        sxx = gsum<TPC>(sxx);
        syy = gsum<TPC>(syy);
        sxy = gsum<TPC>(sxy);
        const bool lower = a < b;
        const double spp = lower ? sxx : syy, sqq = lower ? syy : sxx;
        if (fmin(spp, sqq) > floor2 && sxy * sxy > tol2 * spp * sqq) {
          // tan of the rotation angle, t = sign(d) 2 c / (|d| + sqrt(d^2 + 4 c^2))
          // with d = sqq - spp and c = sxy (the smaller root of t^2 + 2 (d / 2c) t - 1)
          const double dd = sqq - spp;
          const double hyp = sqrt_refined(fma(dd, dd, 4.0 * sxy * sxy));
          const double tt = (dd >= 0.0 ? 2.0 * sxy : -2.0 * sxy) * rcp_refined(fabs(dd) + hyp);
          const double cn = rsqrt_refined(fma(tt, tt, 1.0));
          const double sn = cn * tt;
          if (sn != 0.0) {
            const double ss = lower ? -sn : sn;
#pragma unroll
            for (int s = 0; s < R; ++s) x[s] = fma(ss, y[s], cn * x[s]);
            // rotations this small leave the columns orthogonal to rounding
            // after one more sweep at most (quadratic convergence): they do not
            // keep the iteration going
            if (fabs(sn) > 1e-8) cs.lastrot = sweep;
          }
        }
      }
      if (active) {
#pragma unroll
        for (int s = 0; s < R; ++s) nxt[g + TPC * s + CLD * a] = x[s];
      }
      __syncthreads();
    }
    // every thread reads the same value here: a write of sweep + 1 can only
    // come from a thread that found a rotation in this sweep
    if (cs.lastrot < sweep) return sweep + 1;
  }
  return 40;
}

// Column norms of the final M (group a) and their descending order (ties by
// the lower index; NaN last, so that order is a permutation).
template <int TPC>
__device__ __forceinline__ void core_order(const double (&x)[CMAX / TPC], int a, int g, int q, CoreShared& cs) {
  constexpr int R = CMAX / TPC;
  double nn = 0.0;
#pragma unroll
  for (int s = 0; s < R; ++s) nn = fma(x[s], x[s], nn);
  nn = gsum<TPC>(nn);
  if (g == 0 && a < q) cs.sig[a] = sqrt(nn);
  __syncthreads();
  if (g == 0 && a < q) {
    const double sa = (cs.sig[a] == cs.sig[a]) ? cs.sig[a] : -1.0;
    int pos = 0;
    for (int i = 0; i < q; ++i) {
      const double si = (cs.sig[i] == cs.sig[i]) ? cs.sig[i] : -1.0;
      pos += (si > sa) || (si == sa && i < a);
    }
    cs.order[pos] = a;
    cs.pos_of[a] = pos;
  }
  __syncthreads();
}

// Rank rule (one thread): smallest k with sum_{i>=k} s_i^2 <= eps^2 sum_i s_i^2,
// the tail accumulated from the smallest value upwards; values at or below
// 1e-13 of the largest count as zero.  *nonfinite is set for a NaN or infinite
// sum of squares (k is then 0).
__device__ __forceinline__ int rank_rule(const CoreShared& cs, int q, double eps, bool* nonfinite) {
  double total = 0.0;
  for (int i = q - 1; i >= 0; --i) {
    const double s = cs.sig[cs.order[i]];
    total += s * s;
  }
  *nonfinite = !(total == total) || total > 1.7e308;
  if (*nonfinite || !(total > 0.0)) return 0;
  const double thr = eps * eps * total;
  double tail = 0.0;
  int k = q;
  for (int j = q - 1; j >= 0; --j) {
    const double s = cs.sig[cs.order[j]];
    tail += s * s;
    if (tail <= thr) k = j;
  }
  const double fl = 1e-13 * cs.sig[cs.order[0]];
  int nz = 0;
  while (nz < q && cs.sig[cs.order[nz]] > fl) ++nz;
  return k < nz ? k : nz;
}

}  // namespace hm
