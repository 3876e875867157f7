// Truncation of blocks of at most 32 x 32 by one wavefront (FP64, gfx950).
//
// The same operation as the small-block kernel (the truncated sum of up to
// four factor pairs, Fig. rkadd and the stages of Fig. rkmerge, rank by the
// relative Frobenius rule) and the same steps: K^T = B_s A_s^T, Householder
// QR of K^T with column pivoting stopped at the rounding level, one-sided
// Jacobi on M = R^T, rank rule, C = U_k and D = B_s (A_s^T U_k).  Here one
// wave does all of it for one item, with no workgroup barrier: a column of
// the current matrix belongs to LPC consecutive lanes (LPC = 64 / columns,
// rounded to 2, 4 or 8), each holding the rows r = g + LPC s, so column sums
// are DPP reductions inside the lane group and the pivot column or a Jacobi
// partner column reaches the other lanes through the wave's own part of LDS.
// Each phase picks LPC from its own column count (K^T: m columns; Jacobi:
// the core width; D: the rank), so narrow matrices use more lanes per column.
#pragma once
#include <hip/hip_runtime.h>

#include "core.h"
#include "dev_util.h"
#include "hm_types.h"

namespace hm {

constexpr int TINY_MAX = 32;  // m, n <= 32
constexpr int TSCH = 8;       // stacked columns staged per chunk
constexpr int TSLD = 10;      // staged rows: row-major with this stride (doubles)
constexpr int TMLD = 33;      // column-major M and U_k: leading dimension

// The wave's part of LDS.
struct TinyShared {
  DTruncPart part[4];
  int k[4];
  int coff[4];
  double sig[TINY_MAX];
  int order[TINY_MAX];
  int pos_of[TINY_MAX];
  double sA[TINY_MAX * TSLD];  // staged chunk of A_s (row i, stacked column u)
  double sB[TINY_MAX * TSLD];  // staged chunk of B_s
  double sT[TSCH * TINY_MAX];  // T = A_chunk^T U_k (u + TSCH p)
  double vb[TINY_MAX];         // the pivot column of a QR step
  double buf[TINY_MAX * TMLD];  // M (Jacobi), then U_k
};
constexpr int TINY_LDS = (int)sizeof(TinyShared);
static_assert(TINY_LDS % 16 == 0, "wave regions stay 16-byte aligned");

// Orders the wave's LDS accesses and keeps the compiler from moving them
// across this point; the wave's LDS operations complete in issue order.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// sum over the LPC lanes of a column (the same order in every lane of it)
template <int LPC>
__device__ __forceinline__ double lsum(double v) {
  if (LPC >= 2) v += dpp<DPP_XOR1>(v);
  if (LPC >= 4) v += dpp<DPP_XOR2>(v);
  if (LPC >= 8) v += dpp<DPP_HALF_MIRROR>(v);
  if (LPC >= 16) v += dpp<DPP_MIRROR>(v);
  return v;
}

// Element v (0..7) of this lane's share of stacked columns [c0, c0 + TSCH)
// of A_s (m rows) and B_s (n rows): lanes 0..31 take rows 0..31 of one
// column, lanes 32..63 of the next; zero outside the parts, the sizes and l.
__device__ __forceinline__ double tiny_elem(const TinyShared& sh, int nparts, int m, int n, int l, int c0, int v) {
  const int lane = threadIdx.x & 63;
  const int e = lane + 64 * v;
  const int side = e / (TINY_MAX * TSCH);  // 0: A_s, 1: B_s
  const int rem = e % (TINY_MAX * TSCH);
  const int i = rem % TINY_MAX, u = rem / TINY_MAX;
  return stacked_elem(sh.part, sh.coff, nparts, side, i, side ? n : m, c0 + u, l);
}

constexpr int TPRE = 4;  // chunks whose loads are issued together

// Issue the loads of chunks g0 .. g0 + TPRE - 1 (every load of a group is in
// flight at once: one memory latency per group instead of one per chunk).
__device__ __forceinline__ void tiny_load(const TinyShared& sh, int nparts, int m, int n, int l, int g0,
                                          double (&pre)[TPRE][8]) {
#pragma unroll
  for (int ch = 0; ch < TPRE; ++ch)
#pragma unroll
    for (int v = 0; v < 8; ++v) pre[ch][v] = tiny_elem(sh, nparts, m, n, l, (g0 + ch) * TSCH, v);
}

// Put one loaded chunk into sA / sB (row i, stacked column u).
__device__ __forceinline__ void tiny_put(TinyShared& sh, const double (&x)[8]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const int e = lane + 64 * v;
    const int side = e / (TINY_MAX * TSCH);
    const int rem = e % (TINY_MAX * TSCH);
    const int i = rem % TINY_MAX, u = rem / TINY_MAX;
    (side == 0 ? sh.sA : sh.sB)[i * TSLD + u] = x[v];
  }
}
static_assert(2 * TINY_MAX * TSCH == 8 * 64, "a chunk is eight values per lane");

struct TinyQr {
  int qe = 0;          // core width
  bool finite = true;  // K holds no NaN or infinity
  bool zero = false;   // K == 0
};

template <int LPC>
__device__ __forceinline__ TinyQr tiny_scaled_qr(TinyShared& sh, double (&w)[TINY_MAX / LPC], int m, int n);

// Phases 1-2 with LPC lanes per column of W = K^T (n x m, m <= 64 / LPC):
// form W, scale it by a power of two (max |K| in [1, 2)), factor it with
// column pivoting, and leave M = R(0:qe, :)^T in sh.buf (column-major, ld
// TMLD; rows >= m are not written when m <= 16 and are never read).
template <int LPC>
__device__ __forceinline__ TinyQr tiny_form_and_qr(TinyShared& sh, int nparts, int m, int n, int l) {
  constexpr int RPL = TINY_MAX / LPC;
  const int lane = threadIdx.x & 63;
  const int c = lane / LPC, g = lane % LPC;
  double w[RPL];
#pragma unroll
  for (int s = 0; s < RPL; ++s) w[s] = 0.0;
  for (int g0 = 0; g0 * TSCH < l; g0 += TPRE) {
    double pre[TPRE][8];
    tiny_load(sh, nparts, m, n, l, g0, pre);
#pragma unroll
    for (int ch = 0; ch < TPRE; ++ch) {
      if ((g0 + ch) * TSCH >= l) break;
      tiny_put(sh, pre[ch]);
      wave_sync();
#pragma unroll
      for (int u = 0; u < TSCH; u += 2) {
        const double2 a = *(const double2*)&sh.sA[(c < TINY_MAX ? c : 0) * TSLD + u];
#pragma unroll
        for (int s = 0; s < RPL; ++s) {
          const double2 b = *(const double2*)&sh.sB[(g + LPC * s) * TSLD + u];
          w[s] = fma(a.x, b.x, w[s]);
          w[s] = fma(a.y, b.y, w[s]);
        }
      }
      wave_sync();
    }
  }
  if (c >= m) {
#pragma unroll
    for (int s = 0; s < RPL; ++s) w[s] = 0.0;
  }
  return tiny_scaled_qr<LPC>(sh, w, m, n);
}

// Phase 2 on W (n x m, m <= 64 / LPC) held as above (column c = lane / LPC,
// rows g + LPC s; zero outside n x m): scale it by a power of two (max |K| in
// [1, 2)), factor it with column pivoting and leave M = R(0:qe, :)^T in sh.buf.
template <int LPC>
__device__ __forceinline__ TinyQr tiny_scaled_qr(TinyShared& sh, double (&w)[TINY_MAX / LPC], int m, int n) {
  constexpr int RPL = TINY_MAX / LPC;
  const int lane = threadIdx.x & 63;
  const int c = lane / LPC, g = lane % LPC;
  TinyQr out;
  double amax = 0.0;
#pragma unroll
  for (int s = 0; s < RPL; ++s) amax = fmax(amax, fabs(w[s]));
  amax = wave_max(amax);
  out.finite = amax <= 1.7976931348623157e308;  // false for NaN and inf
  out.zero = amax == 0.0;
  if (!out.finite || out.zero) return out;
  const int ex = ilogb(amax);
#pragma unroll
  for (int s = 0; s < RPL; ++s) w[s] = ldexp(w[s], -ex);

  // Householder QR of W (n x m) with column pivoting, as in the block-wide
  // core: the pivot is the open column of largest remaining norm (ties: the
  // lower column); stop at 1e-15 of the largest initial column norm
  const int q = m < n ? m : n;
  int mine = -1;
  double thr = 0.0;
  int j = 0;
  for (;; ++j) {
    const bool open = mine < 0 && c < m;
    double n0 = 0.0, n1 = 0.0;
#pragma unroll
    for (int s = 0; s < RPL; s += 2) {
      const int r = g + LPC * s;
      n0 = r >= j ? fma(w[s], w[s], n0) : n0;
      n1 = r + LPC >= j ? fma(w[s + 1], w[s + 1], n1) : n1;
    }
    const double nn = lsum<LPC>(n0 + n1);
    const double val = open ? nn : -1.0;
    const double vmax = wave_max(val);
    const unsigned long long hit = __ballot(val == vmax);
    const int p = (__ffsll(hit) - 1) / LPC;
    if (j == 0) thr = 1e-30 * vmax;
    if (!(vmax > thr) || j >= q) break;
    const bool piv = c == p;
    if (piv) {
#pragma unroll
      for (int s = 0; s < RPL; ++s) sh.vb[g + LPC * s] = w[s];
    }
    wave_sync();
    double pv[RPL];
#pragma unroll
    for (int s = 0; s < RPL; ++s) pv[s] = sh.vb[g + LPC * s];
    wave_sync();
    double s2 = 0.0, al = 0.0;
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      const int r = g + LPC * s;
      s2 = r > j ? fma(pv[s], pv[s], s2) : s2;
      al = r == j ? pv[s] : al;
    }
    s2 = lsum<LPC>(s2);
    al = lsum<LPC>(al);
    const bool nz = s2 > 0.0;
    const double beta = nz ? -copysign(sqrt_refined(fma(al, al, s2)), al) : al;
    const double tv = nz ? (beta - al) * rcp_refined(beta) : 0.0;
    const double inv = nz ? rcp_refined(al - beta) : 0.0;
    double v[RPL];
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      const int r = g + LPC * s;
      v[s] = r == j ? 1.0 : (r > j ? pv[s] * inv : 0.0);
    }
    mine = piv ? j : mine;
    const bool upd = mine < 0 && c < m;
    double d0 = 0.0, d1 = 0.0;
#pragma unroll
    for (int s = 0; s < RPL; s += 2) {
      d0 = fma(v[s], w[s], d0);
      d1 = fma(v[s + 1], w[s + 1], d1);
    }
    const double f = upd ? tv * lsum<LPC>(d0 + d1) : 0.0;
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      const int r = g + LPC * s;
      const double wn = fma(-f, v[s], w[s]);
      w[s] = piv ? (r == j ? beta : (r > j ? 0.0 : w[s])) : wn;
    }
  }
  out.qe = j;
  // M(c, r) = R(r, c) for r < qe (a pivot column: rows up to its step)
  if (c < TINY_MAX) {
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      const int r = g + LPC * s;
      sh.buf[c + TMLD * r] = (r < j && (mine < 0 || r <= mine) && c < m) ? w[s] : 0.0;
    }
  }
  wave_sync();
  return out;
}

// Phases 3-4 with LPC lanes per column of M (m x qe, qe <= 64 / LPC): one-sided
// Jacobi in the circle order of the block-wide core, then the singular values,
// their order and U_k (k from the caller's rule, applied through `rank`) in
// sh.buf.  Returns the sweeps; the rank rule runs in between (rank_of).
template <int LPC, typename RankOf>
__device__ __forceinline__ int tiny_jacobi(TinyShared& sh, int m, int qe, RankOf rank_of, int* k_out) {
  constexpr int RPL = TINY_MAX / LPC;
  const int lane = threadIdx.x & 63;
  const int a = lane / LPC, g = lane % LPC;
  const bool active = a < qe;
  double x[RPL];
#pragma unroll
  for (int s = 0; s < RPL; ++s) {
    const int i = g + LPC * s;
    x[s] = (active && i < m) ? sh.buf[i + TMLD * a] : 0.0;
  }
  double nn = 0.0;
#pragma unroll
  for (int s = 0; s < RPL; ++s) nn = fma(x[s], x[s], nn);
  const double cmax = wave_max(lsum<LPC>(nn));
  const double floor2 = 1e-26 * cmax;
  const double tol2 = 1e-30;
  const int N = qe + (qe & 1), N1 = N - 1;
  int sweeps = 40;
  for (int sweep = 0; sweep < 40; ++sweep) {
    bool moved = false;
    for (int r = 0; r < N1; ++r) {
      int b = a == N1 ? r : (a == r ? N1 : 2 * r - a);
      if (b < 0) b += N1;
      else if (b >= N1 && a != r) b -= N1;
      const bool pair = active && b < qe;
      // rows >= m of the buffer may hold another item's values: never read
      double y[RPL];
#pragma unroll
      for (int s = 0; s < RPL; ++s) y[s] = (pair && g + LPC * s < m) ? sh.buf[g + LPC * s + TMLD * b] : 0.0;
      wave_sync();
      if (pair) {
        double sxx = 0.0, syy = 0.0, sxy = 0.0;
#pragma unroll
        for (int s = 0; s < RPL; ++s) {
          sxx = fma(x[s], x[s], sxx);
          syy = fma(y[s], y[s], syy);
          sxy = fma(x[s], y[s], sxy);
        }
        sxx = lsum<LPC>(sxx);
        syy = lsum<LPC>(syy);
        sxy = lsum<LPC>(sxy);
        const bool lower = a < b;
        const double spp = lower ? sxx : syy, sqq = lower ? syy : sxx;
        if (fmin(spp, sqq) > floor2 && sxy * sxy > tol2 * spp * sqq) {
          const double dd = sqq - spp;
          const double hyp = sqrt_refined(fma(dd, dd, 4.0 * sxy * sxy));
          const double tt = (dd >= 0.0 ? 2.0 * sxy : -2.0 * sxy) * rcp_refined(fabs(dd) + hyp);
          const double cn = rsqrt_refined(fma(tt, tt, 1.0));
          const double sn = cn * tt;
          if (sn != 0.0) {
            const double ss = lower ? -sn : sn;
#pragma unroll
            for (int s = 0; s < RPL; ++s) x[s] = fma(ss, y[s], cn * x[s]);
            moved = moved || fabs(sn) > 1e-8;
          }
        }
      }
      if (active) {
#pragma unroll
        for (int s = 0; s < RPL; ++s) sh.buf[g + LPC * s + TMLD * a] = x[s];
      }
      wave_sync();
    }
    if (__ballot(moved) == 0) {
      sweeps = sweep + 1;
      break;
    }
  }
  // singular values (column norms) and their descending order (ties: the
  // lower index; NaN last)
  nn = 0.0;
#pragma unroll
  for (int s = 0; s < RPL; ++s) nn = fma(x[s], x[s], nn);
  nn = lsum<LPC>(nn);
  if (g == 0 && active) sh.sig[a] = sqrt(nn);
  wave_sync();
  if (g == 0 && active) {
    const double sa = (sh.sig[a] == sh.sig[a]) ? sh.sig[a] : -1.0;
    int pos = 0;
    for (int i = 0; i < qe; ++i) {
      const double si = (sh.sig[i] == sh.sig[i]) ? sh.sig[i] : -1.0;
      pos += (si > sa) || (si == sa && i < a);
    }
    sh.order[pos] = a;
    sh.pos_of[a] = pos;
  }
  wave_sync();
  const int k = rank_of();
  *k_out = k;
  // U(:, pos) = M(:, order[pos]) / s into sh.buf (every read of M is done)
  if (active) {
    const int pos = sh.pos_of[a];
    const double sa = sh.sig[a];
    if (pos < k) {
#pragma unroll
      for (int s = 0; s < RPL; ++s) {
        const int i = g + LPC * s;
        sh.buf[i + TMLD * pos] = (i < m && sa > 0.0) ? x[s] / sa : 0.0;
      }
    }
  }
  wave_sync();
  return sweeps;
}

// Phase 5 with LPC lanes per column of D (n x k, k <= 64 / LPC):
// D = B_s (A_s^T U_k) by chunks of TSCH stacked columns, written to d.D.
template <int LPC>
__device__ __forceinline__ void tiny_rebuild(TinyShared& sh, const DTrunc& d, int nparts, int m, int n, int l, int k) {
  constexpr int RPL = TINY_MAX / LPC;
  const int lane = threadIdx.x & 63;
  const int p = lane / LPC, g = lane % LPC;
  double acc[RPL];
#pragma unroll
  for (int s = 0; s < RPL; ++s) acc[s] = 0.0;
  for (int g0 = 0; g0 * TSCH < l; g0 += TPRE) {
    double pre[TPRE][8];
    tiny_load(sh, nparts, m, n, l, g0, pre);
#pragma unroll
    for (int ch = 0; ch < TPRE; ++ch) {
      if ((g0 + ch) * TSCH >= l) break;
      tiny_put(sh, pre[ch]);
      wave_sync();
#pragma unroll
      for (int v = 0; v < TSCH * TINY_MAX / 64; ++v) {
        const int e = lane + 64 * v;
        const int u = e % TSCH, pp = e / TSCH;
        if (pp < k) {
          double t = 0.0;
          for (int i = 0; i < m; ++i) t = fma(sh.sA[i * TSLD + u], sh.buf[i + TMLD * pp], t);
          sh.sT[u + TSCH * pp] = t;
        }
      }
      wave_sync();
      if (p < k) {
#pragma unroll
        for (int u = 0; u < TSCH; u += 2) {
          const double t0 = sh.sT[u + TSCH * p], t1 = sh.sT[u + 1 + TSCH * p];
#pragma unroll
          for (int s = 0; s < RPL; ++s) {
            const double2 b = *(const double2*)&sh.sB[(g + LPC * s) * TSLD + u];
            acc[s] = fma(b.x, t0, acc[s]);
            acc[s] = fma(b.y, t1, acc[s]);
          }
        }
      }
      wave_sync();
    }
  }
  // outputs (every read of the stacks is done: they may alias C and D)
  for (int e = lane; e < m * k; e += 64) {
    const int i = e % m, pp = e / m;
    d.C[i + (size_t)d.ldc * pp] = sh.buf[i + TMLD * pp];
  }
  if (p < k) {
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      const int jrow = g + LPC * s;
      if (jrow < n) d.D[jrow + (size_t)d.ldd * p] = acc[s];
    }
  }
}

// Rank rule on the ordered values in LDS (every lane computes the same):
// smallest k with sum_{i>=k} s_i^2 <= eps^2 sum_i s_i^2, values at or below
// 1e-13 of the largest counting as zero; *bad for a NaN or infinite sum.
__device__ __forceinline__ int tiny_rank_rule(const TinyShared& sh, int q, double eps, bool* bad) {
  double total = 0.0;
  for (int i = q - 1; i >= 0; --i) {
    const double s = sh.sig[sh.order[i]];
    total += s * s;
  }
  *bad = !(total == total) || total > 1.7e308;
  if (*bad || !(total > 0.0)) return 0;
  const double thr = eps * eps * total;
  double tail = 0.0;
  int k = q;
  for (int j = q - 1; j >= 0; --j) {
    const double s = sh.sig[sh.order[j]];
    tail += s * s;
    if (tail <= thr) k = j;
  }
  const double fl = 1e-13 * sh.sig[sh.order[0]];
  int nz = 0;
  while (nz < q && sh.sig[sh.order[nz]] > fl) ++nz;
  return k < nz ? k : nz;
}

// One item (m, n <= 32) by the calling wave; `item` numbers it in the
// launch for the status block.
__device__ __forceinline__ void trunc_tiny_item(const DTrunc& d, const DTruncPart* __restrict__ parts, int* status,
                                                double eps, int* size_log, TinyShared& sh, int item) {
  const int lane = threadIdx.x & 63;
  const StackCounts sc = stacked_counts(parts, d.part0, d.nparts, sh.k, sh.coff, sh.part);
  wave_sync();
  const int l = sc.l;
  const bool skip = ((d.flags & TRUNC_SKIP_IF_PART0_EMPTY) && sc.k0 == 0) ||
                    ((d.flags & TRUNC_SKIP_IF_HEAD_EMPTY) && l == sc.klast);
  if (skip) return;
  if (l == 0) {
    if (lane == 0) *d.rank = 0;
    return;
  }
  const long long clk0 = clock64();
  const int m = d.m, n = d.n;
  TinyQr qr;
  if (m <= 8)
    qr = tiny_form_and_qr<8>(sh, d.nparts, m, n, l);
  else if (m <= 16)
    qr = tiny_form_and_qr<4>(sh, d.nparts, m, n, l);
  else
    qr = tiny_form_and_qr<2>(sh, d.nparts, m, n, l);
  const long long clk1 = clock64();
  const int qe = qr.qe;
  bool bad = !qr.finite;
  auto rank_of = [&]() {
    int k = 0;
    if (qr.finite && !qr.zero) k = tiny_rank_rule(sh, qe, eps, &bad);
    if (d.kfix >= 0 && qr.finite && !qr.zero) k = d.kfix < qe ? d.kfix : qe;
    if (bad) k = 0;
    return k;
  };
  int k = 0, sweeps = 0;
  if (qr.finite && !qr.zero && qe > 0) {
    if (qe <= 8)
      sweeps = tiny_jacobi<8>(sh, m, qe, rank_of, &k);
    else if (qe <= 16)
      sweeps = tiny_jacobi<4>(sh, m, qe, rank_of, &k);
    else
      sweeps = tiny_jacobi<2>(sh, m, qe, rank_of, &k);
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
    const unsigned long long bytes = 8ULL * (unsigned long long)(m + n) * (unsigned long long)(l + k);
    atomicAdd((unsigned long long*)(status + 4), bytes);
    atomicAdd((unsigned long long*)(status + 6), bytes);
  }
  const long long clk3 = clock64();
  if (k > 0) {
    if (k <= 8)
      tiny_rebuild<8>(sh, d, d.nparts, m, n, l, k);
    else if (k <= 16)
      tiny_rebuild<4>(sh, d, d.nparts, m, n, l, k);
    else
      tiny_rebuild<2>(sh, d, d.nparts, m, n, l, k);
  }
  if (lane == 0) {
    *d.rank = k;
    if (size_log) size_log[8 * (size_t)d.log_idx + 7] = (int)((clock64() - clk3) >> 4);
  }
}

}  // namespace hm
