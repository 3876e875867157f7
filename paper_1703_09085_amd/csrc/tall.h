// Register-resident path of the general truncation kernel (FP64, gfx950).
//
// For blocks larger than 64 x 64 whose stacked rank l is at most 64.  Steps
// (Fig. rkadd, arranged as in the general kernel):
//   1. each stack (A_s: m x l, B_s: n x l) is gathered into registers: column
//      c belongs to the G = 512 / L threads t with t / G == c (L the next power
//      of two >= l, at least 8), thread t holds rows t % G + G s (at most 32
//      rows per thread, so a register block holds RB = 32 G rows); Householder
//      QR with one barrier per step; the reflectors go to the workspace, R to
//      LDS.  A stack of more than RB rows is split into P balanced row blocks
//      (TSQR): each block is factored, the P stacked l x l factors are factored
//      once more, and Q = diag(Q_1 .. Q_P) Q_top
//   2. the core K^T = R_B R_A^T (q_B x q_A, both <= 64) goes through the
//      dense-core routines with 8 threads per column: column-pivoted QR
//      stopped at the rounding level, one-sided Jacobi on the revealed
//      columns, rank rule
//   3. U_k and T = R_A^T U_k are formed in LDS
//   4. for k <= TALL_D_DIRECT, D = K^T C = B_s A_s^T Q_A U_k = B_s T, one pass
//      over the B stack (A_s^T Q_A = R_A^T; Q_B is not needed)
//   5. C = Q_A [U_k; 0], and for larger k D = Q_B [R_B T; 0]: the reflectors
//      are staged through LDS one at a time and applied to the columns held
//      in registers
#pragma once
#include <hip/hip_runtime.h>

#include "core.h"
#include "dev_util.h"
#include "hm_types.h"

namespace hm {

constexpr int TALL_TB = 512;
constexpr int TALL_VB = 2048;                 // rows of a staged reflector (largest m, n)
// ranks up to which D is formed in one pass over the B stack (D = B_s R_A^T U_k);
// above it D = Q_B [R_B R_A^T U_k; 0], which rereads no stack row per column
// chunk
constexpr int TALL_D_DIRECT = 16;
constexpr int TALL_RLD = 64;                  // leading dimension of R_A, R_B, U_k, K^T U_k
constexpr int TALL_CORE = 2 * CBUF + 2 * CMAX;  // core buffers + core reflector pair
// LDS layout (doubles): [0, TALL_CORE) core buffers, overlaid by two staged
// reflectors (2 x TALL_VB <= TALL_CORE); then R_A, R_B (64 x 64 each) and
// three tau vectors (A, B, a row block of the TSQR).
constexpr int TALL_RA = TALL_CORE;
constexpr int TALL_RB = TALL_RA + CMAX * TALL_RLD;
constexpr int TALL_TAU = TALL_RB + CMAX * TALL_RLD;
constexpr int TALL_LDS_DOUBLES = TALL_TAU + 3 * CMAX;
static_assert(2 * TALL_VB <= TALL_CORE, "staged reflectors overlay the core buffers");

__device__ __forceinline__ int pow2_at_least(int v, int lo) {
  int p = lo;
  while (p < v) p *= 2;
  return p;
}

// rows per thread that a column-group layout needs for nr rows and a width of
// wcols columns (0 when more than 32: 32 rows already take about 250 VGPRs,
// the most that two wavefronts per SIMD allow)
__device__ __forceinline__ int tall_rpt(int nr, int wcols) {
  const int G = TALL_TB / wcols;
  const int need = (nr + G - 1) / G;
  return need <= 8 ? 8 : need <= 16 ? 16 : need <= 32 ? 32 : 0;
}

// rows of one register block for stacked rank l
__device__ __forceinline__ int tall_block_rows(int l) { return 32 * (TALL_TB / pow2_at_least(l, 8)); }

// number of row blocks of a stack with nr rows (1: no TSQR)
__device__ __forceinline__ int tall_blocks(int nr, int l) {
  const int RB = tall_block_rows(l);
  return (nr + RB - 1) / RB;
}

// every stack is one register block, or P blocks whose P stacked l x l
// factors form one register block again
__device__ __forceinline__ bool tall_fits(int m, int n, int l) {
  if (l > CMAX) return false;
  const int RB = tall_block_rows(l);
  const int pa = tall_blocks(m, l), pb = tall_blocks(n, l);
  return (pa == 1 || pa * l <= RB) && (pb == 1 || pb * l <= RB);
}

// workspace doubles of one item: the factored stacks, the factored stacks of
// the R factors of the blocks, the intermediate Q_top [S; 0] and the taus of
// the blocks (each TSQR part is at most 32 * 512 = 16384 doubles)
__device__ __forceinline__ long long tall_ws_need(int m, int n, int l) {
  const int pa = tall_blocks(m, l), pb = tall_blocks(n, l);
  long long need = (long long)(m + n) * l;
  if (pa > 1 || pb > 1) need += 3LL * 16384 + 64LL * (pa + pb);
  return (need + 31) & ~31LL;
}

struct TallShared {
  DTruncPart part[4];
  int k[4];
  int coff[4];
  int rank;
  double tau2[2][2];  // concurrent stack QR: current and next tau of each side
  CoreShared core;
};

// Householder reflector of the pivot column j held by the calling group of G
// threads (rows g + G s): v to vb (all RPT * G rows), tau to *tau and taus[j].
template <int RPT>
__device__ __forceinline__ void tall_pivot(double (&w)[RPT], int j, int g, int G, double* __restrict__ vb,
                                           double* tau, double* taus) {
  double s2 = 0.0, al = 0.0;
#pragma unroll
  for (int s = 0; s < RPT; ++s) {
    const int r = g + G * s;
    if (r > j) s2 = fma(w[s], w[s], s2);
    if (r == j) al = w[s];
  }
  s2 = group_sum(s2, G);
  al = group_sum(al, G);
  double beta = al, t = 0.0, inv = 0.0;
  if (s2 > 0.0) {
    beta = -copysign(sqrt(fma(al, al, s2)), al);
    t = (beta - al) / beta;
    inv = 1.0 / (al - beta);
  }
#pragma unroll
  for (int s = 0; s < RPT; ++s) {
    const int r = g + G * s;
    double v = 0.0;
    if (r == j) {
      v = 1.0;
      w[s] = beta;
    } else if (r > j) {
      v = w[s] * inv;
      w[s] = v;
    }
    vb[r] = v;
  }
  if (g == 0) {
    *tau = t;
    taus[j] = t;
  }
}

// Step j of the Householder QR of a register-resident stack: every group
// applies reflector j (vb, tau tj) with a factor that is zero for the columns
// it must not change (c <= j, c >= l, j >= q), and the group of column j + 1
// then builds reflector j + 1 (to vbn, *taun and taus[j + 1]).  The register
// updates are selects rather than branches, so that the compiler keeps w in
// place instead of copying it at every join.
template <int RPT>
__device__ __forceinline__ void tall_step(double (&w)[RPT], int c, int g, int G, int j, int q, int l,
                                          const double* __restrict__ vb, double tj, double* __restrict__ vbn,
                                          double* taun, double* taus) {
  // a wave whose columns are all finished (c <= j) or padding (c >= l)
  // skips the update (the condition is the same in the whole wave)
  const bool upd = j < q && c > j && c < l;
  if (__ballot(upd) != 0) {
    double d0 = 0.0, d1 = 0.0;
#pragma unroll
    for (int s = 0; s < RPT; s += 2) {
      d0 = fma(vb[g + G * s], w[s], d0);
      d1 = fma(vb[g + G * (s + 1)], w[s + 1], d1);
    }
    const double dsum = group_sum(d0 + d1, G);
    const double f = upd ? tj * dsum : 0.0;
#pragma unroll
    for (int s = 0; s < RPT; ++s) w[s] = fma(-f, vb[g + G * s], w[s]);
  }
  const int jn = j + 1;
  const bool piv = c == jn && jn < q;
  if (__ballot(piv) == 0) return;  // only the wave that holds column j + 1 goes on
  double s2 = 0.0, al = 0.0;
#pragma unroll
  for (int s = 0; s < RPT; ++s) {
    const int r = g + G * s;
    s2 = r > jn ? fma(w[s], w[s], s2) : s2;
    al = r == jn ? w[s] : al;
  }
  s2 = group_sum(s2, G);
  al = group_sum(al, G);
  const bool nz = s2 > 0.0;
  // the stacks are not scaled: IEEE square root and divisions
  const double beta = nz ? -copysign(sqrt(fma(al, al, s2)), al) : al;
  const double t = nz ? (beta - al) / beta : 0.0;
  const double inv = nz ? 1.0 / (al - beta) : 0.0;
#pragma unroll
  for (int s = 0; s < RPT; ++s) {
    const int r = g + G * s;
    const double v = r == jn ? 1.0 : (r > jn ? w[s] * inv : 0.0);
    const double wn = r == jn ? beta : (r > jn ? v : w[s]);
    w[s] = piv ? wn : w[s];
    if (piv) vbn[r] = v;
  }
  if (piv && g == 0) {
    *taun = t;
    taus[jn] = t;
  }
}

// Gather rows [row0, row0 + nr) of stack side (0: A_s = [alpha_p A_p], 1:
// B_s = [B_p]), or of the plain column-major matrix src (ld lds) when src is
// given; QR them; store the factored block (R above, reflectors below the
// diagonal) to ws (nr x l, ld nr; not when ws is null) and its R factor to R
// (ld ldr): all rows r < rrows, zero below the diagonal and below row
// min(nr, l).
template <int RPT>
__device__ __forceinline__ void tall_stack(const TallShared& sh, int nparts, int side, const double* src, int lds,
                                           int row0, int nr, int l, double* __restrict__ ws, double* R, int ldr,
                                           int rrows, double* __restrict__ taus, double* vbig, CoreShared& cs) {
  const int t = threadIdx.x;
  const int L = pow2_at_least(l, 8);
  const int G = TALL_TB / L;
  const int c = t / G, g = t % G;
  double w[RPT];
  int p = 0;
  if (c < l)
    while (p + 1 < nparts && c >= sh.coff[p + 1]) ++p;
  const DTruncPart& P = sh.part[p];
  const int cc = c - sh.coff[p];
  // the column's source, row r at col[r * rs] for lo <= r < hi; with few rows
  // per thread the loads are branch-free (all in flight together; more would
  // not fit the registers)
  const double* col;
  size_t rs;
  int lo, hi;
  double alpha = 1.0;
  if (src) {
    col = src + (size_t)lds * c;
    rs = 1;
    lo = 0;
    hi = nr;
  } else {
    const double* base = side ? P.B : P.A;
    const int ld = side ? P.ldb : P.lda, roff = side ? P.col_off : P.row_off, prows = side ? P.cols : P.rows;
    const bool tr = side ? P.tb != 0 : P.ta != 0;
    rs = tr ? (size_t)ld : 1;
    lo = roff - row0;
    hi = lo + prows;
    col = base + (tr ? (size_t)cc : (size_t)cc * ld);
    alpha = side ? 1.0 : P.alpha;
  }
  if (hi > nr) hi = nr;
  if (c >= l) hi = lo;
  if constexpr (RPT <= 8) {
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      const int r = g + G * s;
      w[s] = load_or_zero(col + (ptrdiff_t)(r - lo) * (ptrdiff_t)rs, r >= lo && r < hi, alpha);
    }
  } else {
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      const int r = g + G * s;
      w[s] = (r >= lo && r < hi) ? alpha * col[(ptrdiff_t)(r - lo) * (ptrdiff_t)rs] : 0.0;
    }
  }
  __syncthreads();  // src may be ws itself (in-place factorisation of the top stack)
  const int q = nr < l ? nr : l;
  if (c == 0) tall_pivot<RPT>(w, 0, g, G, vbig, &cs.tau[0], taus);
  __syncthreads();
  for (int j = 0; j < q; ++j) {
    const int par = j & 1;
    tall_step<RPT>(w, c, g, G, j, q, l, vbig + par * TALL_VB, cs.tau[par], vbig + (par ^ 1) * TALL_VB,
                   &cs.tau[par ^ 1], taus);
    __syncthreads();
  }
  if (c < l) {
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      const int r = g + G * s;
      if (ws && r < nr) ws[r + (size_t)nr * c] = w[s];
      if (r < rrows) R[r + (size_t)ldr * c] = (r <= c && r < q) ? w[s] : 0.0;
    }
  }
  __syncthreads();
}

// out (nr x ncols, ld ldo, global) <- Q [S; 0] with Q = H_0 ... H_{q-1} stored
// in ws (nr x l, reflector j below row j, its unit diagonal implicit) and S
// (qsrc x ncols, ld lds, LDS or global).  Columns are processed in chunks of
// width CW held in registers: group c (G = TALL_TB / CW threads) holds column
// c0 + c, rows g + G s.  The reflectors go through LDS (stage: TALL_CORE
// doubles) a few at a time, the last ones first, each zero-padded to RPT G
// rows.  Every group owns its column, so a staged chunk is applied without
// barriers.
template <int RPT>
__device__ __forceinline__ void tall_apply(const double* __restrict__ ws, int nr, int q, const double* __restrict__ taus,
                                           const double* S, int lds, int qsrc, int ncols, double* __restrict__ out,
                                           int ldo, int CW, double* stage) {
  const int t = threadIdx.x;
  const int G = TALL_TB / CW;
  const int c = t / G, g = t % G;
  const int rp = RPT * G;         // rows of a staged reflector (>= nr)
  const int CH = TALL_CORE / rp;  // reflectors per staged chunk (>= 4)
  for (int c0 = 0; c0 < ncols; c0 += CW) {
    const int col = c0 + c;
    const bool live = col < ncols;  // the same in the whole group
    double x[RPT];
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      const int r = g + G * s;
      x[s] = (live && r < qsrc) ? S[r + (size_t)lds * col] : 0.0;
    }
    for (int jhi = q; jhi > 0; jhi -= CH) {
      const int jlo = jhi > CH ? jhi - CH : 0;
      __syncthreads();  // every group is done with the previous chunk
      for (int e = t; e < (jhi - jlo) * rp; e += TALL_TB) {
        const int jj = e / rp, r = e - jj * rp, j = jlo + jj;
        stage[e] = (r < j || r >= nr) ? 0.0 : (r == j ? 1.0 : ws[r + (size_t)nr * j]);
      }
      __syncthreads();
      if (live) {
        for (int j = jhi - 1; j >= jlo; --j) {
          const double* vb = stage + (j - jlo) * rp;
          double d0 = 0.0, d1 = 0.0;
#pragma unroll
          for (int s = 0; s < RPT; s += 2) {
            d0 = fma(vb[g + G * s], x[s], d0);
            d1 = fma(vb[g + G * (s + 1)], x[s + 1], d1);
          }
          const double f = taus[j] * group_sum(d0 + d1, G);
#pragma unroll
          for (int s = 0; s < RPT; ++s) x[s] = fma(-f, vb[g + G * s], x[s]);
        }
      }
    }
    __syncthreads();  // S may overlap out; every thread has read it
    if (live) {
#pragma unroll
      for (int s = 0; s < RPT; ++s) {
        const int r = g + G * s;
        if (r < nr) out[r + (size_t)ldo * col] = x[s];
      }
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void tall_stack_any(const TallShared& sh, int nparts, int side, const double* src, int lds,
                                               int row0, int nr, int l, double* ws, double* R, int ldr, int rrows,
                                               double* taus, double* vbig, CoreShared& cs) {
  switch (tall_rpt(nr, pow2_at_least(l, 8))) {
    case 8: tall_stack<8>(sh, nparts, side, src, lds, row0, nr, l, ws, R, ldr, rrows, taus, vbig, cs); break;
    case 16: tall_stack<16>(sh, nparts, side, src, lds, row0, nr, l, ws, R, ldr, rrows, taus, vbig, cs); break;
    default: tall_stack<32>(sh, nparts, side, src, lds, row0, nr, l, ws, R, ldr, rrows, taus, vbig, cs); break;
  }
}

__device__ __forceinline__ void tall_apply_any(const double* ws, int nr, int q, const double* taus, const double* S,
                                               int lds, int qsrc, int ncols, double* out, int ldo, double* vbig) {
  // column chunk: 32 wide (16 threads per column, reductions by DPP within
  // a row of lanes) unless more columns are asked for, narrower when the rows
  // do not fit 32 per thread
  int CW = ncols <= 32 ? 32 : 64;
  while (CW > 8 && tall_rpt(nr, CW) == 0) CW /= 2;
  switch (tall_rpt(nr, CW)) {
    case 8: tall_apply<8>(ws, nr, q, taus, S, lds, qsrc, ncols, out, ldo, CW, vbig); break;
    case 16: tall_apply<16>(ws, nr, q, taus, S, lds, qsrc, ncols, out, ldo, CW, vbig); break;
    default: tall_apply<32>(ws, nr, q, taus, S, lds, qsrc, ncols, out, ldo, CW, vbig); break;
  }
}

// Rows per thread when each stack side gets half the work-group (G = 256 / L
// threads per column, L the next power of two >= l): 8, 16 or 32, or 0 when
// the taller side does not fit one register block.
__device__ __forceinline__ int tall_rpt2(int m, int n, int l) {
  const int G = (TALL_TB / 2) / pow2_at_least(l, 8);
  const int nr = m > n ? m : n;
  const int need = (nr + G - 1) / G;
  return need <= 8 ? 8 : need <= 16 ? 16 : need <= 32 ? 32 : 0;
}

// Both stacks factored at once: threads [0, 256) take A_s, [256, 512) take
// B_s, each side as in tall_stack with G = 256 / L threads per column and one
// register block, sharing the barriers (the side with fewer steps idles).
// Each side's factored stack goes to its workspace (nr x l, ld nr; not kept
// when the workspace pointer is null), its R to
// RA / RB (ld TALL_RLD, 64 rows) and its taus to tauA / tauB; the reflector
// buffers are TALL_VB / 2 doubles per side and parity.
template <int RPT>
__device__ __forceinline__ void tall_stack2(TallShared& sh, int nparts, int m, int n, int l, double* __restrict__ wsA,
                                            double* __restrict__ wsB, double* RA, double* RB, double* tauA,
                                            double* tauB, double* vbig) {
  constexpr int HALF = TALL_TB / 2, VBH = TALL_VB / 2;
  const int t = threadIdx.x;
  const int side = t / HALF, tt = t % HALF;
  const int L = pow2_at_least(l, 8);
  const int G = HALF / L;
  const int c = tt / G, g = tt % G;
  const int nr = side ? n : m;
  double* const ws = side ? wsB : wsA;
  double* const R = side ? RB : RA;
  double* const taus = side ? tauB : tauA;
  double* const vbs = vbig + side * 2 * VBH;
  double w[RPT];
  int p = 0;
  if (c < l)
    while (p + 1 < nparts && c >= sh.coff[p + 1]) ++p;
  const DTruncPart& P = sh.part[p];
  const int cc = c - sh.coff[p];
  // the column's source, row r at col[(r - lo) * rs] for lo <= r < hi; with
  // few rows per thread the loads are branch-free (all in flight together)
  const double* col = side ? P.B : P.A;
  const int ld = side ? P.ldb : P.lda, lo = side ? P.col_off : P.row_off;
  const bool tr = side ? P.tb != 0 : P.ta != 0;
  const size_t rs = tr ? (size_t)ld : 1;
  col += tr ? (size_t)cc : (size_t)cc * ld;
  int hi = lo + (side ? P.cols : P.rows);
  if (hi > nr) hi = nr;
  if (c >= l) hi = lo;
  const double alpha = side ? 1.0 : P.alpha;
  if constexpr (RPT <= 8) {
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      const int r = g + G * s;
      w[s] = load_or_zero(col + (ptrdiff_t)(r - lo) * (ptrdiff_t)rs, r >= lo && r < hi, alpha);
    }
  } else {
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      const int r = g + G * s;
      w[s] = (r >= lo && r < hi) ? alpha * col[(ptrdiff_t)(r - lo) * (ptrdiff_t)rs] : 0.0;
    }
  }
  __syncthreads();
  const int q = nr < l ? nr : l;
  const int qa = m < l ? m : l, qb = n < l ? n : l;
  const int qmax = qa > qb ? qa : qb;
  if (c == 0 && q > 0) tall_pivot<RPT>(w, 0, g, G, vbs, &sh.tau2[side][0], taus);
  __syncthreads();
  for (int j = 0; j < qmax; ++j) {
    const int par = j & 1;
    tall_step<RPT>(w, c, g, G, j, q, l, vbs + par * VBH, sh.tau2[side][par], vbs + (par ^ 1) * VBH,
                   &sh.tau2[side][par ^ 1], taus);
    __syncthreads();
  }
  if (c < l) {
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      const int r = g + G * s;
      if (ws && r < nr) ws[r + (size_t)nr * c] = w[s];
      if (r < CMAX) R[r + (size_t)TALL_RLD * c] = (r <= c && r < q) ? w[s] : 0.0;
    }
  }
  __syncthreads();
}

// Workspace of one stack side: the factored row blocks (nr x l), and with P > 1
// blocks the stacked block factors (P l x l, factored in place) and the taus
// of the blocks (64 each).
struct TallSide {
  int nr, P;
  double* blocks;
  double* top;
  double* taus;
};

__device__ __forceinline__ int tall_block_start(int nr, int P, int i) { return (int)(((long long)nr * i) / P); }

// QR of one stack side (TSQR when it has several row blocks): R of the whole
// stack to R (LDS, ld TALL_RLD), its taus to tau (LDS); the reflectors stay in
// the workspace when keep is set (Q is applied later).
__device__ __forceinline__ void tall_side_qr(const TallShared& sh, int nparts, int side, const TallSide& S, int l,
                                             double* R, double* tau, double* tau_tmp, double* vbig, CoreShared& cs,
                                             bool keep) {
  if (S.P == 1) {
    tall_stack_any(sh, nparts, side, nullptr, 0, 0, S.nr, l, keep ? S.blocks : nullptr, R, TALL_RLD, CMAX, tau, vbig,
                   cs);
    return;
  }
  const int ldt = S.P * l;
  for (int i = 0; i < S.P; ++i) {
    const int r0 = tall_block_start(S.nr, S.P, i), r1 = tall_block_start(S.nr, S.P, i + 1);
    tall_stack_any(sh, nparts, side, nullptr, 0, r0, r1 - r0, l, keep ? S.blocks + (size_t)r0 * l : nullptr,
                   S.top + (size_t)i * l, ldt, l, tau_tmp, vbig, cs);
    if (threadIdx.x < l) S.taus[64 * i + threadIdx.x] = tau_tmp[threadIdx.x];
  }
  __syncthreads();
  tall_stack_any(sh, nparts, side, S.top, ldt, 0, ldt, l, keep ? S.top : nullptr, R, TALL_RLD, CMAX, tau, vbig, cs);
}

// out (nr x ncols) <- Q [Ssrc; 0] for the Q of one stack side (TSQR: Q_top
// first into the intermediate Y, then each block's Q).
__device__ __forceinline__ void tall_side_apply(const TallSide& S, int l, const double* tau, double* tau_tmp,
                                                const double* src, int qsrc, int ncols, double* out, int ldo, double* Y,
                                                double* vbig) {
  if (S.P == 1) {
    tall_apply_any(S.blocks, S.nr, S.nr < l ? S.nr : l, tau, src, TALL_RLD, qsrc, ncols, out, ldo, vbig);
    return;
  }
  const int ldt = S.P * l;
  tall_apply_any(S.top, ldt, l, tau, src, TALL_RLD, qsrc, ncols, Y, ldt, vbig);
  for (int i = 0; i < S.P; ++i) {
    const int r0 = tall_block_start(S.nr, S.P, i), r1 = tall_block_start(S.nr, S.P, i + 1);
    if (threadIdx.x < l) tau_tmp[threadIdx.x] = S.taus[64 * i + threadIdx.x];
    __syncthreads();
    tall_apply_any(S.blocks + (size_t)r0 * l, r1 - r0, l, tau_tmp, Y + (size_t)i * l, ldt, l, ncols, out + r0, ldo,
                   vbig);
  }
}

// D = B_s T (n x k) into out (ld n), T (l x k) in LDS with ld TALL_RLD: each
// thread takes rows t, t + TALL_TB, ..., eight output and eight stacked
// columns at a time (the loads of eight stacked columns in flight together).
__device__ __forceinline__ void tall_d_from_stack(const TallShared& sh, int nparts, int n, int l, int k,
                                                  const double* T, double* __restrict__ out) {
  for (int j = threadIdx.x; j < n; j += TALL_TB) {
    for (int c0 = 0; c0 < k; c0 += 8) {
      double acc[8];
#pragma unroll
      for (int cc = 0; cc < 8; ++cc) acc[cc] = 0.0;
      for (int p0 = 0; p0 < l; p0 += 8) {
        double b[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) b[u] = stacked_elem(sh.part, sh.coff, nparts, 1, j, n, p0 + u, l);
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int cc = 0; cc < 8; ++cc) {
            const bool in = p0 + u < l && c0 + cc < k;
            const double tv = T[in ? (p0 + u) + TALL_RLD * (c0 + cc) : 0];
            acc[cc] = fma(b[u], in ? tv : 0.0, acc[cc]);
          }
      }
#pragma unroll
      for (int cc = 0; cc < 8; ++cc)
        if (c0 + cc < k) out[j + (size_t)n * (c0 + cc)] = acc[cc];
    }
  }
}

// The whole truncation of one item on the register-resident path.  ws:
// tall_ws_need(m, n, l) doubles of workspace; smem: TALL_LDS_DOUBLES doubles
// of LDS.
__device__ __forceinline__ void tall_path(const DTrunc& d, TallShared& sh, int nparts, int l, double* __restrict__ ws,
                                          double* smem, int* status, double eps, int* size_log) {
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int m = d.m, n = d.n;
  double* const vbig = smem;
  double* const buf0 = smem;
  double* const buf1 = smem + CBUF;
  double* const cvb = smem + 2 * CBUF;
  double* const RA = smem + TALL_RA;
  double* const RB = smem + TALL_RB;
  double* const tauA = smem + TALL_TAU;
  double* const tauB = tauA + CMAX;
  double* const tau_tmp = tauB + CMAX;
  CoreShared& cs = sh.core;
  const int qa = m < l ? m : l, qb = n < l ? n : l;
  const int q = qa < qb ? qa : qb;
  TallSide SA, SB;
  SA.nr = m;
  SA.P = tall_blocks(m, l);
  SB.nr = n;
  SB.P = tall_blocks(n, l);
  SA.blocks = ws;
  SB.blocks = ws + (size_t)m * l;
  double* extra = ws + (size_t)(m + n) * l;  // TSQR parts, 16384 doubles each
  SA.top = extra;
  SB.top = extra + 16384;
  double* const Y = extra + 2 * 16384;
  SA.taus = extra + 3 * 16384;
  SB.taus = SA.taus + 64 * SA.P;
  const long long clk0 = clock64();

  // 1. both stacks
  // both stacks at once when each fits one register block of half the
  // work-group, else one after the other (with TSQR for tall stacks); the
  // reflectors of B_s are kept only when D may need them (rank above
  // TALL_D_DIRECT, so l above it)
  const bool keepB = l > TALL_D_DIRECT;
  double* const wsB = keepB ? SB.blocks : nullptr;
  switch (SA.P == 1 && SB.P == 1 ? tall_rpt2(m, n, l) : 0) {
    case 8: tall_stack2<8>(sh, nparts, m, n, l, SA.blocks, wsB, RA, RB, tauA, tauB, vbig); break;
    case 16: tall_stack2<16>(sh, nparts, m, n, l, SA.blocks, wsB, RA, RB, tauA, tauB, vbig); break;
    case 32: tall_stack2<32>(sh, nparts, m, n, l, SA.blocks, wsB, RA, RB, tauA, tauB, vbig); break;
    default:
      tall_side_qr(sh, nparts, 0, SA, l, RA, tauA, tau_tmp, vbig, cs, true);
      tall_side_qr(sh, nparts, 1, SB, l, RB, tauB, tau_tmp, vbig, cs, keepB);
  }
  const long long clk1 = clock64();

  // 2. core W = K^T = R_B R_A^T (qb x qa): group i (8 threads) holds column i
  constexpr int TPC = 8, R = CMAX / TPC;
  const int c8 = t >> 3, g8 = t & 7;
  double w[R];
#pragma unroll
  for (int s = 0; s < R; ++s) {
    const int j = g8 + TPC * s;
    double acc = 0.0;
    if (c8 < qa && j < qb) {
      const int p0 = c8 > j ? c8 : j;
      for (int p = p0; p < l; ++p) acc = fma(RB[j + TALL_RLD * p], RA[c8 + TALL_RLD * p], acc);
    }
    w[s] = acc;
  }
  double amax = 0.0;
#pragma unroll
  for (int s = 0; s < R; ++s) amax = fmax(amax, fabs(w[s]));
  amax = wave_max(amax);
  if (lane == 0) cs.red[wave] = amax;
  __syncthreads();
  amax = 0.0;
#pragma unroll
  for (int i = 0; i < TALL_TB / 64; ++i) amax = fmax(amax, cs.red[i]);
  const bool finite = amax <= 1.7976931348623157e308;
  const bool zero = amax == 0.0;
  double x[R];
#pragma unroll
  for (int s = 0; s < R; ++s) x[s] = 0.0;
  int sweeps = 0;
  int qe = q;  // width of the Jacobi core
  if (finite && !zero) {
    const int e = ilogb(amax);
#pragma unroll
    for (int s = 0; s < R; ++s) w[s] = ldexp(w[s], -e);
    __syncthreads();  // cs.red is reused below
    // pivoted QR stopped at the rounding level, Jacobi on the qe columns of
    // M = R(0:qe, :)^T (rows in the original order)
    QrcpState st;
    qe = core_qrcp<TPC>(w, c8, g8, qb, qa, cvb, cs, 0, CMAX, st);
    core_to_m_piv<TPC>(w, x, c8, g8, qa, qe, st.mine, buf0);
    sweeps = core_jacobi<TPC>(x, c8, g8, qe, buf0, buf1, cs);
    core_order<TPC>(x, c8, g8, qe, cs);
  }
  const long long clk2 = clock64();
  if (t == 0) {
    int k = 0;
    bool bad = !finite;
    if (finite && !zero) k = rank_rule(cs, qe, eps, &bad);
    if (d.kfix >= 0 && finite && !zero) k = d.kfix < qe ? d.kfix : qe;
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
      e[4] = sweeps | (qe << 16);  // Jacobi sweeps, core width
      e[5] = (int)((clk1 - clk0) >> 4);
      e[6] = (int)((clk2 - clk1) >> 4);
    }
    atomicAdd((unsigned long long*)(status + 2), 1ULL);
    atomicAdd((unsigned long long*)(status + 4), 8ULL * (unsigned long long)(m + n) * (unsigned long long)(l + k));
  }
  __syncthreads();
  const int k = sh.rank;
  if (k > 0) {
    // 3. U_k (qa x k) into buf0, T = R_A^T U_k (l x k) into buf1, U_k over
    //    R_B (ld TALL_RLD)
    const int pos = (c8 < qe) ? cs.pos_of[c8] : CMAX;
    if (pos < k) {
      const double sa = cs.sig[c8];
#pragma unroll
      for (int s = 0; s < R; ++s) {
        const int i = g8 + TPC * s;
        if (i < qa) buf0[i + TALL_RLD * pos] = sa > 0.0 ? x[s] / sa : 0.0;
      }
    }
    __syncthreads();
    for (int e = t; e < l * k; e += TALL_TB) {
      const int p = e % l, col = e / l;
      const int iend = p + 1 < qa ? p + 1 : qa;
      double acc = 0.0;
      for (int i = 0; i < iend; ++i) acc = fma(RA[i + TALL_RLD * p], buf0[i + TALL_RLD * col], acc);
      buf1[p + TALL_RLD * col] = acc;
    }
    __syncthreads();
    const bool direct = k <= TALL_D_DIRECT;
    if (!direct) {
      // S = K^T U_k in the Q_B basis = R_B T (qb x k) over R_A
      for (int e = t; e < qb * k; e += TALL_TB) {
        const int j = e % qb, col = e / qb;
        double acc = 0.0;
        for (int p = j; p < l; ++p) acc = fma(RB[j + TALL_RLD * p], buf1[p + TALL_RLD * col], acc);
        RA[j + TALL_RLD * col] = acc;
      }
      __syncthreads();
    }
    for (int e = t; e < qa * k; e += TALL_TB) {
      const int i = e % qa, col = e / qa;
      RB[i + TALL_RLD * col] = buf0[i + TALL_RLD * col];  // the staged reflectors overlay buf0
    }
    if (direct) {
      // 4. D = K^T Q_A U_k = B_s A_s^T Q_A U_k = B_s T (A_s^T Q_A = R_A^T):
      //    one pass over the B stack, staged in the B stack's workspace
      //    (unused: its reflectors were not kept) because D may alias the
      //    stack's first part
      tall_d_from_stack(sh, nparts, n, l, k, buf1, SB.blocks);
      __syncthreads();
      for (int e = t; e < n * k; e += TALL_TB) {
        const int j = e % n, col = e / n;
        d.D[j + (size_t)d.ldd * col] = SB.blocks[j + (size_t)n * col];
      }
    } else {
      __syncthreads();
    }
    // 5. C = Q_A [U_k; 0]; for larger ranks D = Q_B [S; 0]
    tall_side_apply(SA, l, tauA, tau_tmp, RB, qa, k, d.C, d.ldc, Y, vbig);
    if (!direct) tall_side_apply(SB, l, tauB, tau_tmp, RA, qb, k, d.D, d.ldd, Y, vbig);
  }
  if (t == 0) {
    *d.rank = k;
    if (size_log) size_log[8 * (size_t)d.log_idx + 7] = (int)((clock64() - clk2) >> 4);
  }
}

}  // namespace hm
