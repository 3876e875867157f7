// Plain FP64 CPU oracle for hierarchical-matrix arithmetic with accumulated
// updates (Boerm, "Hierarchical matrix arithmetic with accumulated updates").
//
// TEST INFRASTRUCTURE ONLY.  This library is the independent reference that the
// GPU library is checked against.  Only the test suite, the smoke check and the
// CPU-baseline leg of the benchmark may load it.  It shares no code, header or
// helper with the GPU library.
//
// Everything here is deliberately slow and literal: naive loops, Householder QR,
// one-sided (Hestenes) Jacobi SVD, depth-first recursion in the paper's order.
//
// Numbered readings of the paper that this file implements (each is listed with
// its justification in the design notes of the repository):
//   R1  addevaltrans updates X <- X + alpha N^* Y (Fig. addeval prints Y + ...).
//   R2  the recursion of addeval/addevaltrans passes the son's sub-vectors.
//   R3  rkupdate adds alpha A B^* to inadmissible leaves (Fig. rkupdate drops alpha).
//   R4  addproduct applies alpha once, in rkadd; the thin products use 1.
//   R5  the son flush of Fig. flush targets Z restricted to t' x r'.
//   R6  "choose new rank k": the smallest k whose discarded tail satisfies
//       sum_{i>k} sigma_i^2 <= eps^2 sum_i sigma_i^2 (relative Frobenius, per block).
//   R7  an update whose low-rank factors have zero columns is a no-op (no
//       re-truncation of the target).
//   R8  rkmerge merges block columns through adjoints, then block rows.
//   R9  H-LU (standard and accumulated) follows the block-LR pattern of Sect. 6
//       (no pivoting, L unit lower, R upper, stored in place).
//   R10 economy QR when the stacked rank exceeds the block size.
//   R11 the rank rule counts singular values at or below 1e-13 sigma_1 as zero:
//       FP64 data determine no smaller singular values, so the exact rank that
//       the rule asks for at eps = 0 is read as this numerical rank.
//   R14 Fig. invert: the last product, H12 G21, goes into the accumulator of
//       (t1, t1) that is flushed into G11 (the figure names that of (t2, t2));
//       a leaf is flushed before its inverse is formed (the figure inverts
//       without flushing); the leaf inverse is the dense inverse, formed from
//       the unpivoted LU.
//   R15 H-Cholesky (the paper only says it is treated like the inversion):
//       G = L L^*, L in the lower blocks (zeros above the diagonal of the
//       diagonal leaves; the blocks above the diagonal are not used).
//       chol(t) = chol(t0); G10 <- G10 L00^{-*}; G11 <- G11 - G10 G10^* on
//       the lower blocks of G11; chol(t1).  Products X Y^* with Y stored as
//       its own block follow the four branches of Fig. addproduct with the
//       roles of Y's factors exchanged; accumulated: Schur complements go to
//       accumulators without a flush, a block is flushed before it is solved
//       or factorised, and the accumulator of a diagonal block is split into
//       its lower sons only.
//   R16 Fused accumulation (not in the paper; the H^2-style backward
//       transformation that motivates accumulation suggests it): in a split,
//       the low-rank products that reach one son accumulator are added in
//       groups of three consecutive products, each group truncated together
//       with the accumulator in one truncation of the stacked sum; a group
//       whose products all have zero columns is a no-op.
//   R17 The boundary-element matrices of Sect. 7 (no quadrature is given):
//       Galerkin with piecewise constants on flat triangles.  Single layer
//       V_ij = int_Ti int_Tj 1/(4 pi |x - y|); double layer plus half the
//       mass matrix K_ij = |T_i|/2 delta_ij + int_Ti int_Tj
//       <y - x, n_y> / (4 pi |x - y|^3), the sign for which 1/2 + K maps
//       constants to themselves on a closed surface.  Off the diagonal both
//       integrals use the 7-point degree-5 rule (Radon) on each triangle; on
//       the diagonal the double-layer integrand vanishes (flat triangle) and
//       the single layer takes the 7-point rule outside and the closed-form
//       integral of 1/|x - y| over the triangle inside.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

namespace {

// ------------------------------------------------------------------------
// Dense linear algebra (column-major, plain loops)
// ------------------------------------------------------------------------

// C(m x n) += alpha * op(A) * op(B), op(A) is m x k, op(B) is k x n.
void gemm(bool ta, bool tb, int m, int n, int k, double alpha, const double* A, int lda,
          const double* B, int ldb, double* C, int ldc) {
  if (m <= 0 || n <= 0 || k <= 0) return;
  for (int j = 0; j < n; ++j) {
    for (int p = 0; p < k; ++p) {
      double b = tb ? B[j + (size_t)p * ldb] : B[p + (size_t)j * ldb];
      b *= alpha;
      double* c = C + (size_t)j * ldc;
      if (!ta) {
        const double* a = A + (size_t)p * lda;
        for (int i = 0; i < m; ++i) c[i] += a[i] * b;
      } else {
        for (int i = 0; i < m; ++i) c[i] += A[p + (size_t)i * lda] * b;
      }
    }
  }
}

// Euclidean norm with scaling (no overflow or underflow of the squares).
double nrm2(int n, const double* x) {
  double scale = 0.0;
  for (int i = 0; i < n; ++i) scale = std::max(scale, std::fabs(x[i]));
  if (scale == 0.0 || !std::isfinite(scale)) return scale;
  double s = 0.0;
  for (int i = 0; i < n; ++i) {
    double v = x[i] / scale;
    s += v * v;
  }
  return scale * std::sqrt(s);
}

// Householder QR in place (LAPACK geqr2 convention): R in the upper triangle,
// reflector vectors below the diagonal with an implicit unit leading entry,
// H_j = I - tau_j v_j v_j^T.  Number of reflectors = min(m, n).
void house_qr(int m, int n, double* A, int lda, double* tau) {
  int q = std::min(m, n);
  for (int j = 0; j < q; ++j) {
    double* x = A + j + (size_t)j * lda;
    int len = m - j;
    double alpha = x[0];
    double xn = nrm2(len - 1, x + 1);
    if (xn == 0.0) {
      tau[j] = 0.0;
      continue;
    }
    double beta = -std::copysign(std::hypot(alpha, xn), alpha);
    tau[j] = (beta - alpha) / beta;
    // divide (the reciprocal of a subnormal denominator would overflow)
    const double den = alpha - beta;
    for (int i = 1; i < len; ++i) x[i] /= den;
    x[0] = beta;
    for (int c = j + 1; c < n; ++c) {
      double* y = A + j + (size_t)c * lda;
      double w = y[0];
      for (int i = 1; i < len; ++i) w += x[i] * y[i];
      w *= tau[j];
      y[0] -= w;
      for (int i = 1; i < len; ++i) y[i] -= w * x[i];
    }
  }
}

// C(m x c) <- Q C where Q = H_0 H_1 ... H_{q-1} from house_qr.
void apply_q(int m, int q, const double* V, int ldv, const double* tau, double* C, int ldc,
             int c) {
  for (int j = q - 1; j >= 0; --j) {
    if (tau[j] == 0.0) continue;
    const double* v = V + j + (size_t)j * ldv;
    int len = m - j;
    for (int col = 0; col < c; ++col) {
      double* y = C + j + (size_t)col * ldc;
      double w = y[0];
      for (int i = 1; i < len; ++i) w += v[i] * y[i];
      w *= tau[j];
      y[0] -= w;
      for (int i = 1; i < len; ++i) y[i] -= w * v[i];
    }
  }
}

// One-sided (Hestenes) Jacobi on the columns of M (p x q, p >= q).
// On exit the columns of M are mutually orthogonal (M = U Sigma), V (q x q)
// holds the accumulated rotations so that M_in V = M_out.
void jacobi_cols(int p, int q, double* M, int ldm, double* V, int ldv) {
  for (int j = 0; j < q; ++j)
    for (int i = 0; i < q; ++i) V[i + (size_t)j * ldv] = (i == j) ? 1.0 : 0.0;
  const double tol = 1e-15;
  for (int sweep = 0; sweep < 80; ++sweep) {
    bool rotated = false;
    for (int i = 0; i < q - 1; ++i) {
      for (int j = i + 1; j < q; ++j) {
        double* mi = M + (size_t)i * ldm;
        double* mj = M + (size_t)j * ldm;
        // column pair scaled by its largest entry: a, b, c are then free of
        // underflow and the rotation is scale invariant
        double w = 0;
        for (int r = 0; r < p; ++r) w = std::max(w, std::max(std::fabs(mi[r]), std::fabs(mj[r])));
        if (w == 0.0) continue;
        double a = 0, b = 0, c = 0;
        for (int r = 0; r < p; ++r) {
          double x = mi[r] / w, y = mj[r] / w;
          a += x * x;
          b += y * y;
          c += x * y;
        }
        if (c == 0.0 || std::fabs(c) <= tol * std::sqrt(a) * std::sqrt(b)) continue;
        rotated = true;
        double zeta = (b - a) / (2.0 * c);
        double t = std::copysign(1.0, zeta) / (std::fabs(zeta) + std::hypot(1.0, zeta));
        double cs = 1.0 / std::sqrt(1.0 + t * t);
        double sn = cs * t;
        for (int r = 0; r < p; ++r) {
          double x = mi[r], y = mj[r];
          mi[r] = cs * x - sn * y;
          mj[r] = sn * x + cs * y;
        }
        double* vi = V + (size_t)i * ldv;
        double* vj = V + (size_t)j * ldv;
        for (int r = 0; r < q; ++r) {
          double x = vi[r], y = vj[r];
          vi[r] = cs * x - sn * y;
          vj[r] = sn * x + cs * y;
        }
      }
    }
    if (!rotated) break;
  }
}

// Thin SVD of M (p x q): M = U diag(sigma) V^T with r = min(p, q) triples,
// sigma sorted non-increasingly.  Householder QR first, then Jacobi on the
// triangular factor.  U is p x r, V is q x r.
void thin_svd(int p, int q, const double* M, int ldm, std::vector<double>& U,
              std::vector<double>& sigma, std::vector<double>& V) {
  int r = std::min(p, q);
  U.assign((size_t)p * r, 0.0);
  V.assign((size_t)q * r, 0.0);
  sigma.assign(r, 0.0);
  if (r == 0) return;
  bool tall = p >= q;
  int pp = tall ? p : q, qq = tall ? q : p;  // work on M or M^T, pp >= qq = r
  std::vector<double> W((size_t)pp * qq);
  for (int j = 0; j < qq; ++j)
    for (int i = 0; i < pp; ++i)
      W[i + (size_t)j * pp] = tall ? M[i + (size_t)j * ldm] : M[j + (size_t)i * ldm];
  std::vector<double> tau(qq);
  house_qr(pp, qq, W.data(), pp, tau.data());
  std::vector<double> Rm((size_t)qq * qq, 0.0);
  for (int j = 0; j < qq; ++j)
    for (int i = 0; i <= j; ++i) Rm[i + (size_t)j * qq] = W[i + (size_t)j * pp];
  std::vector<double> Vr((size_t)qq * qq);
  jacobi_cols(qq, qq, Rm.data(), qq, Vr.data(), qq);
  std::vector<double> nrm(qq);
  for (int j = 0; j < qq; ++j) nrm[j] = nrm2(qq, Rm.data() + (size_t)j * qq);
  std::vector<int> order(qq);
  for (int j = 0; j < qq; ++j) order[j] = j;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nrm[a] > nrm[b]; });
  // Left vectors of the work matrix: Q [Rm_j / sigma_j; 0]
  std::vector<double> L((size_t)pp * qq, 0.0), Rv((size_t)qq * qq);
  for (int jj = 0; jj < qq; ++jj) {
    int j = order[jj];
    sigma[jj] = nrm[j];
    for (int i = 0; i < qq; ++i) {
      L[i + (size_t)jj * pp] = nrm[j] > 0 ? Rm[i + (size_t)j * qq] / nrm[j] : 0.0;
      Rv[i + (size_t)jj * qq] = Vr[i + (size_t)j * qq];
    }
  }
  apply_q(pp, qq, W.data(), pp, tau.data(), L.data(), pp, qq);
  // W^T... : if tall, M = L S Rv^T; else M^T = L S Rv^T -> M = Rv S L^T
  if (tall) {
    U = L;
    V = Rv;
  } else {
    U = Rv;
    V = L;
  }
}

// Rank rule R6.  tail[j] = sum_{i>j} sigma_i^2 summed from the smallest
// singular value upwards; k = smallest j with tail[j] <= eps^2 tail[0].
int choose_rank(const std::vector<double>& sigma, double eps, double* margin_k,
                double* margin_km1) {
  int q = (int)sigma.size();
  std::vector<double> tail(q + 1, 0.0);
  for (int i = q - 1; i >= 0; --i) tail[i] = tail[i + 1] + sigma[i] * sigma[i];
  double thr = eps * eps * tail[0];
  int k = 0;
  if (tail[0] > 0.0) {
    k = q;
    for (int j = 0; j <= q; ++j)
      if (tail[j] <= thr) {
        k = j;
        break;
      }
  }
  // R11: values at or below 1e-13 sigma_1 are rounding noise
  int nz = 0;
  while (nz < q && sigma[nz] > 1e-13 * sigma[0]) ++nz;
  if (k > nz) k = nz;
  if (margin_k) *margin_k = thr > 0 ? std::fabs(tail[k] - thr) / thr : INFINITY;
  if (margin_km1) *margin_km1 = (thr > 0 && k > 0) ? std::fabs(tail[k - 1] - thr) / thr : INFINITY;
  return k;
}

// ------------------------------------------------------------------------
// Statistics and truncation log
// ------------------------------------------------------------------------
struct Stats {
  int64_t trunc_update = 0;   // rkadd inside rkupdate (target = matrix leaf)
  int64_t trunc_accum = 0;    // rkadd into an accumulator
  int64_t trunc_merge = 0;    // rowmerge truncations
  int64_t dense_updates = 0;  // N += alpha A B^*
  int64_t addproduct = 0;     // addproduct calls
  int64_t pending = 0;        // products appended to a pending list
  int64_t products = 0;       // low-rank products formed (both variants)
  int64_t leaf_lu = 0;
  int64_t merges = 0;         // rkmerge calls
  int64_t trunc_flops = 0;    // (m+n) * l^2 per truncation, a size measure
};

struct LogRec {
  int32_t kind, m, n, k1, k2, k;
  double margin_k, margin_km1;
};

struct Ctx {
  double eps = 0.0;
  bool fused = false;  // R16: products of a split added to an accumulator three at a time
  Stats st;
  bool log = false;
  std::vector<LogRec> logv;
};

// ------------------------------------------------------------------------
// Low-rank matrices and the truncated addition (Fig. rkadd)
// ------------------------------------------------------------------------
struct RK {
  int rows = 0, cols = 0, k = 0;
  std::vector<double> A, B;  // rows x k, cols x k
};

enum { KIND_UPDATE = 0, KIND_ACCUM = 1, KIND_MERGE = 2, KIND_RAW = 3 };

// R2 <- trunc(R2 + alpha R1), R1 = A B^*, R2 = C D^* (Fig. rkadd).
void rkadd(Ctx& cx, int kind, double alpha, int k1, const double* A, int lda, const double* B,
           int ldb, RK& R2, std::vector<double>* sigma_out = nullptr) {
  if (k1 == 0) return;  // R7
  int m = R2.rows, n = R2.cols, k2 = R2.k, l = k1 + k2;
  // QR of the stacked right factor [B D]
  std::vector<double> S((size_t)n * l);
  for (int j = 0; j < k1; ++j)
    for (int i = 0; i < n; ++i) S[i + (size_t)j * n] = B[i + (size_t)j * ldb];
  for (int j = 0; j < k2; ++j)
    for (int i = 0; i < n; ++i) S[i + (size_t)(k1 + j) * n] = R2.B[i + (size_t)j * n];
  int qB = std::min(n, l);
  std::vector<double> tauB(qB);
  house_qr(n, l, S.data(), n, tauB.data());
  // Ahat = [alpha A, C] R_B^*  (m x qB); R_B is qB x l upper trapezoidal
  std::vector<double> Ahat((size_t)m * qB, 0.0);
  for (int c = 0; c < qB; ++c) {
    for (int j = c; j < l; ++j) {
      double rb = S[c + (size_t)j * n];
      double coef = (j < k1) ? alpha * rb : rb;
      const double* col = (j < k1) ? A + (size_t)j * lda : R2.A.data() + (size_t)(j - k1) * m;
      double* out = Ahat.data() + (size_t)c * m;
      for (int i = 0; i < m; ++i) out[i] += col[i] * coef;
    }
  }
  std::vector<double> U, sigma, Vh;
  thin_svd(m, qB, Ahat.data(), m, U, sigma, Vh);
  double mk = 0, mk1 = 0;
  int k = choose_rank(sigma, cx.eps, &mk, &mk1);
  // C <- U(:, 1:k);  D <- Q_B [Vhat(:, 1:k) Sigma_k; 0]
  RK out;
  out.rows = m;
  out.cols = n;
  out.k = k;
  out.A.assign((size_t)m * k, 0.0);
  out.B.assign((size_t)n * k, 0.0);
  for (int j = 0; j < k; ++j) {
    for (int i = 0; i < m; ++i) out.A[i + (size_t)j * m] = U[i + (size_t)j * m];
    for (int i = 0; i < qB; ++i) out.B[i + (size_t)j * n] = Vh[i + (size_t)j * qB] * sigma[j];
  }
  apply_q(n, qB, S.data(), n, tauB.data(), out.B.data(), n, k);
  R2 = std::move(out);
  if (kind == KIND_UPDATE) cx.st.trunc_update++;
  if (kind == KIND_ACCUM) cx.st.trunc_accum++;
  if (kind == KIND_MERGE) cx.st.trunc_merge++;
  cx.st.trunc_flops += (int64_t)(m + n) * l * l;
  if (cx.log) cx.logv.push_back({kind, m, n, k1, k2, k, mk, mk1});
  if (sigma_out) *sigma_out = sigma;
}

// R2 <- trunc(R2 + sum_q alpha_q A_q B_q^*): the stacked form of Fig. rkadd
// with several updates (R16).  QR of [B_1 ... B_g D], then the SVD of
// [alpha_1 A_1 ... alpha_g A_g C] R_B^*.  Updates with zero columns add
// nothing; when all have zero columns R2 is left as it is.
struct Upd {
  double alpha;
  int k;
  const double* A;
  int lda;
  const double* B;
  int ldb;
};

void rkadd_multi(Ctx& cx, int kind, const std::vector<Upd>& u, RK& R2) {
  int k1 = 0;
  for (const Upd& q : u) k1 += q.k;
  if (k1 == 0) return;
  int m = R2.rows, n = R2.cols, k2 = R2.k, l = k1 + k2;
  std::vector<double> S((size_t)n * l);
  int c = 0;
  for (const Upd& q : u)
    for (int j = 0; j < q.k; ++j, ++c)
      for (int i = 0; i < n; ++i) S[i + (size_t)c * n] = q.B[i + (size_t)j * q.ldb];
  for (int j = 0; j < k2; ++j, ++c)
    for (int i = 0; i < n; ++i) S[i + (size_t)c * n] = R2.B[i + (size_t)j * n];
  int qB = std::min(n, l);
  std::vector<double> tauB(qB);
  house_qr(n, l, S.data(), n, tauB.data());
  // the stacked left factor [alpha_1 A_1 ... C]
  std::vector<double> As((size_t)m * l);
  c = 0;
  for (const Upd& q : u)
    for (int j = 0; j < q.k; ++j, ++c)
      for (int i = 0; i < m; ++i) As[i + (size_t)c * m] = q.alpha * q.A[i + (size_t)j * q.lda];
  for (int j = 0; j < k2; ++j, ++c)
    for (int i = 0; i < m; ++i) As[i + (size_t)c * m] = R2.A[i + (size_t)j * m];
  std::vector<double> Ahat((size_t)m * qB, 0.0);
  for (int cc = 0; cc < qB; ++cc)
    for (int j = cc; j < l; ++j) {
      double rb = S[cc + (size_t)j * n];
      for (int i = 0; i < m; ++i) Ahat[i + (size_t)cc * m] += As[i + (size_t)j * m] * rb;
    }
  std::vector<double> U, sigma, Vh;
  thin_svd(m, qB, Ahat.data(), m, U, sigma, Vh);
  double mk = 0, mk1 = 0;
  int k = choose_rank(sigma, cx.eps, &mk, &mk1);
  RK out;
  out.rows = m;
  out.cols = n;
  out.k = k;
  out.A.assign((size_t)m * k, 0.0);
  out.B.assign((size_t)n * k, 0.0);
  for (int j = 0; j < k; ++j) {
    for (int i = 0; i < m; ++i) out.A[i + (size_t)j * m] = U[i + (size_t)j * m];
    for (int i = 0; i < qB; ++i) out.B[i + (size_t)j * n] = Vh[i + (size_t)j * qB] * sigma[j];
  }
  apply_q(n, qB, S.data(), n, tauB.data(), out.B.data(), n, k);
  R2 = std::move(out);
  if (kind == KIND_ACCUM) cx.st.trunc_accum++;
  cx.st.trunc_flops += (int64_t)(m + n) * l * l;
  if (cx.log) cx.logv.push_back({kind, m, n, k1, k2, k, mk, mk1});
}

// rowmerge (Fig. rkmerge): R = [R_1 ... R_p] with R_j = A_j B_j^* on column
// blocks of widths n_j.  Returns the truncated factorisation of the whole row.
RK rowmerge(Ctx& cx, const std::vector<const RK*>& parts) {
  RK out;
  int p = (int)parts.size();
  int m = parts[0]->rows, n = 0, qs = 0;
  for (auto* r : parts) {
    n += r->cols;
    qs += std::min(r->cols, r->k);
  }
  out.rows = m;
  out.cols = n;
  out.k = 0;
  if (qs == 0) return out;
  std::vector<std::vector<double>> QB(p), tau(p);
  std::vector<double> Ahat((size_t)m * qs, 0.0);
  int col0 = 0;
  for (int j = 0; j < p; ++j) {
    const RK& r = *parts[j];
    int qj = std::min(r.cols, r.k);
    QB[j] = r.B;
    tau[j].assign(qj, 0.0);
    if (qj == 0) continue;
    house_qr(r.cols, r.k, QB[j].data(), r.cols, tau[j].data());
    // A_j R_{B,j}^* : m x qj
    for (int c = 0; c < qj; ++c)
      for (int jj = c; jj < r.k; ++jj) {
        double rb = QB[j][c + (size_t)jj * r.cols];
        for (int i = 0; i < m; ++i)
          Ahat[i + (size_t)(col0 + c) * m] += r.A[i + (size_t)jj * m] * rb;
      }
    col0 += qj;
  }
  std::vector<double> U, sigma, Vh;
  thin_svd(m, qs, Ahat.data(), m, U, sigma, Vh);
  double mk = 0, mk1 = 0;
  int k = choose_rank(sigma, cx.eps, &mk, &mk1);
  out.k = k;
  out.A.assign((size_t)m * k, 0.0);
  out.B.assign((size_t)n * k, 0.0);
  for (int c = 0; c < k; ++c)
    for (int i = 0; i < m; ++i) out.A[i + (size_t)c * m] = U[i + (size_t)c * m];
  // B = blockdiag(Q_{B,j}) Vhat(:, 1:k) Sigma_k
  col0 = 0;
  int row0 = 0;
  for (int j = 0; j < p; ++j) {
    const RK& r = *parts[j];
    int qj = std::min(r.cols, r.k);
    if (qj > 0) {
      std::vector<double> T((size_t)r.cols * k, 0.0);
      for (int c = 0; c < k; ++c)
        for (int i = 0; i < qj; ++i)
          T[i + (size_t)c * r.cols] = Vh[(col0 + i) + (size_t)c * qs] * sigma[c];
      apply_q(r.cols, qj, QB[j].data(), r.cols, tau[j].data(), T.data(), r.cols, k);
      for (int c = 0; c < k; ++c)
        for (int i = 0; i < r.cols; ++i) out.B[(row0 + i) + (size_t)c * n] = T[i + (size_t)c * r.cols];
    }
    col0 += qj;
    row0 += r.cols;
  }
  cx.st.trunc_merge++;
  cx.st.trunc_flops += (int64_t)(m + n) * qs * qs;
  if (cx.log) cx.logv.push_back({KIND_MERGE, m, n, qs, 0, k, mk, mk1});
  return out;
}

RK adjoint(const RK& r) {
  RK a;
  a.rows = r.cols;
  a.cols = r.rows;
  a.k = r.k;
  a.A = r.B;
  a.B = r.A;
  return a;
}

// rkmerge of a p x q grid (row-major), reading R8: block columns first (through
// adjoints), then the block row.
RK rkmerge(Ctx& cx, const std::vector<const RK*>& grid, int p, int q) {
  std::vector<RK> cols(q);
  for (int j = 0; j < q; ++j) {
    std::vector<RK> adj(p);
    std::vector<const RK*> ptr(p);
    for (int i = 0; i < p; ++i) {
      adj[i] = adjoint(*grid[i * q + j]);
      ptr[i] = &adj[i];
    }
    cols[j] = adjoint(rowmerge(cx, ptr));
  }
  std::vector<const RK*> ptr(q);
  for (int j = 0; j < q; ++j) ptr[j] = &cols[j];
  cx.st.merges++;
  return rowmerge(cx, ptr);
}

// ------------------------------------------------------------------------
// Cluster tree and block tree (Defs. cluster tree / block tree)
// ------------------------------------------------------------------------
struct Cluster {
  int off = 0, size = 0, level = 0, nsons = 0;
  int son[2] = {-1, -1};
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
};

struct CTree {
  int dim = 0;
  std::vector<int> perm;  // position -> original index
  std::vector<Cluster> c;
};

// Geometric bisection: split a cluster at the midpoint of the longest side of
// its tight bounding box (lowest axis on ties); points with coordinate <= mid
// go to the first son, in their original relative order.
int build_cluster(CTree& T, const double* x, int off, int size, int level, int leaf) {
  int id = (int)T.c.size();
  T.c.emplace_back();
  Cluster cl;
  cl.off = off;
  cl.size = size;
  cl.level = level;
  for (int d = 0; d < T.dim; ++d) {
    cl.lo[d] = INFINITY;
    cl.hi[d] = -INFINITY;
  }
  for (int i = off; i < off + size; ++i)
    for (int d = 0; d < T.dim; ++d) {
      double v = x[(size_t)T.perm[i] * T.dim + d];
      cl.lo[d] = std::min(cl.lo[d], v);
      cl.hi[d] = std::max(cl.hi[d], v);
    }
  int axis = 0;
  double ext = -1;
  for (int d = 0; d < T.dim; ++d)
    if (cl.hi[d] - cl.lo[d] > ext) {
      ext = cl.hi[d] - cl.lo[d];
      axis = d;
    }
  if (size > leaf && ext > 0) {
    double mid = 0.5 * (cl.lo[axis] + cl.hi[axis]);
    std::vector<int> left, right;
    for (int i = off; i < off + size; ++i) {
      int g = T.perm[i];
      if (x[(size_t)g * T.dim + axis] <= mid)
        left.push_back(g);
      else
        right.push_back(g);
    }
    int p = off;
    for (int g : left) T.perm[p++] = g;
    for (int g : right) T.perm[p++] = g;
    cl.nsons = 2;
    T.c[id] = cl;
    int s0 = build_cluster(T, x, off, (int)left.size(), level + 1, leaf);
    int s1 = build_cluster(T, x, off + (int)left.size(), (int)right.size(), level + 1, leaf);
    T.c[id].son[0] = s0;
    T.c[id].son[1] = s1;
  } else {
    T.c[id] = cl;
  }
  return id;
}

enum { NONLEAF = 0, RKLEAF = 1, DENSE = 2 };

struct Node {
  int t = -1, s = -1, kind = NONLEAF, rows = 0, cols = 0, roff = 0, coff = 0;
  int nt = 0, ns = 0;  // number of row / column sons
  std::vector<Node*> sons;
  RK rk;
  std::vector<double> N;
  ~Node() {
    for (Node* p : sons) delete p;
  }
  Node* son(int i, int j) const { return sons[(size_t)i * ns + j]; }
};

Node* make_node(const CTree& T, int t, int s, int kind) {
  Node* b = new Node;
  b->t = t;
  b->s = s;
  b->kind = kind;
  b->rows = T.c[t].size;
  b->cols = T.c[s].size;
  b->roff = T.c[t].off;
  b->coff = T.c[s].off;
  if (kind == RKLEAF) {
    b->rk.rows = b->rows;
    b->rk.cols = b->cols;
  }
  if (kind == DENSE) b->N.assign((size_t)b->rows * b->cols, 0.0);
  return b;
}

// Admissibility: max(diam t, diam s) <= eta dist(t, s), evaluated on squared
// quantities of the tight bounding boxes; dist = 0 is never admissible.
bool admissible(const CTree& T, int t, int s, double eta) {
  const Cluster &a = T.c[t], &b = T.c[s];
  double dt = 0, ds = 0, dist = 0;
  for (int d = 0; d < T.dim; ++d) {
    dt += (a.hi[d] - a.lo[d]) * (a.hi[d] - a.lo[d]);
    ds += (b.hi[d] - b.lo[d]) * (b.hi[d] - b.lo[d]);
    double g = std::max(0.0, std::max(b.lo[d] - a.hi[d], a.lo[d] - b.hi[d]));
    dist += g * g;
  }
  return dist > 0 && std::max(dt, ds) <= eta * eta * dist;
}

Node* build_block(const CTree& T, int t, int s, double eta) {
  if (admissible(T, t, s, eta)) return make_node(T, t, s, RKLEAF);
  if (T.c[t].nsons == 0 || T.c[s].nsons == 0) return make_node(T, t, s, DENSE);
  Node* b = make_node(T, t, s, NONLEAF);
  b->nt = T.c[t].nsons;
  b->ns = T.c[s].nsons;
  for (int i = 0; i < b->nt; ++i)
    for (int j = 0; j < b->ns; ++j) b->sons.push_back(build_block(T, T.c[t].son[i], T.c[s].son[j], eta));
  return b;
}

Node* clone(const Node* a) {
  Node* b = new Node;
  b->t = a->t;
  b->s = a->s;
  b->kind = a->kind;
  b->rows = a->rows;
  b->cols = a->cols;
  b->roff = a->roff;
  b->coff = a->coff;
  b->nt = a->nt;
  b->ns = a->ns;
  b->rk = a->rk;
  b->N = a->N;
  for (Node* p : a->sons) b->sons.push_back(clone(p));
  return b;
}

void zero_node(Node* a) {
  if (a->kind == DENSE) std::fill(a->N.begin(), a->N.end(), 0.0);
  if (a->kind == RKLEAF) {
    a->rk.k = 0;
    a->rk.A.clear();
    a->rk.B.clear();
  }
  for (Node* p : a->sons) zero_node(p);
}

// ------------------------------------------------------------------------
// addeval / addevaltrans (Fig. addeval, readings R1, R2)
// ------------------------------------------------------------------------
// Y(#t x c) += alpha G|_{t x s} W, W is #s x c.
void addeval(double alpha, const Node* G, const double* W, int ldw, int c, double* Y, int ldy) {
  if (c == 0) return;
  if (G->kind == DENSE) {
    gemm(false, false, G->rows, c, G->cols, alpha, G->N.data(), G->rows, W, ldw, Y, ldy);
  } else if (G->kind == RKLEAF) {
    int k = G->rk.k;
    if (k == 0) return;
    std::vector<double> Z((size_t)k * c, 0.0);
    gemm(true, false, k, c, G->cols, alpha, G->rk.B.data(), G->cols, W, ldw, Z.data(), k);
    gemm(false, false, G->rows, c, k, 1.0, G->rk.A.data(), G->rows, Z.data(), k, Y, ldy);
  } else {
    for (Node* b : G->sons)
      addeval(alpha, b, W + (b->coff - G->coff), ldw, c, Y + (b->roff - G->roff), ldy);
  }
}

// X(#s x c) += alpha G|_{t x s}^* Y, Y is #t x c.
void addevaltrans(double alpha, const Node* G, const double* Y, int ldy, int c, double* X, int ldx) {
  if (c == 0) return;
  if (G->kind == DENSE) {
    gemm(true, false, G->cols, c, G->rows, alpha, G->N.data(), G->rows, Y, ldy, X, ldx);
  } else if (G->kind == RKLEAF) {
    int k = G->rk.k;
    if (k == 0) return;
    std::vector<double> Z((size_t)k * c, 0.0);
    gemm(true, false, k, c, G->rows, alpha, G->rk.A.data(), G->rows, Y, ldy, Z.data(), k);
    gemm(false, false, G->cols, c, k, 1.0, G->rk.B.data(), G->cols, Z.data(), k, X, ldx);
  } else {
    for (Node* b : G->sons)
      addevaltrans(alpha, b, Y + (b->roff - G->roff), ldy, c, X + (b->coff - G->coff), ldx);
  }
}

// ------------------------------------------------------------------------
// Low-rank representation of X|_{t x s} Y|_{s x r} when (t,s) or (s,r) is a
// leaf: the four branches of Fig. addproduct (without alpha, reading R4).
// ------------------------------------------------------------------------
struct LRProd {
  int rows = 0, cols = 0, k = 0;
  std::vector<double> A, B;  // rows x k, cols x k
};

void identity(std::vector<double>& M, int n) {
  M.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) M[i + (size_t)i * n] = 1.0;
}

LRProd lowrank_product(Ctx& cx, const Node* X, const Node* Y) {
  LRProd p;
  p.rows = X->rows;
  p.cols = Y->cols;
  int nt = X->rows, ns = X->cols, nr = Y->cols;
  cx.st.products++;
  if (X->kind == DENSE) {
    if (nt <= ns) {  // A = I, B = Y^* N_X^*
      p.k = nt;
      identity(p.A, nt);
      p.B.assign((size_t)nr * nt, 0.0);
      std::vector<double> NT((size_t)ns * nt);
      for (int i = 0; i < nt; ++i)
        for (int j = 0; j < ns; ++j) NT[j + (size_t)i * ns] = X->N[i + (size_t)j * nt];
      addevaltrans(1.0, Y, NT.data(), ns, nt, p.B.data(), nr);
    } else {  // A = N_X, B = Y^* I
      p.k = ns;
      p.A = X->N;
      p.B.assign((size_t)nr * ns, 0.0);
      std::vector<double> I;
      identity(I, ns);
      addevaltrans(1.0, Y, I.data(), ns, ns, p.B.data(), nr);
    }
  } else if (Y->kind == DENSE) {
    if (nr <= ns) {  // B = I, A = X N_Y
      p.k = nr;
      identity(p.B, nr);
      p.A.assign((size_t)nt * nr, 0.0);
      addeval(1.0, X, Y->N.data(), ns, nr, p.A.data(), nt);
    } else {  // B = N_Y^*, A = X I
      p.k = ns;
      p.B.assign((size_t)nr * ns, 0.0);
      for (int i = 0; i < ns; ++i)
        for (int j = 0; j < nr; ++j) p.B[j + (size_t)i * nr] = Y->N[i + (size_t)j * ns];
      p.A.assign((size_t)nt * ns, 0.0);
      std::vector<double> I;
      identity(I, ns);
      addeval(1.0, X, I.data(), ns, ns, p.A.data(), nt);
    }
  } else if (X->kind == RKLEAF) {  // A = A_X, B = Y^* B_X
    p.k = X->rk.k;
    p.A = X->rk.A;
    p.B.assign((size_t)nr * p.k, 0.0);
    addevaltrans(1.0, Y, X->rk.B.data(), ns, p.k, p.B.data(), nr);
  } else {  // Y admissible leaf: B = B_Y, A = X A_Y
    p.k = Y->rk.k;
    p.B = Y->rk.B;
    p.A.assign((size_t)nt * p.k, 0.0);
    addeval(1.0, X, Y->rk.A.data(), ns, p.k, p.A.data(), nt);
  }
  return p;
}

// ------------------------------------------------------------------------
// rkupdate (Fig. rkupdate, reading R3)
// ------------------------------------------------------------------------
void rkupdate(Ctx& cx, double alpha, int k, const double* A, int lda, const double* B, int ldb,
              Node* Z) {
  if (k == 0) return;  // R7
  if (Z->kind == DENSE) {
    gemm(false, true, Z->rows, Z->cols, k, alpha, A, lda, B, ldb, Z->N.data(), Z->rows);
    cx.st.dense_updates++;
  } else if (Z->kind == RKLEAF) {
    rkadd(cx, KIND_UPDATE, alpha, k, A, lda, B, ldb, Z->rk);
  } else {
    for (Node* b : Z->sons)
      rkupdate(cx, alpha, k, A + (b->roff - Z->roff), lda, B + (b->coff - Z->coff), ldb, b);
  }
}

// Temporary sons of a leaf Z (dense sub-blocks or restricted factors).
void make_temps(const CTree& T, Node* Z) {
  const Cluster &ct = T.c[Z->t], &cs = T.c[Z->s];
  Z->nt = ct.nsons;
  Z->ns = cs.nsons;
  for (int i = 0; i < ct.nsons; ++i)
    for (int j = 0; j < cs.nsons; ++j) {
      Node* b = make_node(T, ct.son[i], cs.son[j], Z->kind);
      int ro = b->roff - Z->roff, co = b->coff - Z->coff;
      if (Z->kind == DENSE) {
        for (int c = 0; c < b->cols; ++c)
          for (int r = 0; r < b->rows; ++r)
            b->N[r + (size_t)c * b->rows] = Z->N[(ro + r) + (size_t)(co + c) * Z->rows];
      } else {
        int k = Z->rk.k;
        b->rk.k = k;
        b->rk.A.assign((size_t)b->rows * k, 0.0);
        b->rk.B.assign((size_t)b->cols * k, 0.0);
        for (int c = 0; c < k; ++c) {
          for (int r = 0; r < b->rows; ++r)
            b->rk.A[r + (size_t)c * b->rows] = Z->rk.A[(ro + r) + (size_t)c * Z->rows];
          for (int r = 0; r < b->cols; ++r)
            b->rk.B[r + (size_t)c * b->cols] = Z->rk.B[(co + r) + (size_t)c * Z->cols];
        }
      }
      Z->sons.push_back(b);
    }
}

void merge_temps(Ctx& cx, Node* Z) {
  if (Z->kind == DENSE) {
    for (Node* b : Z->sons) {
      int ro = b->roff - Z->roff, co = b->coff - Z->coff;
      for (int c = 0; c < b->cols; ++c)
        for (int r = 0; r < b->rows; ++r)
          Z->N[(ro + r) + (size_t)(co + c) * Z->rows] = b->N[r + (size_t)c * b->rows];
    }
  } else {
    std::vector<const RK*> grid;
    for (Node* b : Z->sons) grid.push_back(&b->rk);
    Z->rk = rkmerge(cx, grid, Z->nt, Z->ns);
  }
  for (Node* b : Z->sons) delete b;
  Z->sons.clear();
  Z->nt = Z->ns = 0;
}

bool is_leaf(const Node* b) { return b->kind != NONLEAF; }

// ------------------------------------------------------------------------
// Standard multiplication Z <- blocktrunc(Z + alpha X Y)  (Sect. 4)
// ------------------------------------------------------------------------
void mul_std(Ctx& cx, const CTree& T, double alpha, const Node* X, const Node* Y, Node* Z) {
  if (is_leaf(X) || is_leaf(Y)) {
    LRProd p = lowrank_product(cx, X, Y);
    rkupdate(cx, alpha, p.k, p.A.data(), p.rows, p.B.data(), p.cols, Z);
    return;
  }
  bool temps = is_leaf(Z);
  if (temps) make_temps(T, Z);
  for (int i = 0; i < X->nt; ++i)
    for (int j = 0; j < Y->ns; ++j)
      for (int l = 0; l < X->ns; ++l) mul_std(cx, T, alpha, X->son(i, l), Y->son(l, j), Z->son(i, j));
  if (temps) merge_temps(cx, Z);
}

// ------------------------------------------------------------------------
// Accumulators: addproduct / split / flush (Figs. addproduct, split, flush)
// ------------------------------------------------------------------------
struct Pending {
  double alpha;
  const Node* X;
  const Node* Y;
  bool trans = false;  // the product X Y^* (H-Cholesky) instead of X Y
};

struct Acc {
  RK R;
  std::vector<Pending> P;
};

Acc empty_acc(int rows, int cols) {
  Acc a;
  a.R.rows = rows;
  a.R.cols = cols;
  return a;
}

void addproduct(Ctx& cx, double alpha, const Node* X, const Node* Y, Acc& acc) {
  cx.st.addproduct++;
  if (is_leaf(X) || is_leaf(Y)) {
    LRProd p = lowrank_product(cx, X, Y);
    rkadd(cx, KIND_ACCUM, alpha, p.k, p.A.data(), p.rows, p.B.data(), p.cols, acc.R);
  } else {
    acc.P.push_back({alpha, X, Y});
    cx.st.pending++;
  }
}

void addproduct_t(Ctx& cx, double alpha, const Node* X, const Node* Y, Acc& acc);
LRProd lowrank_product_t(Ctx& cx, const Node* X, const Node* Y);

// The pending products of acc restricted to the son (i, j), added to the son
// accumulator a: one truncation per leaf product, or (R16) in groups of three
// consecutive leaf products, each group with a in one truncation.
void add_restricted(Ctx& cx, const Acc& acc, int i, int j, Acc& a) {
  if (!cx.fused) {
    for (const Pending& p : acc.P)
      for (int l = 0; l < p.X->ns; ++l) {
        if (p.trans)
          addproduct_t(cx, p.alpha, p.X->son(i, l), p.Y->son(j, l), a);
        else
          addproduct(cx, p.alpha, p.X->son(i, l), p.Y->son(l, j), a);
      }
    return;
  }
  std::vector<LRProd> prods;
  std::vector<double> alphas;
  for (const Pending& p : acc.P)
    for (int l = 0; l < p.X->ns; ++l) {
      const Node* X = p.X->son(i, l);
      const Node* Y = p.trans ? p.Y->son(j, l) : p.Y->son(l, j);
      cx.st.addproduct++;
      if (is_leaf(X) || is_leaf(Y)) {
        prods.push_back(p.trans ? lowrank_product_t(cx, X, Y) : lowrank_product(cx, X, Y));
        alphas.push_back(p.alpha);
      } else {
        a.P.push_back({p.alpha, X, Y, p.trans});
        cx.st.pending++;
      }
    }
  for (size_t g = 0; g < prods.size(); g += 3) {
    std::vector<Upd> u;
    for (size_t q = g; q < std::min(prods.size(), g + 3); ++q)
      u.push_back({alphas[q], prods[q].k, prods[q].A.data(), prods[q].rows, prods[q].B.data(), prods[q].cols});
    rkadd_multi(cx, KIND_ACCUM, u, a.R);
  }
}

// Son accumulators in row-major order over sons(t) x sons(r).
std::vector<Acc> split(Ctx& cx, const CTree& T, int t, int r, Acc& acc) {
  const Cluster &ct = T.c[t], &cr = T.c[r];
  std::vector<Acc> out;
  for (int i = 0; i < ct.nsons; ++i)
    for (int j = 0; j < cr.nsons; ++j) {
      const Cluster &ti = T.c[ct.son[i]], &rj = T.c[cr.son[j]];
      Acc a = empty_acc(ti.size, rj.size);
      int k = acc.R.k;
      a.R.k = k;
      a.R.A.assign((size_t)ti.size * k, 0.0);
      a.R.B.assign((size_t)rj.size * k, 0.0);
      for (int c = 0; c < k; ++c) {
        for (int q = 0; q < ti.size; ++q)
          a.R.A[q + (size_t)c * ti.size] = acc.R.A[(ti.off - ct.off + q) + (size_t)c * ct.size];
        for (int q = 0; q < rj.size; ++q)
          a.R.B[q + (size_t)c * rj.size] = acc.R.B[(rj.off - cr.off + q) + (size_t)c * cr.size];
      }
      add_restricted(cx, acc, i, j, a);
      out.push_back(std::move(a));
    }
  return out;
}

// Split of the accumulator of a diagonal block (t, t) of the H-Cholesky into
// its lower sons (t0, t0), (t1, t0), (t1, t1), in that order: the restricted
// low-rank part and the pending products re-added for every son of s, as in
// split(); the upper son is not formed.
std::vector<Acc> split_lower(Ctx& cx, const CTree& T, int t, Acc& acc) {
  const Cluster& ct = T.c[t];
  std::vector<Acc> out;
  for (int i = 0; i < ct.nsons; ++i)
    for (int j = 0; j <= i; ++j) {
      const Cluster &ti = T.c[ct.son[i]], &tj = T.c[ct.son[j]];
      Acc a = empty_acc(ti.size, tj.size);
      int k = acc.R.k;
      a.R.k = k;
      a.R.A.assign((size_t)ti.size * k, 0.0);
      a.R.B.assign((size_t)tj.size * k, 0.0);
      for (int c = 0; c < k; ++c) {
        for (int q = 0; q < ti.size; ++q)
          a.R.A[q + (size_t)c * ti.size] = acc.R.A[(ti.off - ct.off + q) + (size_t)c * ct.size];
        for (int q = 0; q < tj.size; ++q)
          a.R.B[q + (size_t)c * tj.size] = acc.R.B[(tj.off - ct.off + q) + (size_t)c * ct.size];
      }
      add_restricted(cx, acc, i, j, a);
      out.push_back(std::move(a));
    }
  return out;
}

void flush(Ctx& cx, const CTree& T, Acc& acc, Node* Z) {
  if (acc.P.empty()) {
    rkupdate(cx, 1.0, acc.R.k, acc.R.A.data(), acc.R.rows, acc.R.B.data(), acc.R.cols, Z);
  } else {
    bool temps = is_leaf(Z);
    if (temps) make_temps(T, Z);
    std::vector<Acc> sons = split(cx, T, Z->t, Z->s, acc);
    for (int i = 0; i < Z->nt; ++i)
      for (int j = 0; j < Z->ns; ++j) flush(cx, T, sons[(size_t)i * Z->ns + j], Z->son(i, j));
    if (temps) merge_temps(cx, Z);
  }
  acc.R.k = 0;
  acc.R.A.clear();
  acc.R.B.clear();
  acc.P.clear();
}

void mul_acc(Ctx& cx, const CTree& T, double alpha, const Node* X, const Node* Y, Node* Z) {
  Acc acc = empty_acc(Z->rows, Z->cols);
  addproduct(cx, alpha, X, Y, acc);
  flush(cx, T, acc, Z);
}

// ------------------------------------------------------------------------
// Dense leaf factorisation and thin-RHS triangular solves (reading R9)
// ------------------------------------------------------------------------
void dense_lu(int n, double* N) {
  for (int k = 0; k < n; ++k) {
    double piv = N[k + (size_t)k * n];
    if (piv == 0.0) throw std::runtime_error("zero pivot in leaf LU");
    for (int i = k + 1; i < n; ++i) N[i + (size_t)k * n] /= piv;
    for (int j = k + 1; j < n; ++j) {
      double u = N[k + (size_t)j * n];
      for (int i = k + 1; i < n; ++i) N[i + (size_t)j * n] -= N[i + (size_t)k * n] * u;
    }
  }
}

// X(#t x c) <- L_tt^{-1} X, L unit lower (strict lower part of G|_{t x t}).
void solve_L(const Node* G, double* X, int ldx, int c) {
  if (c == 0) return;
  if (G->kind == DENSE) {
    int n = G->rows;
    for (int col = 0; col < c; ++col) {
      double* x = X + (size_t)col * ldx;
      for (int i = 0; i < n; ++i) {
        double s = x[i];
        for (int p = 0; p < i; ++p) s -= G->N[i + (size_t)p * n] * x[p];
        x[i] = s;
      }
    }
    return;
  }
  const Node *G00 = G->son(0, 0), *G10 = G->son(1, 0), *G11 = G->son(1, 1);
  double* X0 = X;
  double* X1 = X + (G11->roff - G->roff);
  solve_L(G00, X0, ldx, c);
  addeval(-1.0, G10, X0, ldx, c, X1, ldx);
  solve_L(G11, X1, ldx, c);
}

// X(#t x c) <- R_tt^{-*} X, R upper (upper part of G|_{t x t}).
void solve_Rt(const Node* G, double* X, int ldx, int c) {
  if (c == 0) return;
  if (G->kind == DENSE) {
    int n = G->rows;
    for (int col = 0; col < c; ++col) {
      double* x = X + (size_t)col * ldx;
      for (int i = 0; i < n; ++i) {
        double s = x[i];
        for (int p = 0; p < i; ++p) s -= G->N[p + (size_t)i * n] * x[p];
        x[i] = s / G->N[i + (size_t)i * n];
      }
    }
    return;
  }
  const Node *G00 = G->son(0, 0), *G01 = G->son(0, 1), *G11 = G->son(1, 1);
  double* X0 = X;
  double* X1 = X + (G11->roff - G->roff);
  solve_Rt(G00, X0, ldx, c);
  addevaltrans(-1.0, G01, X0, ldx, c, X1, ldx);
  solve_Rt(G11, X1, ldx, c);
}

// X(#t x c) <- R_tt^{-1} X (used by the preconditioner solve only).
void solve_R(const Node* G, double* X, int ldx, int c) {
  if (c == 0) return;
  if (G->kind == DENSE) {
    int n = G->rows;
    for (int col = 0; col < c; ++col) {
      double* x = X + (size_t)col * ldx;
      for (int i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (int p = i + 1; p < n; ++p) s -= G->N[i + (size_t)p * n] * x[p];
        x[i] = s / G->N[i + (size_t)i * n];
      }
    }
    return;
  }
  const Node *G00 = G->son(0, 0), *G01 = G->son(0, 1), *G11 = G->son(1, 1);
  double* X0 = X;
  double* X1 = X + (G11->roff - G->roff);
  solve_R(G11, X1, ldx, c);
  addeval(-1.0, G01, X1, ldx, c, X0, ldx);
  solve_R(G00, X0, ldx, c);
}

// Leaf cases of the block solves: G|_{t x r} <- L^{-1} G|_{t x r}, G R^{-1}.
void lsolve_leaf(const Node* L, Node* X) {
  if (X->kind == DENSE)
    solve_L(L, X->N.data(), X->rows, X->cols);
  else
    solve_L(L, X->rk.A.data(), X->rows, X->rk.k);
}

void rsolve_leaf(const Node* R, Node* X) {
  if (X->kind == DENSE) {
    // X R = B  <=>  R^* X^* = B^*
    int m = X->rows, n = X->cols;
    std::vector<double> Xt((size_t)n * m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < n; ++j) Xt[j + (size_t)i * n] = X->N[i + (size_t)j * m];
    solve_Rt(R, Xt.data(), n, m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < n; ++j) X->N[i + (size_t)j * m] = Xt[j + (size_t)i * n];
  } else {
    solve_Rt(R, X->rk.B.data(), X->cols, X->rk.k);
  }
}

void check_binary(const Node* G) {
  if (G->nt != 2 || G->ns != 2) throw std::runtime_error("H-LU needs a binary cluster tree");
}

// Standard H-LU: lu(t) = lu(t0); lsolve(t0,t1); rsolve(t1,t0);
// G11 <- G11 - G10 G01 (standard multiplication); lu(t1).
void lsolve_std(Ctx& cx, const CTree& T, const Node* L, Node* X);
void rsolve_std(Ctx& cx, const CTree& T, const Node* R, Node* X);

void lu_std(Ctx& cx, const CTree& T, Node* G) {
  if (G->kind == DENSE) {
    dense_lu(G->rows, G->N.data());
    cx.st.leaf_lu++;
    return;
  }
  check_binary(G);
  lu_std(cx, T, G->son(0, 0));
  lsolve_std(cx, T, G->son(0, 0), G->son(0, 1));
  rsolve_std(cx, T, G->son(0, 0), G->son(1, 0));
  mul_std(cx, T, -1.0, G->son(1, 0), G->son(0, 1), G->son(1, 1));
  lu_std(cx, T, G->son(1, 1));
}

void lsolve_std(Ctx& cx, const CTree& T, const Node* L, Node* X) {
  if (is_leaf(X)) {
    lsolve_leaf(L, X);
    return;
  }
  check_binary(L);
  for (int j = 0; j < X->ns; ++j) {
    lsolve_std(cx, T, L->son(0, 0), X->son(0, j));
    mul_std(cx, T, -1.0, L->son(1, 0), X->son(0, j), X->son(1, j));
    lsolve_std(cx, T, L->son(1, 1), X->son(1, j));
  }
}

void rsolve_std(Ctx& cx, const CTree& T, const Node* R, Node* X) {
  if (is_leaf(X)) {
    rsolve_leaf(R, X);
    return;
  }
  check_binary(R);
  for (int i = 0; i < X->nt; ++i) {
    rsolve_std(cx, T, R->son(0, 0), X->son(i, 0));
    mul_std(cx, T, -1.0, X->son(i, 0), R->son(0, 1), X->son(i, 1));
    rsolve_std(cx, T, R->son(1, 1), X->son(i, 1));
  }
}

// Accumulated H-LU: the pattern of Fig. invert applied to the block LR
// factorisation.  A block is flushed right before it is used; Schur
// complements are only added to accumulators.
void lsolve_acc(Ctx& cx, const CTree& T, const Node* L, Node* X, Acc& acc);
void rsolve_acc(Ctx& cx, const CTree& T, const Node* R, Node* X, Acc& acc);

void lu_acc(Ctx& cx, const CTree& T, Node* G, Acc& acc) {
  if (G->kind == DENSE) {
    flush(cx, T, acc, G);
    dense_lu(G->rows, G->N.data());
    cx.st.leaf_lu++;
    return;
  }
  check_binary(G);
  std::vector<Acc> a = split(cx, T, G->t, G->s, acc);
  acc.R.k = 0;
  acc.P.clear();
  lu_acc(cx, T, G->son(0, 0), a[0]);
  lsolve_acc(cx, T, G->son(0, 0), G->son(0, 1), a[1]);
  rsolve_acc(cx, T, G->son(0, 0), G->son(1, 0), a[2]);
  addproduct(cx, -1.0, G->son(1, 0), G->son(0, 1), a[3]);
  lu_acc(cx, T, G->son(1, 1), a[3]);
}

void lsolve_acc(Ctx& cx, const CTree& T, const Node* L, Node* X, Acc& acc) {
  if (is_leaf(X)) {
    flush(cx, T, acc, X);
    lsolve_leaf(L, X);
    return;
  }
  check_binary(L);
  std::vector<Acc> a = split(cx, T, X->t, X->s, acc);
  acc.R.k = 0;
  acc.P.clear();
  for (int j = 0; j < X->ns; ++j) {
    lsolve_acc(cx, T, L->son(0, 0), X->son(0, j), a[j]);
    addproduct(cx, -1.0, L->son(1, 0), X->son(0, j), a[X->ns + j]);
    lsolve_acc(cx, T, L->son(1, 1), X->son(1, j), a[X->ns + j]);
  }
}

void rsolve_acc(Ctx& cx, const CTree& T, const Node* R, Node* X, Acc& acc) {
  if (is_leaf(X)) {
    flush(cx, T, acc, X);
    rsolve_leaf(R, X);
    return;
  }
  check_binary(R);
  std::vector<Acc> a = split(cx, T, X->t, X->s, acc);
  acc.R.k = 0;
  acc.P.clear();
  for (int i = 0; i < X->nt; ++i) {
    rsolve_acc(cx, T, R->son(0, 0), X->son(i, 0), a[(size_t)i * X->ns]);
    addproduct(cx, -1.0, X->son(i, 0), R->son(0, 1), a[(size_t)i * X->ns + 1]);
    rsolve_acc(cx, T, R->son(1, 1), X->son(i, 1), a[(size_t)i * X->ns + 1]);
  }
}

// ------------------------------------------------------------------------
// H-Cholesky factorisation (reading R15)
// ------------------------------------------------------------------------
// Low-rank form of X|_{t x s} (Y|_{r x s})^* when X or Y is a leaf: the four
// branches of Fig. addproduct applied to Y^*, whose factors are those of Y
// exchanged (a dense Y^* is N_Y^*, a low-rank Y^* = B_Y A_Y^*).
LRProd lowrank_product_t(Ctx& cx, const Node* X, const Node* Y) {
  LRProd p;
  p.rows = X->rows;
  p.cols = Y->rows;
  int nt = X->rows, ns = X->cols, nr = Y->rows;
  cx.st.products++;
  if (X->kind == DENSE) {
    if (nt <= ns) {  // A = I, B = (X Y^*)^* = Y N_X^*
      p.k = nt;
      identity(p.A, nt);
      p.B.assign((size_t)nr * nt, 0.0);
      std::vector<double> NT((size_t)ns * nt);
      for (int i = 0; i < nt; ++i)
        for (int j = 0; j < ns; ++j) NT[j + (size_t)i * ns] = X->N[i + (size_t)j * nt];
      addeval(1.0, Y, NT.data(), ns, nt, p.B.data(), nr);
    } else {  // A = N_X, B = Y I
      p.k = ns;
      p.A = X->N;
      p.B.assign((size_t)nr * ns, 0.0);
      std::vector<double> I;
      identity(I, ns);
      addeval(1.0, Y, I.data(), ns, ns, p.B.data(), nr);
    }
  } else if (Y->kind == DENSE) {
    if (nr <= ns) {  // B = I, A = X N_Y^*
      p.k = nr;
      identity(p.B, nr);
      p.A.assign((size_t)nt * nr, 0.0);
      std::vector<double> NT((size_t)ns * nr);
      for (int i = 0; i < nr; ++i)
        for (int j = 0; j < ns; ++j) NT[j + (size_t)i * ns] = Y->N[i + (size_t)j * nr];
      addeval(1.0, X, NT.data(), ns, nr, p.A.data(), nt);
    } else {  // B = N_Y, A = X I
      p.k = ns;
      p.B = Y->N;
      p.A.assign((size_t)nt * ns, 0.0);
      std::vector<double> I;
      identity(I, ns);
      addeval(1.0, X, I.data(), ns, ns, p.A.data(), nt);
    }
  } else if (X->kind == RKLEAF) {  // A = A_X, B = Y B_X
    p.k = X->rk.k;
    p.A = X->rk.A;
    p.B.assign((size_t)nr * p.k, 0.0);
    addeval(1.0, Y, X->rk.B.data(), ns, p.k, p.B.data(), nr);
  } else {  // Y admissible leaf: A = X B_Y, B = A_Y
    p.k = Y->rk.k;
    p.B = Y->rk.A;
    p.A.assign((size_t)nt * p.k, 0.0);
    addeval(1.0, X, Y->rk.B.data(), ns, p.k, p.A.data(), nt);
  }
  return p;
}

// Z <- blocktrunc(Z + alpha X Y^*), standard algorithm.
void mul_t_std(Ctx& cx, const CTree& T, double alpha, const Node* X, const Node* Y, Node* Z) {
  if (is_leaf(X) || is_leaf(Y)) {
    LRProd p = lowrank_product_t(cx, X, Y);
    rkupdate(cx, alpha, p.k, p.A.data(), p.rows, p.B.data(), p.cols, Z);
    return;
  }
  bool temps = is_leaf(Z);
  if (temps) make_temps(T, Z);
  for (int i = 0; i < X->nt; ++i)
    for (int j = 0; j < Y->nt; ++j)
      for (int l = 0; l < X->ns; ++l) mul_t_std(cx, T, alpha, X->son(i, l), Y->son(j, l), Z->son(i, j));
  if (temps) merge_temps(cx, Z);
}

// rkupdate of a diagonal block Z = (t, t), lower blocks only.
void rkupdate_lower(Ctx& cx, double alpha, int k, const double* A, int lda, const double* B, int ldb, Node* Z) {
  if (k == 0) return;
  if (is_leaf(Z)) {
    rkupdate(cx, alpha, k, A, lda, B, ldb, Z);
    return;
  }
  for (int i = 0; i < Z->nt; ++i)
    for (int j = 0; j <= i; ++j) {
      Node* b = Z->son(i, j);
      const double* Ai = A + (b->roff - Z->roff);
      const double* Bj = B + (b->coff - Z->coff);
      if (i == j)
        rkupdate_lower(cx, alpha, k, Ai, lda, Bj, ldb, b);
      else
        rkupdate(cx, alpha, k, Ai, lda, Bj, ldb, b);
    }
}

// Z = (t, t) <- Z + alpha X X^* on the lower blocks, standard algorithm.
void symmul_std(Ctx& cx, const CTree& T, double alpha, const Node* X, Node* Z) {
  if (is_leaf(X)) {
    LRProd p = lowrank_product_t(cx, X, X);
    rkupdate_lower(cx, alpha, p.k, p.A.data(), p.rows, p.B.data(), p.cols, Z);
    return;
  }
  for (int i = 0; i < X->nt; ++i)
    for (int j = 0; j <= i; ++j)
      for (int l = 0; l < X->ns; ++l) {
        if (i == j)
          symmul_std(cx, T, alpha, X->son(i, l), Z->son(i, i));
        else
          mul_t_std(cx, T, alpha, X->son(i, l), X->son(j, l), Z->son(i, j));
      }
}

// Dense Cholesky of a leaf: L L^* with L in the lower triangle, zeros above.
void dense_chol(int n, double* N) {
  for (int k = 0; k < n; ++k) {
    double d = N[k + (size_t)k * n];
    for (int p = 0; p < k; ++p) d -= N[k + (size_t)p * n] * N[k + (size_t)p * n];
    if (!(d > 0.0)) throw std::runtime_error("leaf Cholesky: matrix not positive definite");
    const double l = std::sqrt(d);
    N[k + (size_t)k * n] = l;
    for (int i = k + 1; i < n; ++i) {
      double v = N[i + (size_t)k * n];
      for (int p = 0; p < k; ++p) v -= N[i + (size_t)p * n] * N[k + (size_t)p * n];
      N[i + (size_t)k * n] = v / l;
    }
  }
  for (int j = 1; j < n; ++j)
    for (int i = 0; i < j; ++i) N[i + (size_t)j * n] = 0.0;
}

// W (#t x c) <- L_tt^{-1} W with the lower Cholesky factor of (t, t).
void solve_Lc(const Node* L, double* W, int ldw, int c) {
  if (c == 0) return;
  if (L->kind == DENSE) {
    int n = L->rows;
    for (int col = 0; col < c; ++col) {
      double* w = W + (size_t)col * ldw;
      for (int i = 0; i < n; ++i) {
        double v = w[i];
        for (int p = 0; p < i; ++p) v -= L->N[i + (size_t)p * n] * w[p];
        w[i] = v / L->N[i + (size_t)i * n];
      }
    }
    return;
  }
  const Node *L00 = L->son(0, 0), *L10 = L->son(1, 0), *L11 = L->son(1, 1);
  double* W1 = W + (L11->roff - L->roff);
  solve_Lc(L00, W, ldw, c);
  addeval(-1.0, L10, W, ldw, c, W1, ldw);
  solve_Lc(L11, W1, ldw, c);
}

// Leaf X (r x t) <- X L_tt^{-*}: X^* <- L^{-1} X^* (dense), B <- L^{-1} B.
void rsolve_t_leaf(const Node* L, Node* X) {
  if (X->kind == DENSE) {
    int m = X->rows, n = X->cols;
    std::vector<double> Xt((size_t)n * m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < n; ++j) Xt[j + (size_t)i * n] = X->N[i + (size_t)j * m];
    solve_Lc(L, Xt.data(), n, m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < n; ++j) X->N[i + (size_t)j * m] = Xt[j + (size_t)i * n];
  } else {
    solve_Lc(L, X->rk.B.data(), X->cols, X->rk.k);
  }
}

// X (r x t) <- X L_tt^{-*}, standard.
void rsolve_t_std(Ctx& cx, const CTree& T, const Node* L, Node* X) {
  if (is_leaf(X)) {
    rsolve_t_leaf(L, X);
    return;
  }
  check_binary(L);
  for (int i = 0; i < X->nt; ++i) {
    rsolve_t_std(cx, T, L->son(0, 0), X->son(i, 0));
    mul_t_std(cx, T, -1.0, X->son(i, 0), L->son(1, 0), X->son(i, 1));
    rsolve_t_std(cx, T, L->son(1, 1), X->son(i, 1));
  }
}

void chol_std(Ctx& cx, const CTree& T, Node* G) {
  if (G->kind == DENSE) {
    dense_chol(G->rows, G->N.data());
    cx.st.leaf_lu++;
    return;
  }
  check_binary(G);
  chol_std(cx, T, G->son(0, 0));
  rsolve_t_std(cx, T, G->son(0, 0), G->son(1, 0));
  symmul_std(cx, T, -1.0, G->son(1, 0), G->son(1, 1));
  chol_std(cx, T, G->son(1, 1));
}

// addproduct for X Y^* (Fig. addproduct with Y^*).
void addproduct_t(Ctx& cx, double alpha, const Node* X, const Node* Y, Acc& acc) {
  cx.st.addproduct++;
  if (is_leaf(X) || is_leaf(Y)) {
    LRProd p = lowrank_product_t(cx, X, Y);
    rkadd(cx, KIND_ACCUM, alpha, p.k, p.A.data(), p.rows, p.B.data(), p.cols, acc.R);
  } else {
    acc.P.push_back({alpha, X, Y, true});
    cx.st.pending++;
  }
}

void rsolve_t_acc(Ctx& cx, const CTree& T, const Node* L, Node* X, Acc& acc) {
  if (is_leaf(X)) {
    flush(cx, T, acc, X);
    rsolve_t_leaf(L, X);
    return;
  }
  check_binary(L);
  std::vector<Acc> a = split(cx, T, X->t, X->s, acc);
  acc.R.k = 0;
  acc.P.clear();
  for (int i = 0; i < X->nt; ++i) {
    rsolve_t_acc(cx, T, L->son(0, 0), X->son(i, 0), a[(size_t)i * X->ns]);
    addproduct_t(cx, -1.0, X->son(i, 0), L->son(1, 0), a[(size_t)i * X->ns + 1]);
    rsolve_t_acc(cx, T, L->son(1, 1), X->son(i, 1), a[(size_t)i * X->ns + 1]);
  }
}

// Accumulated H-Cholesky: the accumulator of (t, t) holds the updates of the
// lower blocks of G|_{t x t} that are not yet applied.
void chol_acc(Ctx& cx, const CTree& T, Node* G, Acc& acc) {
  if (G->kind == DENSE) {
    flush(cx, T, acc, G);
    dense_chol(G->rows, G->N.data());
    cx.st.leaf_lu++;
    return;
  }
  check_binary(G);
  std::vector<Acc> a = split_lower(cx, T, G->t, acc);
  acc.R.k = 0;
  acc.P.clear();
  chol_acc(cx, T, G->son(0, 0), a[0]);
  rsolve_t_acc(cx, T, G->son(0, 0), G->son(1, 0), a[1]);
  addproduct_t(cx, -1.0, G->son(1, 0), G->son(1, 0), a[2]);
  chol_acc(cx, T, G->son(1, 1), a[2]);
}

// ------------------------------------------------------------------------
// H-matrix inversion (Sect. 6, the six steps and Fig. invert; reading R14)
// ------------------------------------------------------------------------
// Dense inverse of a leaf in place: unpivoted LU, then the columns of
// (L U)^{-1} by forward and backward substitution with the unit vectors.
void dense_inverse(int n, double* N) {
  std::vector<double> F(N, N + (size_t)n * n);
  dense_lu(n, F.data());
  for (int c = 0; c < n; ++c) {
    std::vector<double> x(n, 0.0);
    x[c] = 1.0;
    for (int i = 0; i < n; ++i)
      for (int p = 0; p < i; ++p) x[i] -= F[i + (size_t)p * n] * x[p];
    for (int i = n - 1; i >= 0; --i) {
      for (int p = i + 1; p < n; ++p) x[i] -= F[i + (size_t)p * n] * x[p];
      x[i] /= F[i + (size_t)i * n];
    }
    for (int i = 0; i < n; ++i) N[i + (size_t)c * n] = x[i];
  }
}

// Zero matrix with the block structure of b (the auxiliary H12, H21).
Node* zero_like(const Node* b) {
  Node* z = clone(b);
  zero_node(z);
  return z;
}

// Standard inversion: G|_{t x t} <- its inverse, every product by the
// standard multiplication.
void inv_std(Ctx& cx, const CTree& T, Node* G) {
  if (G->kind == DENSE) {
    dense_inverse(G->rows, G->N.data());
    cx.st.leaf_lu++;
    return;
  }
  check_binary(G);
  Node *G11 = G->son(0, 0), *G12 = G->son(0, 1), *G21 = G->son(1, 0), *G22 = G->son(1, 1);
  inv_std(cx, T, G11);                            // 1. G11 <- G11^{-1}
  std::unique_ptr<Node> H12(zero_like(G12)), H21(zero_like(G21));
  mul_std(cx, T, 1.0, G11, G12, H12.get());       // 2. H12 = G11^{-1} G12
  mul_std(cx, T, 1.0, G21, G11, H21.get());       //    H21 = G21 G11^{-1}
  mul_std(cx, T, -1.0, H21.get(), G12, G22);      // 3. S = G22 - H21 G12
  inv_std(cx, T, G22);                            // 4. G22 <- S^{-1}
  zero_node(G12);                                 // 5. G12 = -H12 S^{-1}
  mul_std(cx, T, -1.0, H12.get(), G22, G12);
  zero_node(G21);                                 //    G21 = -S^{-1} H21
  mul_std(cx, T, -1.0, G22, H21.get(), G21);
  mul_std(cx, T, -1.0, H12.get(), G21, G11);      // 6. G11 = G11^{-1} - H12 G21
}

// Accumulated inversion (Fig. invert): acc holds the updates not yet applied
// to G|_{t x t}.
void inv_acc(Ctx& cx, const CTree& T, Node* G, Acc& acc) {
  if (G->kind == DENSE) {
    flush(cx, T, acc, G);
    dense_inverse(G->rows, G->N.data());
    cx.st.leaf_lu++;
    return;
  }
  check_binary(G);
  Node *G11 = G->son(0, 0), *G12 = G->son(0, 1), *G21 = G->son(1, 0), *G22 = G->son(1, 1);
  std::vector<Acc> a = split(cx, T, G->t, G->s, acc);
  acc.R.k = 0;
  acc.P.clear();
  Acc &a11 = a[0], &a12 = a[1], &a21 = a[2], &a22 = a[3];
  inv_acc(cx, T, G11, a11);
  flush(cx, T, a12, G12);
  flush(cx, T, a21, G21);
  std::unique_ptr<Node> H12(zero_like(G12)), H21(zero_like(G21));
  addproduct(cx, 1.0, G11, G12, a12);
  flush(cx, T, a12, H12.get());
  addproduct(cx, 1.0, G21, G11, a21);
  flush(cx, T, a21, H21.get());
  addproduct(cx, -1.0, H21.get(), G12, a22);
  inv_acc(cx, T, G22, a22);
  zero_node(G12);
  zero_node(G21);
  addproduct(cx, -1.0, H12.get(), G22, a12);
  flush(cx, T, a12, G12);
  addproduct(cx, -1.0, G22, H21.get(), a21);
  flush(cx, T, a21, G21);
  addproduct(cx, -1.0, H12.get(), G21, a11);
  flush(cx, T, a11, G11);
}

// ------------------------------------------------------------------------
// Boundary-element entries on flat triangles (reading R17)
// ------------------------------------------------------------------------
struct Tri {
  double v[3][3];
};

// The 7-point rule of degree 5 on a triangle (Radon): barycentric points and
// weights relative to the area.
void radon7(const Tri& T, double pts[7][3], double w[7]) {
  const double r15 = std::sqrt(15.0);
  const double b1 = (6.0 + r15) / 21.0, a1 = 1.0 - 2.0 * b1;
  const double b2 = (6.0 - r15) / 21.0, a2 = 1.0 - 2.0 * b2;
  const double w1 = (155.0 + r15) / 1200.0, w2 = (155.0 - r15) / 1200.0;
  const double bary[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {a1, b1, b1}, {b1, a1, b1}, {b1, b1, a1},
                             {a2, b2, b2}, {b2, a2, b2}, {b2, b2, a2}};
  const double ww[7] = {0.225, w1, w1, w1, w2, w2, w2};
  for (int q = 0; q < 7; ++q) {
    for (int d = 0; d < 3; ++d)
      pts[q][d] = bary[q][0] * T.v[0][d] + bary[q][1] * T.v[1][d] + bary[q][2] * T.v[2][d];
    w[q] = ww[q];
  }
}

void sub3(const double* a, const double* b, double* c) {
  for (int d = 0; d < 3; ++d) c[d] = a[d] - b[d];
}
double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// Area and unit normal ((v1 - v0) x (v2 - v0) direction).
double tri_area(const Tri& T, double* nrm) {
  double e1[3], e2[3], c[3];
  sub3(T.v[1], T.v[0], e1);
  sub3(T.v[2], T.v[0], e2);
  cross3(e1, e2, c);
  const double len = std::sqrt(dot3(c, c));
  if (nrm)
    for (int d = 0; d < 3; ++d) nrm[d] = c[d] / len;
  return 0.5 * len;
}

// int_T 1/|x - y| dy for x in the plane of T: the sum over the edges of
// h_e log((r_b + s_b) / (r_a + s_a)), where the edge runs from a to b, s is
// the coordinate along it measured from the foot of x, r the distance to x,
// and h_e the distance of x from the edge's line (positive inside).
double inv_dist_integral(const Tri& T, const double* x) {
  double nrm[3];
  tri_area(T, nrm);
  double sum = 0.0;
  for (int e = 0; e < 3; ++e) {
    const double* a = T.v[e];
    const double* b = T.v[(e + 1) % 3];
    double ab[3], u[3], nu[3], xa[3], xb[3];
    sub3(b, a, ab);
    const double len = std::sqrt(dot3(ab, ab));
    for (int d = 0; d < 3; ++d) u[d] = ab[d] / len;
    cross3(u, nrm, nu);  // in the plane, pointing out of the triangle (counterclockwise edges)
    sub3(a, x, xa);
    sub3(b, x, xb);
    const double h = dot3(xa, nu);  // distance of x from the edge line, positive inside
    const double sa = dot3(xa, u), sb = dot3(xb, u);
    const double ra = std::sqrt(dot3(xa, xa)), rb = std::sqrt(dot3(xb, xb));
    if (std::fabs(h) > 0.0) sum += h * std::log((rb + sb) / (ra + sa));
  }
  return sum;
}

// Galerkin entry (i, j) of the single layer (kind 2) or of 1/2 M + double
// layer (kind 3).
double bem_entry(int kind, const Tri& Ti, const Tri& Tj, bool same) {
  const double pi4 = 4.0 * M_PI;
  double pi[7][3], pj[7][3], wi[7], wj[7], nj[3];
  radon7(Ti, pi, wi);
  radon7(Tj, pj, wj);
  const double ai = tri_area(Ti, nullptr), aj = tri_area(Tj, nj);
  if (same) {
    if (kind == 3) return 0.5 * ai;
    double s = 0.0;
    for (int a = 0; a < 7; ++a) s += wi[a] * inv_dist_integral(Tj, pi[a]);
    return ai * s / pi4;
  }
  double s = 0.0;
  for (int a = 0; a < 7; ++a)
    for (int b = 0; b < 7; ++b) {
      double r[3];
      sub3(pj[b], pi[a], r);  // y - x
      const double d2 = dot3(r, r), d = std::sqrt(d2);
      const double k = kind == 2 ? 1.0 / d : dot3(r, nj) / (d2 * d);
      s += wi[a] * wj[b] * k;
    }
  return ai * aj * s / pi4;
}

// ------------------------------------------------------------------------
// H-matrix object, assembly and export
// ------------------------------------------------------------------------
struct HM {
  std::shared_ptr<CTree> T;
  Node* root = nullptr;
  ~HM() { delete root; }
};

void collect(const Node* b, std::vector<const Node*>& out) {
  out.push_back(b);
  for (const Node* s : b->sons) collect(s, out);
}

void to_dense_rec(const Node* b, double* D, int ld) {
  if (b->kind == DENSE) {
    for (int c = 0; c < b->cols; ++c)
      for (int r = 0; r < b->rows; ++r) D[(b->roff + r) + (size_t)(b->coff + c) * ld] = b->N[r + (size_t)c * b->rows];
  } else if (b->kind == RKLEAF) {
    for (int c = 0; c < b->cols; ++c)
      for (int r = 0; r < b->rows; ++r) {
        double s = 0;
        for (int q = 0; q < b->rk.k; ++q)
          s += b->rk.A[r + (size_t)q * b->rows] * b->rk.B[c + (size_t)q * b->cols];
        D[(b->roff + r) + (size_t)(b->coff + c) * ld] = s;
      }
  } else {
    for (const Node* s : b->sons) to_dense_rec(s, D, ld);
  }
}

thread_local std::string g_err;
Stats g_last_stats;
std::vector<LogRec> g_last_log;
bool g_log_enabled = false;

}  // namespace

// ------------------------------------------------------------------------
// C ABI (test infrastructure)
// ------------------------------------------------------------------------
extern "C" {

const char* or_last_error() { return g_err.c_str(); }

void or_set_log(int enable) { g_log_enabled = enable != 0; }

// Build an H-matrix for points x (n x dim, row-major).  The matrix entries come
// from a CSR matrix given in the original index order (kind 0), from the
// kernel 1/|x - y| with the given diagonal value (kind 1), or from the
// Galerkin single layer (kind 2) or double layer plus half the mass matrix
// (kind 3) on the triangles in vals (n x 9: three vertices each, reading R17;
// x holds the clustering points).  Admissible blocks of kinds 1-3 are
// compressed by the truncated SVD at build_eps.  Returns NULL on error.
void* or_build(int dim, int n, const double* x, int leaf, double eta, int kind,
               const int64_t* rowptr, const int32_t* colind, const double* vals,
               double diag_value, double build_eps) {
  try {
    if (dim < 1 || dim > 3 || n < 1 || leaf < 1) throw std::runtime_error("bad arguments");
    auto T = std::make_shared<CTree>();
    T->dim = dim;
    T->perm.resize(n);
    for (int i = 0; i < n; ++i) T->perm[i] = i;
    build_cluster(*T, x, 0, n, 0, leaf);
    HM* h = new HM;
    h->T = T;
    h->root = build_block(*T, 0, 0, eta);
    std::vector<int> inv(n);
    for (int i = 0; i < n; ++i) inv[T->perm[i]] = i;
    std::vector<const Node*> all;
    collect(h->root, all);
    if (kind == 0) {
      // Sparse input.  Inadmissible leaves are filled densely.  An admissible
      // leaf is exactly zero for stencils on clusters that are not too small
      // (local rank zero, Sect. 3); if it holds entries anyway it is stored
      // exactly as A = its nonzero columns (in increasing order), B = the
      // matching unit vectors.
      for (const Node* cb : all) {
        Node* b = const_cast<Node*>(cb);
        if (b->kind == NONLEAF) continue;
        std::vector<std::pair<int, std::pair<int, double>>> nz;  // (col, (row, val))
        for (int r = 0; r < b->rows; ++r) {
          int gi = T->perm[b->roff + r];
          for (int64_t e = rowptr[gi]; e < rowptr[gi + 1]; ++e) {
            int pj = inv[colind[e]];
            if (pj < b->coff || pj >= b->coff + b->cols) continue;
            if (b->kind == DENSE)
              b->N[r + (size_t)(pj - b->coff) * b->rows] += vals[e];
            else if (vals[e] != 0.0)
              nz.push_back({pj - b->coff, {r, vals[e]}});
          }
        }
        if (b->kind == RKLEAF && !nz.empty()) {
          std::vector<int> cols;
          for (auto& q : nz) cols.push_back(q.first);
          std::sort(cols.begin(), cols.end());
          cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
          int k = (int)cols.size();
          b->rk.k = k;
          b->rk.A.assign((size_t)b->rows * k, 0.0);
          b->rk.B.assign((size_t)b->cols * k, 0.0);
          for (int q = 0; q < k; ++q) b->rk.B[cols[q] + (size_t)q * b->cols] = 1.0;
          for (auto& q : nz) {
            int c = (int)(std::lower_bound(cols.begin(), cols.end(), q.first) - cols.begin());
            b->rk.A[q.second.first + (size_t)c * b->rows] += q.second.second;
          }
        }
      }
    } else {
      Ctx cx;
      cx.eps = build_eps;
      for (const Node* cb : all) {
        Node* b = const_cast<Node*>(cb);
        if (b->kind == NONLEAF) continue;
        std::vector<double> D((size_t)b->rows * b->cols);
        for (int c = 0; c < b->cols; ++c)
          for (int r = 0; r < b->rows; ++r) {
            int gi = T->perm[b->roff + r], gj = T->perm[b->coff + c];
            double v;
            if (kind >= 2) {
              Tri ti, tj;
              std::memcpy(ti.v, vals + (size_t)gi * 9, sizeof(ti.v));
              std::memcpy(tj.v, vals + (size_t)gj * 9, sizeof(tj.v));
              v = bem_entry(kind, ti, tj, gi == gj);
            } else if (gi == gj) {
              v = diag_value;
            } else {
              double d2 = 0;
              for (int d = 0; d < dim; ++d) {
                double g = x[(size_t)gi * dim + d] - x[(size_t)gj * dim + d];
                d2 += g * g;
              }
              v = 1.0 / std::sqrt(d2);
            }
            D[r + (size_t)c * b->rows] = v;
          }
        if (b->kind == DENSE) {
          b->N = D;
        } else {
          std::vector<double> U, sigma, V;
          thin_svd(b->rows, b->cols, D.data(), b->rows, U, sigma, V);
          int k = choose_rank(sigma, build_eps, nullptr, nullptr);
          b->rk.k = k;
          b->rk.A.assign(U.begin(), U.begin() + (size_t)b->rows * k);
          b->rk.B.assign((size_t)b->cols * k, 0.0);
          for (int c = 0; c < k; ++c)
            for (int r = 0; r < b->cols; ++r) b->rk.B[r + (size_t)c * b->cols] = V[r + (size_t)c * b->cols] * sigma[c];
        }
      }
    }
    return h;
  } catch (std::exception& e) {
    g_err = e.what();
    return nullptr;
  }
}

void or_free(void* h) { delete (HM*)h; }

void* or_clone(void* h) {
  HM* a = (HM*)h;
  HM* b = new HM;
  b->T = a->T;
  b->root = clone(a->root);
  return b;
}

// Same structure, all leaves zero (dense zeros, rank 0).
void* or_zeros_like(void* h) {
  HM* b = (HM*)or_clone(h);
  zero_node(b->root);
  return b;
}

int or_n(void* h) { return (int)((HM*)h)->T->perm.size(); }

void or_perm(void* h, int32_t* perm) {
  HM* a = (HM*)h;
  for (size_t i = 0; i < a->T->perm.size(); ++i) perm[i] = a->T->perm[i];
}

int or_num_clusters(void* h) { return (int)((HM*)h)->T->c.size(); }

// Clusters in creation (pre-order) order.
void or_clusters(void* h, int32_t* off, int32_t* size, int32_t* level, int32_t* son0, int32_t* son1) {
  HM* a = (HM*)h;
  for (size_t i = 0; i < a->T->c.size(); ++i) {
    const Cluster& c = a->T->c[i];
    off[i] = c.off;
    size[i] = c.size;
    level[i] = c.level;
    son0[i] = c.son[0];
    son1[i] = c.son[1];
  }
}

int or_num_blocks(void* h) {
  std::vector<const Node*> all;
  collect(((HM*)h)->root, all);
  return (int)all.size();
}

// All blocks in depth-first pre-order: row cluster, column cluster, kind
// (0 non-leaf, 1 admissible, 2 inadmissible), rank (admissible leaves) and the
// index of the parent block (-1 for the root).
void or_blocks(void* h, int32_t* t, int32_t* s, int32_t* kind, int32_t* rank, int32_t* parent) {
  std::vector<const Node*> all;
  collect(((HM*)h)->root, all);
  for (size_t i = 0; i < all.size(); ++i) {
    t[i] = all[i]->t;
    s[i] = all[i]->s;
    kind[i] = all[i]->kind;
    rank[i] = all[i]->kind == RKLEAF ? all[i]->rk.k : -1;
    parent[i] = -1;
  }
  std::unordered_map<const Node*, int32_t> index;
  for (size_t i = 0; i < all.size(); ++i) index[all[i]] = (int32_t)i;
  for (size_t i = 0; i < all.size(); ++i)
    for (const Node* c : all[i]->sons) parent[index[c]] = (int32_t)i;
}

// Dense n x n matrix in cluster (permuted) order, column-major.
void or_to_dense(void* h, double* out) {
  HM* a = (HM*)h;
  int n = (int)a->T->perm.size();
  std::fill(out, out + (size_t)n * n, 0.0);
  to_dense_rec(a->root, out, n);
}

static void store_stats(const Ctx& cx, int64_t* stats) {
  g_last_stats = cx.st;
  g_last_log = cx.logv;
  if (!stats) return;
  const Stats& s = cx.st;
  int64_t v[10] = {s.trunc_update, s.trunc_accum, s.trunc_merge, s.dense_updates, s.addproduct,
                   s.pending, s.products, s.leaf_lu, s.merges, s.trunc_flops};
  for (int i = 0; i < 10; ++i) stats[i] = v[i];
}

// Z <- blocktrunc(Z + alpha X Y); mode 0 standard, 1 accumulated.
int or_addmul(double alpha, void* X, void* Y, void* Z, double eps, int mode, int64_t* stats) {
  try {
    Ctx cx;
    cx.eps = eps;
    cx.log = g_log_enabled;
    cx.fused = mode == 2;
    HM *x = (HM*)X, *y = (HM*)Y, *z = (HM*)Z;
    if (mode == 0)
      mul_std(cx, *z->T, alpha, x->root, y->root, z->root);
    else
      mul_acc(cx, *z->T, alpha, x->root, y->root, z->root);
    store_stats(cx, stats);
    return 0;
  } catch (std::exception& e) {
    g_err = e.what();
    return 1;
  }
}

// In-place H-LU; mode 0 standard, 1 accumulated.
int or_lu(void* G, double eps, int mode, int64_t* stats) {
  try {
    Ctx cx;
    cx.eps = eps;
    cx.log = g_log_enabled;
    cx.fused = mode == 2;
    HM* g = (HM*)G;
    if (mode == 0) {
      lu_std(cx, *g->T, g->root);
    } else {
      Acc acc = empty_acc(g->root->rows, g->root->cols);
      lu_acc(cx, *g->T, g->root, acc);
    }
    store_stats(cx, stats);
    return 0;
  } catch (std::exception& e) {
    g_err = e.what();
    return 1;
  }
}

// In-place H-Cholesky G = L L^* (reading R15); mode 0 standard, 1 accumulated.
int or_chol(void* G, double eps, int mode, int64_t* stats) {
  try {
    Ctx cx;
    cx.eps = eps;
    cx.log = g_log_enabled;
    cx.fused = mode == 2;
    HM* g = (HM*)G;
    if (mode == 0) {
      chol_std(cx, *g->T, g->root);
    } else {
      Acc acc = empty_acc(g->root->rows, g->root->cols);
      chol_acc(cx, *g->T, g->root, acc);
    }
    store_stats(cx, stats);
    return 0;
  } catch (std::exception& e) {
    g_err = e.what();
    return 1;
  }
}

// In-place H-inversion; mode 0 standard, 1 accumulated.
int or_inv(void* G, double eps, int mode, int64_t* stats) {
  try {
    Ctx cx;
    cx.eps = eps;
    cx.log = g_log_enabled;
    cx.fused = mode == 2;
    HM* g = (HM*)G;
    if (mode == 0) {
      inv_std(cx, *g->T, g->root);
    } else {
      Acc acc = empty_acc(g->root->rows, g->root->cols);
      inv_acc(cx, *g->T, g->root, acc);
    }
    store_stats(cx, stats);
    return 0;
  } catch (std::exception& e) {
    g_err = e.what();
    return 1;
  }
}

// In-place H-LU of the leading diagonal block at the given depth of the
// block tree (G restricted to the first cluster of that level), used to time
// a bounded sample of a large factorisation.  Returns the block size.
int or_lu_sub(void* G, int depth, double eps, int mode, int64_t* stats) {
  try {
    HM* g = (HM*)G;
    Node* b = g->root;
    for (int d = 0; d < depth && b->kind == NONLEAF; ++d) b = b->son(0, 0);
    Ctx cx;
    cx.eps = eps;
    cx.fused = mode == 2;
    if (mode == 0) {
      lu_std(cx, *g->T, b);
    } else {
      Acc acc = empty_acc(b->rows, b->cols);
      lu_acc(cx, *g->T, b, acc);
    }
    store_stats(cx, stats);
    return b->rows;
  } catch (std::exception& e) {
    g_err = e.what();
    return -1;
  }
}

// x <- (L R)^{-1} x, x given in cluster (permuted) order.
void or_lu_solve(void* G, double* x, int c) {
  HM* g = (HM*)G;
  int n = (int)g->T->perm.size();
  solve_L(g->root, x, n, c);
  solve_R(g->root, x, n, c);
}

// y += alpha G x (cluster order), x and y are n x c column-major.
void or_matvec(void* G, double alpha, const double* x, double* y, int c) {
  HM* g = (HM*)G;
  int n = (int)g->T->perm.size();
  addeval(alpha, g->root, x, n, c, y, n);
}

// Y(#t x c) += alpha G|_{t x s} W for the block with pre-order index b.
int or_addeval_block(void* G, int b, int trans, double alpha, const double* W, double* Y, int c) {
  std::vector<const Node*> all;
  collect(((HM*)G)->root, all);
  if (b < 0 || b >= (int)all.size()) return 1;
  const Node* nd = all[b];
  if (!trans)
    addeval(alpha, nd, W, nd->cols, c, Y, nd->rows);
  else
    addevaltrans(alpha, nd, W, nd->rows, c, Y, nd->cols);
  return 0;
}

// Truncated addition on raw factors: (C, D) <- trunc_eps(C D^* + alpha A B^*).
// A m x k1, B n x k1, C m x k2, D n x k2 (column-major).  Outputs Cout (m x k),
// Dout (n x k) with capacity min(m, n, k1 + k2) columns; returns k.
// sigma receives the min(m, min(n, k1 + k2)) singular values of the sum.
int or_rkadd(int m, int n, int k1, int k2, double alpha, const double* A, const double* B,
             const double* C, const double* D, double eps, double* Cout, double* Dout, double* sigma) {
  Ctx cx;
  cx.eps = eps;
  cx.log = g_log_enabled;
  RK r;
  r.rows = m;
  r.cols = n;
  r.k = k2;
  r.A.assign(C, C + (size_t)m * k2);
  r.B.assign(D, D + (size_t)n * k2);
  std::vector<double> sg;
  rkadd(cx, KIND_RAW, alpha, k1, A, m, B, n, r, &sg);
  if (k1 == 0) sg.clear();
  for (size_t i = 0; i < sg.size(); ++i) sigma[i] = sg[i];
  std::copy(r.A.begin(), r.A.end(), Cout);
  std::copy(r.B.begin(), r.B.end(), Dout);
  g_last_log = cx.logv;
  return r.k;
}

// Stacked truncated addition (R16): (C, D) <- trunc_eps(C D^* + sum_q
// alpha_q A_q B_q^*) for g updates (A_q m x k_q, B_q n x k_q, column-major);
// outputs as or_rkadd.  Returns k.
int or_rkadd_multi(int m, int n, int g, const int32_t* ks, const double* alphas, const double* const* A,
                   const double* const* B, int k2, const double* C, const double* D, double eps, double* Cout,
                   double* Dout) {
  Ctx cx;
  cx.eps = eps;
  RK r;
  r.rows = m;
  r.cols = n;
  r.k = k2;
  r.A.assign(C, C + (size_t)m * k2);
  r.B.assign(D, D + (size_t)n * k2);
  std::vector<Upd> u;
  for (int q = 0; q < g; ++q) u.push_back({alphas[q], ks[q], A[q], m, B[q], n});
  rkadd_multi(cx, KIND_RAW, u, r);
  std::copy(r.A.begin(), r.A.end(), Cout);
  std::copy(r.B.begin(), r.B.end(), Dout);
  return r.k;
}

// 2 x 2 rkmerge of low-rank pieces R_ij = A_ij B_ij^* (row splits m0, m1 and
// column splits n0, n1; pieces given row-major, each with its own rank).
int or_rkmerge22(int m0, int m1, int n0, int n1, const int32_t* k, const double* const* A,
                 const double* const* B, double eps, double* Aout, double* Bout) {
  Ctx cx;
  cx.eps = eps;
  int ms[2] = {m0, m1}, ns[2] = {n0, n1};
  std::vector<RK> g(4);
  std::vector<const RK*> ptr(4);
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      RK& r = g[i * 2 + j];
      r.rows = ms[i];
      r.cols = ns[j];
      r.k = k[i * 2 + j];
      r.A.assign(A[i * 2 + j], A[i * 2 + j] + (size_t)r.rows * r.k);
      r.B.assign(B[i * 2 + j], B[i * 2 + j] + (size_t)r.cols * r.k);
      ptr[i * 2 + j] = &r;
    }
  RK out = rkmerge(cx, ptr, 2, 2);
  std::copy(out.A.begin(), out.A.end(), Aout);
  std::copy(out.B.begin(), out.B.end(), Bout);
  return out.k;
}

// Galerkin boundary-element entry (kind 2 single layer, 3 double layer plus
// half the mass matrix) of two triangles (9 doubles each); same: i == j.
double or_bem_entry(int kind, const double* ti, const double* tj, int same) {
  Tri a, b;
  std::memcpy(a.v, ti, sizeof(a.v));
  std::memcpy(b.v, tj, sizeof(b.v));
  return bem_entry(kind, a, b, same != 0);
}

// int_T 1/|x - y| dy for x in the plane of the triangle T (9 doubles).
double or_inv_dist_integral(const double* t, const double* x) {
  Tri a;
  std::memcpy(a.v, t, sizeof(a.v));
  return inv_dist_integral(a, x);
}

// Thin SVD of an m x n matrix (for pinning against LAPACK).
void or_svd(int m, int n, const double* M, double* U, double* S, double* V) {
  std::vector<double> u, s, v;
  thin_svd(m, n, M, m, u, s, v);
  std::copy(u.begin(), u.end(), U);
  std::copy(s.begin(), s.end(), S);
  std::copy(v.begin(), v.end(), V);
}

// Householder QR: R (min(m,n) x n) and explicit Q (m x min(m,n)).
void or_qr(int m, int n, const double* M, double* Q, double* R) {
  int q = std::min(m, n);
  std::vector<double> W(M, M + (size_t)m * n), tau(q);
  house_qr(m, n, W.data(), m, tau.data());
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < q; ++i) R[i + (size_t)j * q] = (i <= j) ? W[i + (size_t)j * m] : 0.0;
  std::vector<double> E((size_t)m * q, 0.0);
  for (int i = 0; i < q; ++i) E[i + (size_t)i * m] = 1.0;
  apply_q(m, q, W.data(), m, tau.data(), E.data(), m, q);
  std::copy(E.begin(), E.end(), Q);
}

// Statistics of the last or_addmul / or_lu call (10 counters, see Stats).
void or_last_stats(int64_t* out) {
  const Stats& s = g_last_stats;
  int64_t v[10] = {s.trunc_update, s.trunc_accum, s.trunc_merge, s.dense_updates, s.addproduct,
                   s.pending, s.products, s.leaf_lu, s.merges, s.trunc_flops};
  for (int i = 0; i < 10; ++i) out[i] = v[i];
}

int or_log_size() { return (int)g_last_log.size(); }

// Truncation log: per record kind, m, n, k1, k2, k and the two rank margins.
void or_log(int32_t* ints, double* margins) {
  for (size_t i = 0; i < g_last_log.size(); ++i) {
    const LogRec& r = g_last_log[i];
    int32_t v[6] = {r.kind, r.m, r.n, r.k1, r.k2, r.k};
    for (int j = 0; j < 6; ++j) ints[i * 6 + j] = v[j];
    margins[i * 2] = r.margin_k;
    margins[i * 2 + 1] = r.margin_km1;
  }
}

}  // extern "C"
