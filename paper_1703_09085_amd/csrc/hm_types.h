// Device work descriptors shared by the host scheduler and the gfx950 kernels.
//
// Every H-matrix operation is lowered to batches of five primitive work items:
//   GEMM  - C = beta C + sum_j alpha_j op(A_j) op(B_j)      (H x thin-dense, dense updates)
//   TRUNC - truncated sum of low-rank terms                  (rkadd, rowmerge, rkmerge stages)
//   LU    - dense unpivoted LU of a leaf block
//   TRSM  - triangular solve with a dense leaf factor
//   COPY  - copy / fill of a sub-block, optionally with a rank word
// Matrix dimensions that are ranks decided on the device are "DDim"s: a static
// capacity and an optional pointer to the device int that holds the current
// value, so the host never waits for a rank.
#pragma once
#include "mlp.h"
#include <cstddef>
#include <cstdint>
#include <cstdlib>

namespace hm {

struct DDim {
  int stat;        // capacity (and the value when dyn is null)
  int pad;
  const int* dyn;  // device rank word or nullptr
};

enum Op : int { OP_GEMM = 0, OP_TRUNC = 1, OP_LU = 2, OP_TRSM = 3, OP_COPY = 4, OP_COUNT = 5 };

// One product term of a GEMM work item.
struct DGemmTerm {
  const double* A;
  const double* B;
  double alpha;
  int lda, ldb;
  int ta, tb;  // op(X) = X^T when set
  DDim k;
};

// Output tile [row0, row0 + 64) x [col0, col0 + 64) of C (m x n).
struct DGemm {
  double* C;
  DDim m, n;
  int ldc;
  int ctrans;  // C(i,j) stored at C[j + i*ldc]
  int beta;    // 0: overwrite, 1: accumulate
  int pad;
  int term0, nterms;
  int row0, col0;
};

// One low-rank term alpha A B^T of a truncation, placed at rows
// [row_off, row_off + rows) and columns [col_off, col_off + cols) of the m x n
// block (zero elsewhere).  A is rows x k (lda), B is cols x k (ldb).
struct DTruncPart {
  const double* A;
  const double* B;
  double alpha;
  int lda, ldb;
  int ta, tb;  // A(i,c) = A[c + i*lda] when ta (likewise B)
  int row_off, rows, col_off, cols;
  DDim k;
};

enum TruncFlags : int {
  TRUNC_SKIP_IF_PART0_EMPTY = 1,  // an update with zero columns is a no-op
  // every truncation kernel is launched on the item and takes it only when
  // it belongs to its size class (descriptors made on the device, whose sizes
  // the host does not know)
  TRUNC_CLASS_CHECK = 2,
  // several updates truncated with the target in one item (the last part is
  // the target): a no-op when every update has zero columns
  TRUNC_SKIP_IF_HEAD_EMPTY = 4,
};

// Truncation of sum_p parts into (C, D) with C m x k (ldc), D n x k (ldd),
// k <= cap written to *rank.  Workspace: (m + n) * lmax doubles at ws_off.
// Truncations of blocks with m, n <= TRUNC_SMALL_MAX run in the dense-core
// kernel (one 256-thread workgroup per item); larger ones in the general kernel.
constexpr int TRUNC_SMALL_MAX = 64;

// Blocks of at most 32 x 32 run one per wavefront inside the small-block
// launch; HM_TINY=0 (host environment) sends them through the block-wide path.
constexpr int TRUNC_TINY_MAX = 32;
inline bool tiny_path_enabled() {
  const char* e = std::getenv("HM_TINY");
  return !(e && e[0] == '0');
}
inline bool trunc_is_tiny(int m, int n) { return m <= TRUNC_TINY_MAX && n <= TRUNC_TINY_MAX; }
// The one-wave path for larger blocks of stacked rank <= 16 (HM_THIN=0 turns
// it off; the register-resident and general kernels then take its items).
inline bool thin_path_enabled() {
  const char* e = std::getenv("HM_THIN");
  return !(e && e[0] == '0');
}

struct DTrunc {
  double* C;
  double* D;
  int* rank;
  int m, n, ldc, ldd;
  int cap;
  int part0, nparts;
  int lmax;  // sum of part capacities
  int flags;
  int log_idx;  // position in the optional size log
  int level;    // level of the target block's row cluster (a feature of the rank predictor)
  int kfix;     // >= 0: the rank to keep instead of the rank rule's choice (test hook); -1: the rule
};

// Rank predictor attached to a plan (device memory).  The features of a
// small-block truncation (m, n <= 64): level, log2 m, log2 n, log2(1 + l) and
// log10 of the four singular values of the sketch K omega(:, 0:4) relative to
// |K|_F.  In predict mode the network's rank estimate k^ sets the width
// w = k^ + oversample at which the pivoted QR of the exact path first stops;
// the result of that w-column core is kept when the exact residual meets the
// rank rule's bound, else the QR continues to the exact path.
struct DPredictor {
  MlpWeights w;
  const double* omega;  // 64 x 32 column-major (the first 4 columns are read), supplied by the caller
  int oversample;
  int mode;  // 0: compute and log the features only; 1: predict
};

enum LeafKind : int {
  LEAF_LU = 0,        // unpivoted LU in place: L unit lower, R upper
  LEAF_INVERSE = 1,   // the inverse in place (unpivoted Gauss-Jordan)
  LEAF_CHOLESKY = 2,  // L L^T in place: L in the lower triangle, zeros above
};

// Dense factorisation or inversion of a leaf block (n x n, n <= 64).
struct DLu {
  double* N;
  int n, ld;
  int kind;  // LeafKind
  int pad;
};

enum TrsmKind : int {
  TRSM_L_UNIT = 0,  // X <- L^{-1} X, L unit lower (strict lower part of the leaf)
  TRSM_RT = 1,      // X <- R^{-T} X, R upper (upper part of the leaf)
  TRSM_R = 2,       // X <- R^{-1} X
  TRSM_LC = 3,      // X <- L^{-1} X, L lower with its diagonal (Cholesky factor)
};

// Solve with the dense leaf factor T (n x n, ldt) on X (n x c).  With xtrans
// the operand is the transpose of the stored array (X(i,j) = X[j + i*ldx]).
struct DTrsm {
  const double* T;
  double* X;
  int n, ldt, ldx;
  int kind;
  int xtrans;
  int col0;  // first column handled by this work item (chunks of 64)
  DDim c;
};

enum CopyMode : int { COPY_COPY = 0, COPY_ZERO = 1, COPY_IDENTITY = 2 };

// dst (m x n, ldd) = alpha * op(src) (or zero / identity); optionally *rank_dst = *rank_src.
struct DCopy {
  const double* src;
  double* dst;
  const int* rank_src;
  int* rank_dst;
  double alpha;
  int lds, ldd;
  int strans;
  int mode;
  DDim m, n;
};

// Device status word bits.
enum StatusBits : int {
  ST_RANK_OVERFLOW = 1,  // a truncation needed more columns than its capacity
  ST_ZERO_PIVOT = 2,     // zero pivot in a leaf LU
  ST_NONFINITE = 4,      // NaN or Inf in a truncation
  ST_WS_OVERFLOW = 8,    // the truncation workspace pool was exhausted
  ST_BAD_DESC = 16,      // a descriptor made on the device was invalid or beyond the caller's bounds
};
// Device status block (16 ints): [0] status bits, [1] failing work item + 1,
// [2..3] executed truncations, [4..5] their algorithmic bytes
// 8 (m + n)(l + k), [6..7] the part of those bytes done by the small-block
// kernel, [8..9] truncations done by the rank predictor's range finder,
// [10..11] predicted truncations that fell back to the exact path (64-bit
// counters).
constexpr int STATUS_INTS = 16;

}  // namespace hm
