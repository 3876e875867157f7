// Host replay of the H-matrix algorithms, recorded as work items.
#pragma once
#include <memory>
#include <vector>

#include "program.h"
#include "structure.h"

namespace hm {

// Device-resident H-matrix: tree structure on the host, leaf data on the GPU.
struct DevHMatrix {
  std::shared_ptr<ClusterTree> ct;
  BlockTree bt;
  int kmax = 0;
  int leafmax = 0;
  std::vector<double*> N, A, B;  // per block
  std::vector<int*> R;           // per block rank word (admissible leaves)
  std::vector<int> cap;          // per block rank capacity
  char* pool = nullptr;
  size_t pool_bytes = 0;
  int* ranks = nullptr;
  double* ident = nullptr;  // leafmax x leafmax identity
  AllocRef alloc = default_alloc();  // the allocator that gave pool, ranks and ident
  ~DevHMatrix();
};

struct PNode {
  int t = -1, s = -1, kind = BLK_NONLEAF;
  int nt = 0, ns = 0;
  int rows = 0, cols = 0, roff = 0, coff = 0;
  std::vector<PNode*> sons;
  bool owns_sons = false;
  int objN = -1, objA = -1, objB = -1, objR = -1;
  int cap = 0;
  PNode* son(int i, int j) const { return sons[(size_t)i * ns + j]; }
  ~PNode();
};

struct PlanCounts {
  int64_t trunc_update = 0, trunc_accum = 0, trunc_merge = 0;
  int64_t dense_updates = 0, addproduct = 0, pending = 0, products = 0, leaf_lu = 0, merges = 0;
};

enum Mode : int { MODE_STANDARD = 0, MODE_ACCUMULATED = 1, MODE_FUSED = 2 };

class Planner {
 public:
  Planner(Program& P, const ClusterTree& ct, int kmax, double* ident, int leafmax);
  std::unique_ptr<PNode> attach(DevHMatrix& M);

  void mul(double alpha, PNode* X, PNode* Y, PNode* Z, int mode);
  void lu(PNode* G, int mode);
  // G|_{t x t} <- its inverse (Sect. 6, the block inversion; Fig. invert)
  void inv(PNode* G, int mode);
  // G = L L^T in place, L in the lower blocks (H-Cholesky)
  void chol(PNode* G, int mode);
  // X (n x c dense, cluster order) <- (L R)^{-1} X with the factors stored in G
  void lu_solve(PNode* G, const View& X);
  PlanCounts counts;

 private:
  struct LR {
    View A, B;
    Dim k;
  };
  struct Pend {
    double alpha;
    PNode* X;
    PNode* Y;
    bool trans = false;  // the product X Y^T (H-Cholesky)
  };
  struct Acc {
    int t = -1, r = -1, rows = 0, cols = 0;
    bool has = false;
    int objA = -1, objB = -1, objR = -1, cap = 0;
    std::vector<Pend> P;
  };

  Program& P_;
  const ClusterTree& ct_;
  int kmax_;
  int ident_obj_;
  int leafmax_;
  mutable std::vector<char> split_;  // scratch marks for row_partition
  // scratch region lists of the emitters (no emitter calls another one while
  // it holds them)
  std::vector<Region> rd_, wr_;
  std::vector<HTerm> ts_;  // scratch term list of addeval and addevaltrans

  // views and regions
  View aview(const PNode* b) const;
  View bview(const PNode* b) const;
  View nview(const PNode* b) const;
  View aview(const Acc& a) const;
  View bview(const Acc& a) const;
  View ident(int n) const;
  View temp_view(int rows, Dim cols);
  void add_regions(const View& v, std::vector<Region>& out) const;
  void add_dim(const Dim& d, std::vector<Region>& out) const;
  Region rank_region(int obj) const { return {obj, 0, 1}; }

  // primitive emitters
  void emit_gemm(const View& C, int beta, const std::vector<HTerm>& terms);
  void emit_trunc(int objA, int objB, int objR, int m, int n, int cap, const std::vector<HPart>& parts, int flags,
                  int level);
  void emit_copy(const View& src, const View& dst, Dim m, Dim n, int rank_src, int rank_dst, int mode);
  void emit_trsm(const View& T, const View& X, int n, int kind);
  void emit_lu(const PNode* G, int kind = LEAF_LU);

  // H-matrix operations (Sects. 3-6)
  std::vector<int> row_partition(const PNode* X, bool rows) const;  // uses split_
  void leaves(PNode* X, std::vector<PNode*>& out) const;
  void addeval(double alpha, PNode* X, const View& W, const View& Y, bool accumulate);
  void addevaltrans(double alpha, PNode* X, const View& Yin, const View& Xout, bool accumulate);
  LR lowrank_product(PNode* X, PNode* Y);
  void rkupdate(double alpha, const LR& p, PNode* Z, bool count_update = true);
  void make_temps(PNode* Z);
  void merge_temps(PNode* Z);
  void mul_std(double alpha, PNode* X, PNode* Y, PNode* Z);
  void new_acc_storage(Acc& a);
  void addproduct(double alpha, PNode* X, PNode* Y, Acc& acc);
  std::vector<Acc> split(Acc& acc);
  void flush(Acc& acc, PNode* Z);
  void solve_L(PNode* L, const View& X);
  void solve_Rt(PNode* R, const View& X);
  void solve_R(PNode* R, const View& X);
  void lsolve_leaf(PNode* L, PNode* X);
  void rsolve_leaf(PNode* R, PNode* X);
  PNode* temp_like(const PNode* src);  // zero temporaries with src's block structure
  void zero_blocks(PNode* X);          // X <- 0 (dense leaves zero, ranks zero)
  void inv_std(PNode* G);
  void inv_acc(PNode* G, Acc& acc);
  void acc_add(double alpha, const LR& p, Acc& acc);
  void add_restricted(const Acc& acc, int i, int j, Acc& a);
  bool fused_ = false;  // accumulated mode with the products of a split truncated three at a time
  LR lowrank_product_t(PNode* X, PNode* Y);
  void mul_t_std(double alpha, PNode* X, PNode* Y, PNode* Z);
  void rkupdate_lower(double alpha, const LR& p, PNode* Z);
  void symmul_std(double alpha, PNode* X, PNode* Z);
  void solve_Lc(PNode* L, const View& X);
  void rsolve_t_leaf(PNode* L, PNode* X);
  void rsolve_t_std(PNode* L, PNode* X);
  void chol_std(PNode* G);
  void addproduct_t(double alpha, PNode* X, PNode* Y, Acc& acc);
  std::vector<Acc> split_lower(Acc& acc);
  void rsolve_t_acc(PNode* L, PNode* X, Acc& acc);
  void chol_acc(PNode* G, Acc& acc);
  void lu_std(PNode* G);
  void lsolve_std(PNode* L, PNode* X);
  void rsolve_std(PNode* R, PNode* X);
  void lu_acc(PNode* G, Acc& acc);
  void lsolve_acc(PNode* L, PNode* X, Acc& acc);
  void rsolve_acc(PNode* R, PNode* X, Acc& acc);
  bool leaf(const PNode* b) const { return b->kind != BLK_NONLEAF; }
  bool contains(int outer, int inner) const {
    const Cluster &a = ct_.c[outer], &b = ct_.c[inner];
    return b.off >= a.off && b.off + b.size <= a.off + a.size;
  }
};

}  // namespace hm
