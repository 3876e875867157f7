#include "planner.h"

#include <algorithm>
#include <stdexcept>

namespace hm {

DevHMatrix::~DevHMatrix() {
  alloc->put(pool);
  alloc->put(ranks);
  alloc->put(ident);
}

PNode::~PNode() {
  if (owns_sons)
    for (PNode* p : sons) delete p;
}

Planner::Planner(Program& P, const ClusterTree& ct, int kmax, double* ident, int leafmax)
    : P_(P), ct_(ct), kmax_(kmax), leafmax_(leafmax) {
  ident_obj_ = P_.add_persistent(ident, (int64_t)leafmax * leafmax, leafmax);
}

std::unique_ptr<PNode> Planner::attach(DevHMatrix& M) {
  std::vector<PNode*> nodes(M.bt.b.size(), nullptr);
  for (size_t i = 0; i < M.bt.b.size(); ++i) {
    const Block& b = M.bt.b[i];
    PNode* p = new PNode;
    p->t = b.t;
    p->s = b.s;
    p->kind = b.kind;
    p->rows = ct_.c[b.t].size;
    p->cols = ct_.c[b.s].size;
    p->roff = ct_.c[b.t].off;
    p->coff = ct_.c[b.s].off;
    if (b.kind == BLK_DENSE) p->objN = P_.add_persistent(M.N[i], (int64_t)p->rows * p->cols, p->rows);
    if (b.kind == BLK_RK) {
      p->cap = M.cap[i];
      p->objA = P_.add_persistent(M.A[i], (int64_t)p->rows * p->cap, p->rows);
      p->objB = P_.add_persistent(M.B[i], (int64_t)p->cols * p->cap, p->cols);
      p->objR = P_.add_persistent(M.R[i], 1, 1, true);
    }
    nodes[i] = p;
  }
  for (size_t i = 0; i < M.bt.b.size(); ++i) {
    const Block& b = M.bt.b[i];
    if (b.kind != BLK_NONLEAF) continue;
    PNode* p = nodes[i];
    p->nt = b.nt;
    p->ns = b.ns;
    p->owns_sons = true;
    for (int q = 0; q < b.nt * b.ns; ++q) p->sons.push_back(nodes[b.son0 + q]);
  }
  return std::unique_ptr<PNode>(nodes[0]);
}

// ---------------------------------------------------------------- views
View Planner::aview(const PNode* b) const {
  View v;
  v.obj = b->objA;
  v.ld = b->rows;
  v.rows = b->rows;
  v.cols = {b->cap, b->objR};
  return v;
}
View Planner::bview(const PNode* b) const {
  View v;
  v.obj = b->objB;
  v.ld = b->cols;
  v.rows = b->cols;
  v.cols = {b->cap, b->objR};
  return v;
}
View Planner::nview(const PNode* b) const {
  View v;
  v.obj = b->objN;
  v.ld = b->rows;
  v.rows = b->rows;
  v.cols = {b->cols, -1};
  return v;
}
View Planner::aview(const Acc& a) const {
  View v;
  v.obj = a.objA;
  v.ld = a.rows;
  v.rows = a.rows;
  v.cols = {a.cap, a.objR};
  return v;
}
View Planner::bview(const Acc& a) const {
  View v;
  v.obj = a.objB;
  v.ld = a.cols;
  v.rows = a.cols;
  v.cols = {a.cap, a.objR};
  return v;
}
View Planner::ident(int n) const {
  View v;
  v.obj = ident_obj_;
  v.ld = leafmax_;
  v.rows = n;
  v.cols = {n, -1};
  return v;
}
View Planner::temp_view(int rows, Dim cols) {
  View v;
  v.obj = P_.add_temp((int64_t)rows * std::max(cols.stat, 1), rows);
  v.ld = rows;
  v.rows = rows;
  v.cols = cols;
  return v;
}

void Planner::add_dim(const Dim& d, std::vector<Region>& out) const {
  if (d.rank_obj >= 0) out.push_back(rank_region(d.rank_obj));
}

void Planner::add_regions(const View& v, std::vector<Region>& out) const {
  if (v.obj < 0) return;
  if (v.trans)
    out.push_back({v.obj, 0, std::max(P_.objs[v.obj].rows, 1)});
  else
    out.push_back({v.obj, v.rlo, v.rlo + std::max(v.rows, 1)});
  add_dim(v.cols, out);
}

// ---------------------------------------------------------------- emitters
void Planner::emit_gemm(const View& C, int beta, const std::vector<HTerm>& terms) {
  if (C.rows == 0 || C.cols.stat == 0) return;
  std::vector<Region>& rd = rd_;
  std::vector<Region>& wr = wr_;
  rd.clear();
  wr.clear();
  int term0 = (int)P_.terms.size();
  for (const HTerm& t : terms) {
    grow4(P_.terms);
    P_.terms.push_back(t);
    add_regions(t.A, rd);
    add_regions(t.B, rd);
    add_dim(t.k, rd);
  }
  if (beta) add_regions(C, rd);
  add_dim(C.cols, rd);
  add_regions(C, wr);
  wr.resize(1);  // the output region itself (its rank word is only read)
  int first = (int)P_.gemms.size();
  for (int r0 = 0; r0 < C.rows; r0 += 64)
    for (int c0 = 0; c0 < C.cols.stat; c0 += 64) {
      HGemm g;
      g.C = C;
      g.m = {C.rows, -1};
      g.beta = beta;
      g.term0 = term0;
      g.nterms = (int)terms.size();
      g.row0 = r0;
      g.col0 = c0;
      grow4(P_.gemms);
      P_.gemms.push_back(g);
    }
  int cnt = (int)P_.gemms.size() - first;
  P_.record(OP_GEMM, first, rd, wr);
  for (int q = 1; q < cnt; ++q) P_.push_sibling(OP_GEMM, first + q);
  P_.stats.items[OP_GEMM] += cnt - 1;
}

void Planner::emit_trunc(int objA, int objB, int objR, int m, int n, int cap, const std::vector<HPart>& parts,
                         int flags, int level) {
  if (parts.empty() || parts.size() > 4) throw std::runtime_error("truncation with unsupported part count");
  std::vector<Region>& rd = rd_;
  std::vector<Region>& wr = wr_;
  rd.clear();
  wr.clear();
  HTrunc t;
  t.objA = objA;
  t.objB = objB;
  t.objR = objR;
  t.m = m;
  t.n = n;
  t.cap = cap;
  t.part0 = (int)P_.parts.size();
  t.nparts = (int)parts.size();
  t.lmax = 0;
  t.flags = flags;
  t.level = level;
  for (const HPart& p : parts) {
    grow4(P_.parts);
    P_.parts.push_back(p);
    t.lmax += p.k.stat;
    add_regions(p.A, rd);
    add_regions(p.B, rd);
    add_dim(p.k, rd);
  }
  wr.push_back({objA, 0, m});
  wr.push_back({objB, 0, n});
  wr.push_back(rank_region(objR));
  int idx = (int)P_.truncs.size();
  grow4(P_.truncs);
  P_.truncs.push_back(t);
  P_.record(OP_TRUNC, idx, rd, wr);
}

void Planner::emit_copy(const View& src, const View& dst, Dim m, Dim n, int rank_src, int rank_dst, int mode) {
  std::vector<Region>& rd = rd_;
  std::vector<Region>& wr = wr_;
  rd.clear();
  wr.clear();
  HCopy c;
  c.src = src;
  c.dst = dst;
  c.m = m;
  c.n = n;
  c.mode = mode;
  c.rank_src = rank_src;
  c.rank_dst = rank_dst;
  if (mode == COPY_COPY && src.obj >= 0) add_regions(src, rd);
  add_dim(m, rd);
  add_dim(n, rd);
  if (rank_src >= 0) rd.push_back(rank_region(rank_src));
  if (dst.obj >= 0) wr.push_back({dst.obj, dst.rlo, dst.rlo + std::max(dst.rows, 1)});
  if (rank_dst >= 0) wr.push_back(rank_region(rank_dst));
  int idx = (int)P_.copies.size();
  grow4(P_.copies);
  P_.copies.push_back(c);
  P_.record(OP_COPY, idx, rd, wr);
}

void Planner::emit_trsm(const View& T, const View& X, int n, int kind) {
  if (X.cols.stat == 0) return;
  if (n > 64) throw std::runtime_error("leaf solves support leaves of at most 64 points");
  std::vector<Region>& rd = rd_;
  std::vector<Region>& wr = wr_;
  rd.clear();
  wr.clear();
  add_regions(T, rd);
  add_regions(X, rd);
  add_regions(X, wr);
  wr.resize(1);
  int first = (int)P_.trsms.size();
  for (int c0 = 0; c0 < X.cols.stat; c0 += 32) {
    HTrsm t;
    t.T = T;
    t.X = X;
    t.n = n;
    t.kind = kind;
    t.col0 = c0;
    P_.trsms.push_back(t);
  }
  int cnt = (int)P_.trsms.size() - first;
  P_.record(OP_TRSM, first, rd, wr);
  for (int q = 1; q < cnt; ++q) P_.push_sibling(OP_TRSM, first + q);
  P_.stats.items[OP_TRSM] += cnt - 1;
  P_.trsm_nmax = std::max(P_.trsm_nmax, n);
}

void Planner::emit_lu(const PNode* G, int kind) {
  if (G->rows > 64) throw std::runtime_error("leaf LU supports leaves of at most 64 points");
  std::vector<Region>& rd = rd_;
  std::vector<Region>& wr = wr_;
  rd.clear();
  wr.clear();
  rd.push_back({G->objN, 0, G->rows});
  wr.push_back({G->objN, 0, G->rows});
  int idx = (int)P_.lus.size();
  P_.lus.push_back({G->objN, G->rows, kind});
  P_.record(OP_LU, idx, rd, wr);
  P_.lu_nmax = std::max(P_.lu_nmax, G->rows);
  counts.leaf_lu++;
}

// ---------------------------------------------------------------- addeval
void Planner::leaves(PNode* X, std::vector<PNode*>& out) const {
  if (leaf(X)) {
    out.push_back(X);
    return;
  }
  for (PNode* s : X->sons) leaves(s, out);
}

// Coarsest partition of X's row (or column) cluster that refines the row (or
// column) clusters of all leaves below X.
std::vector<int> Planner::row_partition(const PNode* X, bool rows) const {
  std::vector<PNode*> lv;
  leaves(const_cast<PNode*>(X), lv);
  const int root = rows ? X->t : X->s;
  std::vector<char>& split = split_;
  if (split.size() != ct_.c.size()) split.assign(ct_.c.size(), 0);
  std::vector<int> marked;
  for (PNode* b : lv) {
    int c = rows ? b->t : b->s;
    while (c != root && c >= 0) {
      c = ct_.c[c].parent;
      if (c < 0 || split[c]) break;
      split[c] = 1;
      marked.push_back(c);
    }
  }
  std::vector<int> out, stack{root};
  while (!stack.empty()) {
    int c = stack.back();
    stack.pop_back();
    if (split[c] && ct_.c[c].nsons > 0) {
      for (int q = ct_.c[c].nsons - 1; q >= 0; --q) stack.push_back(ct_.c[c].son[q]);
    } else {
      out.push_back(c);
    }
  }
  for (int c : marked) split[c] = 0;
  return out;
}

// Y (#t x c) = [Y +] alpha X|_{t x s} W  (Fig. addeval).  Phase 1 projects each
// admissible leaf, T_b = alpha B_b^T W|_s; phase 2 sums, per row block tau, the
// contributions N_b|_tau W|_s and A_b|_tau T_b in depth-first leaf order.
void Planner::addeval(double alpha, PNode* X, const View& W, const View& Y, bool accumulate) {
  if (W.cols.stat == 0) return;
  std::vector<PNode*> lv;
  leaves(X, lv);
  std::vector<View> T(lv.size());
  for (size_t q = 0; q < lv.size(); ++q) {
    PNode* b = lv[q];
    if (b->kind != BLK_RK || b->cap == 0) continue;
    T[q] = temp_view(b->cap, W.cols);
    HTerm t;
    t.A = bview(b);
    t.ta = 1;
    t.B = W.rows_sub(b->coff - X->coff, b->cols);
    t.tb = 0;
    t.alpha = alpha;
    t.k = {b->cols, -1};
    View Tm = T[q];
    // rows of T are the (dynamic) rank of b
    // emit with dynamic m
    std::vector<Region>& rd = rd_;
    std::vector<Region>& wr = wr_;
    rd.clear();
    wr.clear();
    int term0 = (int)P_.terms.size();
    grow4(P_.terms);
    P_.terms.push_back(t);
    add_regions(t.A, rd);
    add_regions(t.B, rd);
    add_dim(W.cols, rd);
    wr.push_back({Tm.obj, 0, Tm.rows});
    int first = (int)P_.gemms.size();
    for (int r0 = 0; r0 < b->cap; r0 += 64)
      for (int c0 = 0; c0 < W.cols.stat; c0 += 64) {
        HGemm g;
        g.C = Tm;
        g.m = {b->cap, b->objR};
        g.beta = 0;
        g.term0 = term0;
        g.nterms = 1;
        g.row0 = r0;
        g.col0 = c0;
        grow4(P_.gemms);
        P_.gemms.push_back(g);
      }
    int cnt = (int)P_.gemms.size() - first;
    P_.record(OP_GEMM, first, rd, wr);
    for (int z = 1; z < cnt; ++z) P_.push_sibling(OP_GEMM, first + z);
    P_.stats.items[OP_GEMM] += cnt - 1;
  }
  for (int tau : row_partition(X, true)) {
    const Cluster& ct = ct_.c[tau];
    std::vector<HTerm>& ts = ts_;
    ts.clear();
    for (size_t q = 0; q < lv.size(); ++q) {
      PNode* b = lv[q];
      if (!contains(b->t, tau)) continue;
      const int ro = ct.off - b->roff;
      HTerm t;
      if (b->kind == BLK_DENSE) {
        t.A = nview(b).rows_sub(ro, ct.size);
        t.B = W.rows_sub(b->coff - X->coff, b->cols);
        t.alpha = alpha;
        t.k = {b->cols, -1};
      } else {
        if (b->cap == 0) continue;
        t.A = aview(b).rows_sub(ro, ct.size);
        t.B = T[q];
        t.alpha = 1.0;
        t.k = {b->cap, b->objR};
      }
      ts.push_back(t);
    }
    emit_gemm(Y.rows_sub(ct.off - X->roff, ct.size), accumulate ? 1 : 0, ts);
  }
}

// Xout (#s x c) = [Xout +] alpha X|_{t x s}^T Yin  (Fig. addeval, transposed).
void Planner::addevaltrans(double alpha, PNode* X, const View& Yin, const View& Xout, bool accumulate) {
  if (Yin.cols.stat == 0) return;
  std::vector<PNode*> lv;
  leaves(X, lv);
  std::vector<View> T(lv.size());
  for (size_t q = 0; q < lv.size(); ++q) {
    PNode* b = lv[q];
    if (b->kind != BLK_RK || b->cap == 0) continue;
    T[q] = temp_view(b->cap, Yin.cols);
    HTerm t;
    t.A = aview(b);
    t.ta = 1;
    t.B = Yin.rows_sub(b->roff - X->roff, b->rows);
    t.alpha = alpha;
    t.k = {b->rows, -1};
    std::vector<Region>& rd = rd_;
    std::vector<Region>& wr = wr_;
    rd.clear();
    wr.clear();
    int term0 = (int)P_.terms.size();
    grow4(P_.terms);
    P_.terms.push_back(t);
    add_regions(t.A, rd);
    add_regions(t.B, rd);
    add_dim(Yin.cols, rd);
    wr.push_back({T[q].obj, 0, T[q].rows});
    int first = (int)P_.gemms.size();
    for (int r0 = 0; r0 < b->cap; r0 += 64)
      for (int c0 = 0; c0 < Yin.cols.stat; c0 += 64) {
        HGemm g;
        g.C = T[q];
        g.m = {b->cap, b->objR};
        g.beta = 0;
        g.term0 = term0;
        g.nterms = 1;
        g.row0 = r0;
        g.col0 = c0;
        grow4(P_.gemms);
        P_.gemms.push_back(g);
      }
    int cnt = (int)P_.gemms.size() - first;
    P_.record(OP_GEMM, first, rd, wr);
    for (int z = 1; z < cnt; ++z) P_.push_sibling(OP_GEMM, first + z);
    P_.stats.items[OP_GEMM] += cnt - 1;
  }
  for (int sig : row_partition(X, false)) {
    const Cluster& cs = ct_.c[sig];
    std::vector<HTerm>& ts = ts_;
    ts.clear();
    for (size_t q = 0; q < lv.size(); ++q) {
      PNode* b = lv[q];
      if (!contains(b->s, sig)) continue;
      const int co = cs.off - b->coff;
      HTerm t;
      if (b->kind == BLK_DENSE) {
        View nc = nview(b);
        nc.off += (int64_t)co * nc.ld;
        nc.cols = {cs.size, -1};
        t.A = nc;  // rows x |sigma| block of N_b, used transposed
        t.ta = 1;
        t.B = Yin.rows_sub(b->roff - X->roff, b->rows);
        t.alpha = alpha;
        t.k = {b->rows, -1};
      } else {
        if (b->cap == 0) continue;
        t.A = bview(b).rows_sub(co, cs.size);
        t.B = T[q];
        t.alpha = 1.0;
        t.k = {b->cap, b->objR};
      }
      ts.push_back(t);
    }
    emit_gemm(Xout.rows_sub(cs.off - X->coff, cs.size), accumulate ? 1 : 0, ts);
  }
}

// ---------------------------------------------------------------- products
// Low-rank form of X|_{t x s} Y|_{s x r} when one factor is a leaf: the four
// branches of Fig. addproduct, without alpha (applied once, in the truncation).
Planner::LR Planner::lowrank_product(PNode* X, PNode* Y) {
  LR p;
  const int nt = X->rows, ns = X->cols, nr = Y->cols;
  counts.products++;
  if (X->kind == BLK_DENSE) {
    if (nt <= ns) {
      p.k = {nt, -1};
      p.A = ident(nt);
      p.B = temp_view(nr, p.k);
      View W = nview(X);  // N_X^T as an #s x #t operand
      W.trans = 1;
      W.rows = ns;
      W.cols = {nt, -1};
      addevaltrans(1.0, Y, W, p.B, false);
    } else {
      p.k = {ns, -1};
      p.A = nview(X);
      p.B = temp_view(nr, p.k);
      addevaltrans(1.0, Y, ident(ns), p.B, false);
    }
  } else if (Y->kind == BLK_DENSE) {
    if (nr <= ns) {
      p.k = {nr, -1};
      p.B = ident(nr);
      p.A = temp_view(nt, p.k);
      addeval(1.0, X, nview(Y), p.A, false);
    } else {
      p.k = {ns, -1};
      View Bt = nview(Y);  // N_Y^T as an #r x #s operand
      Bt.trans = 1;
      Bt.rows = nr;
      Bt.cols = {ns, -1};
      p.B = Bt;
      p.A = temp_view(nt, p.k);
      addeval(1.0, X, ident(ns), p.A, false);
    }
  } else if (X->kind == BLK_RK) {
    p.k = {X->cap, X->objR};
    p.A = aview(X);
    if (X->cap == 0) return p;
    p.B = temp_view(nr, p.k);
    addevaltrans(1.0, Y, bview(X), p.B, false);
  } else {
    p.k = {Y->cap, Y->objR};
    p.B = bview(Y);
    if (Y->cap == 0) return p;
    p.A = temp_view(nt, p.k);
    addeval(1.0, X, aview(Y), p.A, false);
  }
  return p;
}

// Fig. rkupdate: dense leaves N += alpha A B^T, admissible leaves rkadd,
// recursion with restricted factors otherwise.
void Planner::rkupdate(double alpha, const LR& p, PNode* Z, bool count_update) {
  if (p.k.stat == 0) return;
  if (Z->kind == BLK_DENSE) {
    HTerm t;
    t.A = p.A;
    t.B = p.B;
    t.tb = 1;
    t.alpha = alpha;
    t.k = p.k;
    emit_gemm(nview(Z), 1, {t});
    counts.dense_updates++;
  } else if (Z->kind == BLK_RK) {
    HPart u;
    u.A = p.A;
    u.B = p.B;
    u.alpha = alpha;
    u.rows = Z->rows;
    u.cols = Z->cols;
    u.k = p.k;
    HPart z;
    z.A = aview(Z);
    z.B = bview(Z);
    z.rows = Z->rows;
    z.cols = Z->cols;
    z.k = {Z->cap, Z->objR};
    emit_trunc(Z->objA, Z->objB, Z->objR, Z->rows, Z->cols, Z->cap, {u, z}, TRUNC_SKIP_IF_PART0_EMPTY,
               ct_.c[Z->t].level);
    if (count_update) counts.trunc_update++;
  } else {
    for (PNode* b : Z->sons) {
      LR q;
      q.A = p.A.rows_sub(b->roff - Z->roff, b->rows);
      q.B = p.B.rows_sub(b->coff - Z->coff, b->cols);
      q.k = p.k;
      rkupdate(alpha, q, b, count_update);
    }
  }
}

// Temporary sons of a leaf Z (Sect. 4): dense sub-blocks or restricted factors.
void Planner::make_temps(PNode* Z) {
  const Cluster &ct = ct_.c[Z->t], &cs = ct_.c[Z->s];
  Z->nt = ct.nsons;
  Z->ns = cs.nsons;
  Z->owns_sons = true;
  for (int i = 0; i < ct.nsons; ++i)
    for (int j = 0; j < cs.nsons; ++j) {
      PNode* b = new PNode;
      b->t = ct.son[i];
      b->s = cs.son[j];
      b->kind = Z->kind;
      b->rows = ct_.c[b->t].size;
      b->cols = ct_.c[b->s].size;
      b->roff = ct_.c[b->t].off;
      b->coff = ct_.c[b->s].off;
      const int ro = b->roff - Z->roff, co = b->coff - Z->coff;
      if (Z->kind == BLK_DENSE) {
        b->objN = P_.add_temp((int64_t)b->rows * b->cols, b->rows);
        View src = nview(Z);
        src.off = ro + (int64_t)co * src.ld;
        src.rlo = ro;
        src.rows = b->rows;
        src.cols = {b->cols, -1};
        emit_copy(src, nview(b), {b->rows, -1}, {b->cols, -1}, -1, -1, COPY_COPY);
      } else {
        b->cap = std::max(Z->cap, std::min(std::min(b->rows, b->cols), kmax_));
        b->objA = P_.add_temp((int64_t)b->rows * b->cap, b->rows);
        b->objB = P_.add_temp((int64_t)b->cols * b->cap, b->cols);
        b->objR = P_.add_temp(1, 1, true);
        Dim kz{Z->cap, Z->objR};
        emit_copy(aview(Z).rows_sub(ro, b->rows), aview(b), {b->rows, -1}, kz, Z->objR, b->objR, COPY_COPY);
        emit_copy(bview(Z).rows_sub(co, b->cols), bview(b), {b->cols, -1}, kz, -1, -1, COPY_COPY);
      }
      Z->sons.push_back(b);
    }
}

// Copy back (dense) or rkmerge (Fig. rkmerge, block columns first).
void Planner::merge_temps(PNode* Z) {
  if (Z->kind == BLK_DENSE) {
    for (PNode* b : Z->sons) {
      View dst = nview(Z);
      const int ro = b->roff - Z->roff, co = b->coff - Z->coff;
      dst.off = ro + (int64_t)co * dst.ld;
      dst.rlo = ro;
      dst.rows = b->rows;
      dst.cols = {b->cols, -1};
      emit_copy(nview(b), dst, {b->rows, -1}, {b->cols, -1}, -1, -1, COPY_COPY);
    }
  } else {
    counts.merges++;
    std::vector<HPart> rowparts;
    for (int j = 0; j < Z->ns; ++j) {
      const Cluster& rj = ct_.c[Z->son(0, j)->s];
      std::vector<HPart> cp;
      for (int i = 0; i < Z->nt; ++i) {
        PNode* b = Z->son(i, j);
        HPart h;
        h.A = aview(b);
        h.B = bview(b);
        h.row_off = b->roff - Z->roff;
        h.rows = b->rows;
        h.col_off = 0;
        h.cols = b->cols;
        h.k = {b->cap, b->objR};
        cp.push_back(h);
      }
      const int capj = std::min(std::min(Z->rows, rj.size), kmax_);
      const int oA = P_.add_temp((int64_t)Z->rows * std::max(capj, 1), Z->rows);
      const int oB = P_.add_temp((int64_t)rj.size * std::max(capj, 1), rj.size);
      const int oR = P_.add_temp(1, 1, true);
      emit_trunc(oA, oB, oR, Z->rows, rj.size, capj, cp, 0, ct_.c[Z->t].level);
      counts.trunc_merge++;
      HPart h;
      h.A.obj = oA;
      h.A.ld = Z->rows;
      h.A.rows = Z->rows;
      h.A.cols = {capj, oR};
      h.B.obj = oB;
      h.B.ld = rj.size;
      h.B.rows = rj.size;
      h.B.cols = {capj, oR};
      h.row_off = 0;
      h.rows = Z->rows;
      h.col_off = rj.off - Z->coff;
      h.cols = rj.size;
      h.k = {capj, oR};
      rowparts.push_back(h);
    }
    emit_trunc(Z->objA, Z->objB, Z->objR, Z->rows, Z->cols, Z->cap, rowparts, 0, ct_.c[Z->t].level);
    counts.trunc_merge++;
  }
  for (PNode* b : Z->sons) delete b;
  Z->sons.clear();
  Z->nt = Z->ns = 0;
  Z->owns_sons = false;
}

// ---------------------------------------------------------------- multiplication
void Planner::mul_std(double alpha, PNode* X, PNode* Y, PNode* Z) {
  if (leaf(X) || leaf(Y)) {
    LR p = lowrank_product(X, Y);
    rkupdate(alpha, p, Z);
    return;
  }
  const bool temps = leaf(Z);
  if (temps) make_temps(Z);
  for (int i = 0; i < X->nt; ++i)
    for (int j = 0; j < Y->ns; ++j)
      for (int l = 0; l < X->ns; ++l) mul_std(alpha, X->son(i, l), Y->son(l, j), Z->son(i, j));
  if (temps) merge_temps(Z);
}

void Planner::new_acc_storage(Acc& a) {
  a.cap = std::min(std::min(a.rows, a.cols), kmax_);
  a.objA = P_.add_temp((int64_t)a.rows * std::max(a.cap, 1), a.rows);
  a.objB = P_.add_temp((int64_t)a.cols * std::max(a.cap, 1), a.cols);
  a.objR = P_.add_temp(1, 1, true);
  a.has = true;
  emit_copy(View(), View(), {0, -1}, {0, -1}, -1, a.objR, COPY_ZERO);
}

// A low-rank product added to an accumulator by a truncation (rkadd).
void Planner::acc_add(double alpha, const LR& p, Acc& acc) {
  if (p.k.stat == 0) return;
  if (!acc.has) new_acc_storage(acc);
  HPart u;
  u.A = p.A;
  u.B = p.B;
  u.alpha = alpha;
  u.rows = acc.rows;
  u.cols = acc.cols;
  u.k = p.k;
  HPart z;
  z.A = aview(acc);
  z.B = bview(acc);
  z.rows = acc.rows;
  z.cols = acc.cols;
  z.k = {acc.cap, acc.objR};
  emit_trunc(acc.objA, acc.objB, acc.objR, acc.rows, acc.cols, acc.cap, {u, z}, TRUNC_SKIP_IF_PART0_EMPTY,
             ct_.c[acc.t].level);
  counts.trunc_accum++;
}

// Fig. addproduct.
void Planner::addproduct(double alpha, PNode* X, PNode* Y, Acc& acc) {
  counts.addproduct++;
  if (leaf(X) || leaf(Y)) {
    LR p = lowrank_product(X, Y);
    if (p.k.stat == 0) return;
    if (!acc.has) new_acc_storage(acc);
    HPart u;
    u.A = p.A;
    u.B = p.B;
    u.alpha = alpha;
    u.rows = acc.rows;
    u.cols = acc.cols;
    u.k = p.k;
    HPart z;
    z.A = aview(acc);
    z.B = bview(acc);
    z.rows = acc.rows;
    z.cols = acc.cols;
    z.k = {acc.cap, acc.objR};
    emit_trunc(acc.objA, acc.objB, acc.objR, acc.rows, acc.cols, acc.cap, {u, z}, TRUNC_SKIP_IF_PART0_EMPTY,
               ct_.c[acc.t].level);
    counts.trunc_accum++;
  } else {
    acc.P.push_back({alpha, X, Y});
    counts.pending++;
  }
}

// The pending products of acc restricted to the son (i, j), added to the son
// accumulator a: each leaf product by its own truncation (Fig. addproduct),
// or, fused, in groups of three consecutive leaf products, each group
// truncated with a in one item (an item whose products all have zero columns
// at run time is a no-op).
void Planner::add_restricted(const Acc& acc, int i, int j, Acc& a) {
  if (!fused_) {
    for (const Pend& p : acc.P)
      for (int l = 0; l < p.X->ns; ++l) {
        if (p.trans)
          addproduct_t(p.alpha, p.X->son(i, l), p.Y->son(j, l), a);
        else
          addproduct(p.alpha, p.X->son(i, l), p.Y->son(l, j), a);
      }
    return;
  }
  std::vector<LR> prods;
  std::vector<double> alphas;
  for (const Pend& p : acc.P)
    for (int l = 0; l < p.X->ns; ++l) {
      PNode* X = p.X->son(i, l);
      PNode* Y = p.trans ? p.Y->son(j, l) : p.Y->son(l, j);
      counts.addproduct++;
      if (leaf(X) || leaf(Y)) {
        prods.push_back(p.trans ? lowrank_product_t(X, Y) : lowrank_product(X, Y));
        alphas.push_back(p.alpha);
      } else {
        a.P.push_back({p.alpha, X, Y, p.trans});
        counts.pending++;
      }
    }
  for (size_t g = 0; g < prods.size(); g += 3) {
    std::vector<HPart> parts;
    for (size_t q = g; q < std::min(prods.size(), g + 3); ++q) {
      if (prods[q].k.stat == 0) continue;
      HPart u;
      u.A = prods[q].A;
      u.B = prods[q].B;
      u.alpha = alphas[q];
      u.rows = a.rows;
      u.cols = a.cols;
      u.k = prods[q].k;
      parts.push_back(u);
    }
    if (parts.empty()) continue;
    if (!a.has) new_acc_storage(a);
    HPart z;
    z.A = aview(a);
    z.B = bview(a);
    z.rows = a.rows;
    z.cols = a.cols;
    z.k = {a.cap, a.objR};
    parts.push_back(z);
    emit_trunc(a.objA, a.objB, a.objR, a.rows, a.cols, a.cap, parts, TRUNC_SKIP_IF_HEAD_EMPTY, ct_.c[a.t].level);
    counts.trunc_accum++;
  }
}

// Fig. split: sons inherit the restricted low-rank part; pending products are
// re-added for every son of s.
std::vector<Planner::Acc> Planner::split(Acc& acc) {
  const Cluster &ct = ct_.c[acc.t], &cr = ct_.c[acc.r];
  std::vector<Acc> out;
  for (int i = 0; i < ct.nsons; ++i)
    for (int j = 0; j < cr.nsons; ++j) {
      Acc a;
      a.t = ct.son[i];
      a.r = cr.son[j];
      a.rows = ct_.c[a.t].size;
      a.cols = ct_.c[a.r].size;
      if (acc.has) {
        a.cap = std::max(acc.cap, std::min(std::min(a.rows, a.cols), kmax_));
        a.objA = P_.add_temp((int64_t)a.rows * std::max(a.cap, 1), a.rows);
        a.objB = P_.add_temp((int64_t)a.cols * std::max(a.cap, 1), a.cols);
        a.objR = P_.add_temp(1, 1, true);
        a.has = true;
        Dim k{acc.cap, acc.objR};
        emit_copy(aview(acc).rows_sub(ct_.c[a.t].off - ct.off, a.rows), aview(a), {a.rows, -1}, k, acc.objR, a.objR,
                  COPY_COPY);
        emit_copy(bview(acc).rows_sub(ct_.c[a.r].off - cr.off, a.cols), bview(a), {a.cols, -1}, k, -1, -1, COPY_COPY);
      }
      add_restricted(acc, i, j, a);
      out.push_back(std::move(a));
    }
  return out;
}

// Fig. flush.
void Planner::flush(Acc& acc, PNode* Z) {
  if (acc.P.empty()) {
    if (acc.has) {
      LR p;
      p.A = aview(acc);
      p.B = bview(acc);
      p.k = {acc.cap, acc.objR};
      rkupdate(1.0, p, Z);
    }
  } else {
    const bool temps = leaf(Z);
    if (temps) make_temps(Z);
    std::vector<Acc> sons = split(acc);
    for (int i = 0; i < Z->nt; ++i)
      for (int j = 0; j < Z->ns; ++j) flush(sons[(size_t)i * Z->ns + j], Z->son(i, j));
    if (temps) merge_temps(Z);
  }
  acc.has = false;
  acc.P.clear();
}

void Planner::mul(double alpha, PNode* X, PNode* Y, PNode* Z, int mode) {
  fused_ = mode == MODE_FUSED;
  if (mode == MODE_STANDARD) {
    mul_std(alpha, X, Y, Z);
  } else {
    Acc acc;
    acc.t = Z->t;
    acc.r = Z->s;
    acc.rows = Z->rows;
    acc.cols = Z->cols;
    addproduct(alpha, X, Y, acc);
    flush(acc, Z);
  }
}

// ---------------------------------------------------------------- H-LU
// X (#t x c) <- L_tt^{-1} X with the unit lower part of the diagonal block.
void Planner::solve_L(PNode* L, const View& X) {
  if (X.cols.stat == 0) return;
  if (L->kind == BLK_DENSE) {
    emit_trsm(nview(L), X, L->rows, TRSM_L_UNIT);
    return;
  }
  PNode *L00 = L->son(0, 0), *L10 = L->son(1, 0), *L11 = L->son(1, 1);
  View X0 = X.rows_sub(0, L00->rows), X1 = X.rows_sub(L00->rows, L11->rows);
  solve_L(L00, X0);
  addeval(-1.0, L10, X0, X1, true);
  solve_L(L11, X1);
}

// X (#t x c) <- R_tt^{-T} X with the upper part of the diagonal block.
void Planner::solve_Rt(PNode* R, const View& X) {
  if (X.cols.stat == 0) return;
  if (R->kind == BLK_DENSE) {
    emit_trsm(nview(R), X, R->rows, TRSM_RT);
    return;
  }
  PNode *R00 = R->son(0, 0), *R01 = R->son(0, 1), *R11 = R->son(1, 1);
  View X0 = X.rows_sub(0, R00->rows), X1 = X.rows_sub(R00->rows, R11->rows);
  solve_Rt(R00, X0);
  addevaltrans(-1.0, R01, X0, X1, true);
  solve_Rt(R11, X1);
}

static void need_binary(const PNode* G);

// X (#t x c) <- R_tt^{-1} X with the upper part of the diagonal block
// (backward substitution by blocks).
void Planner::solve_R(PNode* R, const View& X) {
  if (X.cols.stat == 0) return;
  if (R->kind == BLK_DENSE) {
    emit_trsm(nview(R), X, R->rows, TRSM_R);
    return;
  }
  PNode *R00 = R->son(0, 0), *R01 = R->son(0, 1), *R11 = R->son(1, 1);
  View X0 = X.rows_sub(0, R00->rows), X1 = X.rows_sub(R00->rows, R11->rows);
  solve_R(R11, X1);
  addeval(-1.0, R01, X1, X0, true);
  solve_R(R00, X0);
}

// Solution with the factors of an H-LU: forward substitution with the unit
// lower factor, then backward substitution with the upper one.
void Planner::lu_solve(PNode* G, const View& X) {
  if (G->kind != BLK_DENSE) need_binary(G);
  solve_L(G, X);
  solve_R(G, X);
}

void Planner::lsolve_leaf(PNode* L, PNode* X) {
  if (X->kind == BLK_DENSE)
    solve_L(L, nview(X));
  else if (X->cap > 0)
    solve_L(L, aview(X));
}

void Planner::rsolve_leaf(PNode* R, PNode* X) {
  if (X->kind == BLK_DENSE) {
    View v = nview(X);  // X^T: #s x #t
    v.trans = 1;
    v.rows = X->cols;
    v.cols = {X->rows, -1};
    solve_Rt(R, v);
  } else if (X->cap > 0) {
    solve_Rt(R, bview(X));
  }
}

static void need_binary(const PNode* G) {
  if (G->nt != 2 || G->ns != 2) throw std::runtime_error("H-LU needs a binary cluster tree");
}

void Planner::lu_std(PNode* G) {
  if (G->kind == BLK_DENSE) {
    emit_lu(G);
    return;
  }
  need_binary(G);
  lu_std(G->son(0, 0));
  lsolve_std(G->son(0, 0), G->son(0, 1));
  rsolve_std(G->son(0, 0), G->son(1, 0));
  mul_std(-1.0, G->son(1, 0), G->son(0, 1), G->son(1, 1));
  lu_std(G->son(1, 1));
}

void Planner::lsolve_std(PNode* L, PNode* X) {
  if (leaf(X)) {
    lsolve_leaf(L, X);
    return;
  }
  need_binary(L);
  for (int j = 0; j < X->ns; ++j) {
    lsolve_std(L->son(0, 0), X->son(0, j));
    mul_std(-1.0, L->son(1, 0), X->son(0, j), X->son(1, j));
    lsolve_std(L->son(1, 1), X->son(1, j));
  }
}

void Planner::rsolve_std(PNode* R, PNode* X) {
  if (leaf(X)) {
    rsolve_leaf(R, X);
    return;
  }
  need_binary(R);
  for (int i = 0; i < X->nt; ++i) {
    rsolve_std(R->son(0, 0), X->son(i, 0));
    mul_std(-1.0, X->son(i, 0), R->son(0, 1), X->son(i, 1));
    rsolve_std(R->son(1, 1), X->son(i, 1));
  }
}

void Planner::lu_acc(PNode* G, Acc& acc) {
  if (G->kind == BLK_DENSE) {
    flush(acc, G);
    emit_lu(G);
    return;
  }
  need_binary(G);
  std::vector<Acc> a = split(acc);
  acc.has = false;
  acc.P.clear();
  lu_acc(G->son(0, 0), a[0]);
  lsolve_acc(G->son(0, 0), G->son(0, 1), a[1]);
  rsolve_acc(G->son(0, 0), G->son(1, 0), a[2]);
  addproduct(-1.0, G->son(1, 0), G->son(0, 1), a[3]);
  lu_acc(G->son(1, 1), a[3]);
}

void Planner::lsolve_acc(PNode* L, PNode* X, Acc& acc) {
  if (leaf(X)) {
    flush(acc, X);
    lsolve_leaf(L, X);
    return;
  }
  need_binary(L);
  std::vector<Acc> a = split(acc);
  acc.has = false;
  acc.P.clear();
  for (int j = 0; j < X->ns; ++j) {
    lsolve_acc(L->son(0, 0), X->son(0, j), a[j]);
    addproduct(-1.0, L->son(1, 0), X->son(0, j), a[X->ns + j]);
    lsolve_acc(L->son(1, 1), X->son(1, j), a[X->ns + j]);
  }
}

void Planner::rsolve_acc(PNode* R, PNode* X, Acc& acc) {
  if (leaf(X)) {
    flush(acc, X);
    rsolve_leaf(R, X);
    return;
  }
  need_binary(R);
  std::vector<Acc> a = split(acc);
  acc.has = false;
  acc.P.clear();
  for (int i = 0; i < X->nt; ++i) {
    rsolve_acc(R->son(0, 0), X->son(i, 0), a[(size_t)i * X->ns]);
    addproduct(-1.0, X->son(i, 0), R->son(0, 1), a[(size_t)i * X->ns + 1]);
    rsolve_acc(R->son(1, 1), X->son(i, 1), a[(size_t)i * X->ns + 1]);
  }
}

// ---------------------------------------------------------------- inversion
PNode* Planner::temp_like(const PNode* src) {
  PNode* b = new PNode;
  b->t = src->t;
  b->s = src->s;
  b->kind = src->kind;
  b->rows = src->rows;
  b->cols = src->cols;
  b->roff = src->roff;
  b->coff = src->coff;
  if (src->kind == BLK_DENSE) {
    b->objN = P_.add_temp((int64_t)b->rows * b->cols, b->rows);
    emit_copy(View(), nview(b), {b->rows, -1}, {b->cols, -1}, -1, -1, COPY_ZERO);
  } else if (src->kind == BLK_RK) {
    b->cap = src->cap;
    b->objA = P_.add_temp((int64_t)b->rows * std::max(b->cap, 1), b->rows);
    b->objB = P_.add_temp((int64_t)b->cols * std::max(b->cap, 1), b->cols);
    b->objR = P_.add_temp(1, 1, true);
    emit_copy(View(), View(), {0, -1}, {0, -1}, -1, b->objR, COPY_ZERO);
  } else {
    b->nt = src->nt;
    b->ns = src->ns;
    b->owns_sons = true;
    for (PNode* c : src->sons) b->sons.push_back(temp_like(c));
  }
  return b;
}

void Planner::zero_blocks(PNode* X) {
  if (X->kind == BLK_DENSE)
    emit_copy(View(), nview(X), {X->rows, -1}, {X->cols, -1}, -1, -1, COPY_ZERO);
  else if (X->kind == BLK_RK)
    emit_copy(View(), View(), {0, -1}, {0, -1}, -1, X->objR, COPY_ZERO);
  else
    for (PNode* c : X->sons) zero_blocks(c);
}

// The six steps of the block inversion with standard products: G11 <- G11^-1;
// H12 = G11 G12, H21 = G21 G11; G22 <- S = G22 - H21 G12; G22 <- S^-1;
// G12 = -H12 G22, G21 = -G22 H21; G11 <- G11 - H12 G21.
void Planner::inv_std(PNode* G) {
  if (G->kind == BLK_DENSE) {
    emit_lu(G, LEAF_INVERSE);
    return;
  }
  need_binary(G);
  PNode *G11 = G->son(0, 0), *G12 = G->son(0, 1), *G21 = G->son(1, 0), *G22 = G->son(1, 1);
  inv_std(G11);
  std::unique_ptr<PNode> H12(temp_like(G12)), H21(temp_like(G21));
  mul_std(1.0, G11, G12, H12.get());
  mul_std(1.0, G21, G11, H21.get());
  mul_std(-1.0, H21.get(), G12, G22);
  inv_std(G22);
  zero_blocks(G12);
  mul_std(-1.0, H12.get(), G22, G12);
  zero_blocks(G21);
  mul_std(-1.0, G22, H21.get(), G21);
  mul_std(-1.0, H12.get(), G21, G11);
}

// Fig. invert: the accumulator of (t, t) is split; the off-diagonal blocks
// are flushed before use; the auxiliary products are formed by addproduct and
// flush; the Schur complement only by addproduct (the recursive call flushes
// it); the last product goes into the accumulator of (t1, t1) and is flushed
// into G11.  A leaf is flushed before its inverse is formed.
void Planner::inv_acc(PNode* G, Acc& acc) {
  if (G->kind == BLK_DENSE) {
    flush(acc, G);
    emit_lu(G, LEAF_INVERSE);
    return;
  }
  need_binary(G);
  PNode *G11 = G->son(0, 0), *G12 = G->son(0, 1), *G21 = G->son(1, 0), *G22 = G->son(1, 1);
  std::vector<Acc> a = split(acc);
  acc.has = false;
  acc.P.clear();
  Acc &a11 = a[0], &a12 = a[1], &a21 = a[2], &a22 = a[3];
  inv_acc(G11, a11);
  flush(a12, G12);
  flush(a21, G21);
  std::unique_ptr<PNode> H12(temp_like(G12)), H21(temp_like(G21));
  addproduct(1.0, G11, G12, a12);
  flush(a12, H12.get());
  addproduct(1.0, G21, G11, a21);
  flush(a21, H21.get());
  addproduct(-1.0, H21.get(), G12, a22);
  inv_acc(G22, a22);
  zero_blocks(G12);
  zero_blocks(G21);
  addproduct(-1.0, H12.get(), G22, a12);
  flush(a12, G12);
  addproduct(-1.0, G22, H21.get(), a21);
  flush(a21, G21);
  addproduct(-1.0, H12.get(), G21, a11);
  flush(a11, G11);
}

void Planner::inv(PNode* G, int mode) {
  fused_ = mode == MODE_FUSED;
  if (mode == MODE_STANDARD) {
    inv_std(G);
  } else {
    Acc acc;
    acc.t = G->t;
    acc.r = G->s;
    acc.rows = G->rows;
    acc.cols = G->cols;
    inv_acc(G, acc);
  }
}

// ---------------------------------------------------------------- H-Cholesky
// Low-rank form of X|_{t x s} (Y|_{r x s})^T when X or Y is a leaf: the four
// branches of Fig. addproduct applied to Y^T (the factors of Y exchanged).
Planner::LR Planner::lowrank_product_t(PNode* X, PNode* Y) {
  LR p;
  const int nt = X->rows, ns = X->cols, nr = Y->rows;
  counts.products++;
  if (X->kind == BLK_DENSE) {
    if (nt <= ns) {  // A = I, B = Y N_X^T
      p.k = {nt, -1};
      p.A = ident(nt);
      p.B = temp_view(nr, p.k);
      View W = nview(X);  // N_X^T as an #s x #t operand
      W.trans = 1;
      W.rows = ns;
      W.cols = {nt, -1};
      addeval(1.0, Y, W, p.B, false);
    } else {  // A = N_X, B = Y I
      p.k = {ns, -1};
      p.A = nview(X);
      p.B = temp_view(nr, p.k);
      addeval(1.0, Y, ident(ns), p.B, false);
    }
  } else if (Y->kind == BLK_DENSE) {
    if (nr <= ns) {  // B = I, A = X N_Y^T
      p.k = {nr, -1};
      p.B = ident(nr);
      p.A = temp_view(nt, p.k);
      View W = nview(Y);  // N_Y^T as an #s x #r operand
      W.trans = 1;
      W.rows = ns;
      W.cols = {nr, -1};
      addeval(1.0, X, W, p.A, false);
    } else {  // B = N_Y, A = X I
      p.k = {ns, -1};
      p.B = nview(Y);
      p.A = temp_view(nt, p.k);
      addeval(1.0, X, ident(ns), p.A, false);
    }
  } else if (X->kind == BLK_RK) {  // A = A_X, B = Y B_X
    p.k = {X->cap, X->objR};
    p.A = aview(X);
    if (X->cap == 0) return p;
    p.B = temp_view(nr, p.k);
    addeval(1.0, Y, bview(X), p.B, false);
  } else {  // Y admissible leaf: A = X B_Y, B = A_Y
    p.k = {Y->cap, Y->objR};
    p.B = aview(Y);
    if (Y->cap == 0) return p;
    p.A = temp_view(nt, p.k);
    addeval(1.0, X, bview(Y), p.A, false);
  }
  return p;
}

// Z <- blocktrunc(Z + alpha X Y^T), standard algorithm.
void Planner::mul_t_std(double alpha, PNode* X, PNode* Y, PNode* Z) {
  if (leaf(X) || leaf(Y)) {
    LR p = lowrank_product_t(X, Y);
    rkupdate(alpha, p, Z);
    return;
  }
  const bool temps = leaf(Z);
  if (temps) make_temps(Z);
  for (int i = 0; i < X->nt; ++i)
    for (int j = 0; j < Y->nt; ++j)
      for (int l = 0; l < X->ns; ++l) mul_t_std(alpha, X->son(i, l), Y->son(j, l), Z->son(i, j));
  if (temps) merge_temps(Z);
}

// rkupdate of a diagonal block (t, t): its lower blocks only.
void Planner::rkupdate_lower(double alpha, const LR& p, PNode* Z) {
  if (p.k.stat == 0) return;
  if (leaf(Z)) {
    rkupdate(alpha, p, Z);
    return;
  }
  for (int i = 0; i < Z->nt; ++i)
    for (int j = 0; j <= i; ++j) {
      PNode* b = Z->son(i, j);
      LR q;
      q.A = p.A.rows_sub(b->roff - Z->roff, b->rows);
      q.B = p.B.rows_sub(b->coff - Z->coff, b->cols);
      q.k = p.k;
      if (i == j)
        rkupdate_lower(alpha, q, b);
      else
        rkupdate(alpha, q, b);
    }
}

// Z = (t, t) <- Z + alpha X X^T on its lower blocks, standard algorithm.
void Planner::symmul_std(double alpha, PNode* X, PNode* Z) {
  if (leaf(X)) {
    LR p = lowrank_product_t(X, X);
    rkupdate_lower(alpha, p, Z);
    return;
  }
  for (int i = 0; i < X->nt; ++i)
    for (int j = 0; j <= i; ++j)
      for (int l = 0; l < X->ns; ++l) {
        if (i == j)
          symmul_std(alpha, X->son(i, l), Z->son(i, i));
        else
          mul_t_std(alpha, X->son(i, l), X->son(j, l), Z->son(i, j));
      }
}

// X (#t x c) <- L_tt^{-1} X with the lower Cholesky factor of (t, t).
void Planner::solve_Lc(PNode* L, const View& X) {
  if (X.cols.stat == 0) return;
  if (L->kind == BLK_DENSE) {
    emit_trsm(nview(L), X, L->rows, TRSM_LC);
    return;
  }
  PNode *L00 = L->son(0, 0), *L10 = L->son(1, 0), *L11 = L->son(1, 1);
  View X0 = X.rows_sub(0, L00->rows), X1 = X.rows_sub(L00->rows, L11->rows);
  solve_Lc(L00, X0);
  addeval(-1.0, L10, X0, X1, true);
  solve_Lc(L11, X1);
}

// Leaf X (r x t) <- X L^{-T}: X^T <- L^{-1} X^T (dense), B <- L^{-1} B.
void Planner::rsolve_t_leaf(PNode* L, PNode* X) {
  if (X->kind == BLK_DENSE) {
    View v = nview(X);  // X^T: #t x #r
    v.trans = 1;
    v.rows = X->cols;
    v.cols = {X->rows, -1};
    solve_Lc(L, v);
  } else if (X->cap > 0) {
    solve_Lc(L, bview(X));
  }
}

void Planner::rsolve_t_std(PNode* L, PNode* X) {
  if (leaf(X)) {
    rsolve_t_leaf(L, X);
    return;
  }
  need_binary(L);
  for (int i = 0; i < X->nt; ++i) {
    rsolve_t_std(L->son(0, 0), X->son(i, 0));
    mul_t_std(-1.0, X->son(i, 0), L->son(1, 0), X->son(i, 1));
    rsolve_t_std(L->son(1, 1), X->son(i, 1));
  }
}

// chol(t) = chol(t0); G10 <- G10 L00^{-T}; G11 <- G11 - G10 G10^T (lower
// blocks); chol(t1).
void Planner::chol_std(PNode* G) {
  if (G->kind == BLK_DENSE) {
    emit_lu(G, LEAF_CHOLESKY);
    return;
  }
  need_binary(G);
  chol_std(G->son(0, 0));
  rsolve_t_std(G->son(0, 0), G->son(1, 0));
  symmul_std(-1.0, G->son(1, 0), G->son(1, 1));
  chol_std(G->son(1, 1));
}

// addproduct for X Y^T.
void Planner::addproduct_t(double alpha, PNode* X, PNode* Y, Acc& acc) {
  counts.addproduct++;
  if (leaf(X) || leaf(Y)) {
    acc_add(alpha, lowrank_product_t(X, Y), acc);
  } else {
    acc.P.push_back({alpha, X, Y, true});
    counts.pending++;
  }
}

// Split of the accumulator of a diagonal block (t, t) into its lower sons
// (t0, t0), (t1, t0), (t1, t1), in that order.
std::vector<Planner::Acc> Planner::split_lower(Acc& acc) {
  const Cluster& ct = ct_.c[acc.t];
  std::vector<Acc> out;
  for (int i = 0; i < ct.nsons; ++i)
    for (int j = 0; j <= i; ++j) {
      Acc a;
      a.t = ct.son[i];
      a.r = ct.son[j];
      a.rows = ct_.c[a.t].size;
      a.cols = ct_.c[a.r].size;
      if (acc.has) {
        a.cap = std::max(acc.cap, std::min(std::min(a.rows, a.cols), kmax_));
        a.objA = P_.add_temp((int64_t)a.rows * std::max(a.cap, 1), a.rows);
        a.objB = P_.add_temp((int64_t)a.cols * std::max(a.cap, 1), a.cols);
        a.objR = P_.add_temp(1, 1, true);
        a.has = true;
        Dim k{acc.cap, acc.objR};
        emit_copy(aview(acc).rows_sub(ct_.c[a.t].off - ct.off, a.rows), aview(a), {a.rows, -1}, k, acc.objR, a.objR,
                  COPY_COPY);
        emit_copy(bview(acc).rows_sub(ct_.c[a.r].off - ct.off, a.cols), bview(a), {a.cols, -1}, k, -1, -1, COPY_COPY);
      }
      add_restricted(acc, i, j, a);
      out.push_back(std::move(a));
    }
  return out;
}

void Planner::rsolve_t_acc(PNode* L, PNode* X, Acc& acc) {
  if (leaf(X)) {
    flush(acc, X);
    rsolve_t_leaf(L, X);
    return;
  }
  need_binary(L);
  std::vector<Acc> a = split(acc);
  acc.has = false;
  acc.P.clear();
  for (int i = 0; i < X->nt; ++i) {
    rsolve_t_acc(L->son(0, 0), X->son(i, 0), a[(size_t)i * X->ns]);
    addproduct_t(-1.0, X->son(i, 0), L->son(1, 0), a[(size_t)i * X->ns + 1]);
    rsolve_t_acc(L->son(1, 1), X->son(i, 1), a[(size_t)i * X->ns + 1]);
  }
}

void Planner::chol_acc(PNode* G, Acc& acc) {
  if (G->kind == BLK_DENSE) {
    flush(acc, G);
    emit_lu(G, LEAF_CHOLESKY);
    return;
  }
  need_binary(G);
  std::vector<Acc> a = split_lower(acc);
  acc.has = false;
  acc.P.clear();
  chol_acc(G->son(0, 0), a[0]);
  rsolve_t_acc(G->son(0, 0), G->son(1, 0), a[1]);
  addproduct_t(-1.0, G->son(1, 0), G->son(1, 0), a[2]);
  chol_acc(G->son(1, 1), a[2]);
}

void Planner::chol(PNode* G, int mode) {
  fused_ = mode == MODE_FUSED;
  if (mode == MODE_STANDARD) {
    chol_std(G);
  } else {
    Acc acc;
    acc.t = G->t;
    acc.r = G->s;
    acc.rows = G->rows;
    acc.cols = G->cols;
    chol_acc(G, acc);
  }
}

void Planner::lu(PNode* G, int mode) {
  fused_ = mode == MODE_FUSED;
  if (mode == MODE_STANDARD) {
    lu_std(G);
  } else {
    Acc acc;
    acc.t = G->t;
    acc.r = G->s;
    acc.rows = G->rows;
    acc.cols = G->cols;
    lu_acc(G, acc);
  }
}

}  // namespace hm
