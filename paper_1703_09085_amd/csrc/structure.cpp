#include "structure.h"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace hm {

int ClusterTree::depth() const {
  int d = 0;
  for (const Cluster& cl : c) d = std::max(d, cl.level);
  return d;
}

namespace {

struct Builder {
  ClusterTree& T;
  const double* x;
  int leaf;
  std::vector<int> tmp;

  int node(int off, int size, int level, int parent) {
    int id = (int)T.c.size();
    T.c.emplace_back();
    Cluster cl;
    cl.off = off;
    cl.size = size;
    cl.level = level;
    cl.parent = parent;
    for (int d = 0; d < T.dim; ++d) {
      cl.lo[d] = HUGE_VAL;
      cl.hi[d] = -HUGE_VAL;
    }
    for (int i = off; i < off + size; ++i) {
      const double* p = x + (size_t)T.perm[i] * T.dim;
      for (int d = 0; d < T.dim; ++d) {
        cl.lo[d] = std::min(cl.lo[d], p[d]);
        cl.hi[d] = std::max(cl.hi[d], p[d]);
      }
    }
    int axis = 0;
    double ext = cl.hi[0] - cl.lo[0];
    for (int d = 1; d < T.dim; ++d)
      if (cl.hi[d] - cl.lo[d] > ext) {
        ext = cl.hi[d] - cl.lo[d];
        axis = d;
      }
    T.c[id] = cl;
    if (size <= leaf || !(ext > 0)) return id;
    const double mid = 0.5 * (cl.lo[axis] + cl.hi[axis]);
    // stable partition of perm[off, off + size)
    int nl = 0;
    tmp.resize(size);
    int w = off;
    for (int i = off; i < off + size; ++i) {
      int g = T.perm[i];
      if (x[(size_t)g * T.dim + axis] <= mid)
        T.perm[w++] = g;
      else
        tmp[nl++] = g;
    }
    int nleft = w - off;
    for (int i = 0; i < nl; ++i) T.perm[w + i] = tmp[i];
    T.c[id].nsons = 2;
    int s0 = node(off, nleft, level + 1, id);
    int s1 = node(off + nleft, size - nleft, level + 1, id);
    T.c[id].son[0] = s0;
    T.c[id].son[1] = s1;
    return id;
  }
};

bool admissible(const ClusterTree& T, int t, int s, double eta) {
  const Cluster &a = T.c[t], &b = T.c[s];
  double dt = 0, ds = 0, dist = 0;
  for (int d = 0; d < T.dim; ++d) {
    double ea = a.hi[d] - a.lo[d], eb = b.hi[d] - b.lo[d];
    dt += ea * ea;
    ds += eb * eb;
    double g = std::max(0.0, std::max(b.lo[d] - a.hi[d], a.lo[d] - b.hi[d]));
    dist += g * g;
  }
  return dist > 0 && std::max(dt, ds) <= eta * eta * dist;
}

}  // namespace

std::shared_ptr<ClusterTree> build_cluster_tree(int dim, int64_t n, const double* x, int leaf) {
  if (dim < 1 || dim > 3 || n < 1 || leaf < 1) throw std::invalid_argument("bad cluster tree arguments");
  auto T = std::make_shared<ClusterTree>();
  T->dim = dim;
  T->perm.resize(n);
  for (int64_t i = 0; i < n; ++i) T->perm[i] = (int)i;
  Builder b{*T, x, leaf, {}};
  b.node(0, (int)n, 0, -1);
  return T;
}

BlockTree build_block_tree(const ClusterTree& T, double eta) {
  BlockTree bt;
  bt.b.push_back(Block{0, 0, BLK_NONLEAF, 0, 0, -1, -1});
  // breadth-first expansion keeps the sons of each block contiguous
  for (size_t i = 0; i < bt.b.size(); ++i) {
    Block blk = bt.b[i];
    if (admissible(T, blk.t, blk.s, eta)) {
      bt.b[i].kind = BLK_RK;
      continue;
    }
    const Cluster &ct = T.c[blk.t], &cs = T.c[blk.s];
    if (ct.nsons == 0 || cs.nsons == 0) {
      bt.b[i].kind = BLK_DENSE;
      continue;
    }
    bt.b[i].kind = BLK_NONLEAF;
    bt.b[i].nt = ct.nsons;
    bt.b[i].ns = cs.nsons;
    bt.b[i].son0 = (int)bt.b.size();
    for (int a = 0; a < ct.nsons; ++a)
      for (int c = 0; c < cs.nsons; ++c) bt.b.push_back(Block{ct.son[a], cs.son[c], BLK_NONLEAF, 0, 0, -1, (int)i});
  }
  return bt;
}

}  // namespace hm
