// Cluster tree and block tree of an H-matrix (Defs. cluster tree and block tree).
#pragma once
#include <cstdint>
#include <memory>
#include <vector>

namespace hm {

struct Cluster {
  int off = 0, size = 0, level = 0, nsons = 0;
  int son[2] = {-1, -1};
  int parent = -1;
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
};

struct ClusterTree {
  int dim = 0;
  std::vector<int> perm;  // cluster position -> original index
  std::vector<Cluster> c; // pre-order, root = 0
  int depth() const;
};

// Geometric bisection: a cluster with more than `leaf` points and a bounding box
// of positive extent is split at the midpoint of its longest side (lowest axis on
// ties); points on or below the midpoint form the first son, in their original
// relative order.
std::shared_ptr<ClusterTree> build_cluster_tree(int dim, int64_t n, const double* x, int leaf);

enum BlockKind : int { BLK_NONLEAF = 0, BLK_RK = 1, BLK_DENSE = 2 };

struct Block {
  int t = -1, s = -1, kind = BLK_NONLEAF;
  int nt = 0, ns = 0;   // sons(t), sons(s) counts when non-leaf
  int son0 = -1;        // index of the first son (sons stored contiguously, row-major)
  int parent = -1;
};

// Block tree from (root, root): admissible iff max(diam t, diam s) <= eta dist(t, s)
// with dist > 0 (squared, on tight bounding boxes); otherwise an inadmissible
// leaf when t or s is a leaf cluster; otherwise sons(t) x sons(s) row-major.
struct BlockTree {
  std::vector<Block> b;  // root = 0; sons of a block are contiguous
};

BlockTree build_block_tree(const ClusterTree& ct, double eta);

}  // namespace hm
