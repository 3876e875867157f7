// C ABI: builds from a source description (sparse, stencil or kernel matrix),
// options, rank override, context statistics and truncation batches whose
// descriptors live in device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <unordered_map>
#include <vector>

#include "../../include/hm.h"
#include "api_internal.h"
#include "build_kernels.h"

using namespace hm;

namespace {

// Relative tolerance of the slice truncations that compress an admissible
// kernel block before its final truncation at the build tolerance, and the
// rank capacity of the compressed slices.
constexpr double kSliceTol = 1e-12;
constexpr int kSliceCap = 256;
constexpr int kSliceWidth = 64;
// Device memory for the dense admissible blocks evaluated at once, and for the
// truncation workspace of one launch.
constexpr int64_t kBuildBlockBudget = (int64_t)4 << 30;
constexpr int64_t kBuildWsBudget = (int64_t)2 << 30;

// The (2 dim + 1)-point Laplacian of points on an integer lattice, as CSR in
// the original index order: 2 dim on the diagonal, -1 between points at
// distance 1 (the neighbours in increasing index order).
void stencil_csr(int dim, int64_t n, const double* x, std::vector<int64_t>& rowptr, std::vector<int32_t>& colind,
                 std::vector<double>& vals) {
  std::map<std::array<int64_t, 3>, int64_t> at;
  std::vector<std::array<int64_t, 3>> key((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    std::array<int64_t, 3> k{0, 0, 0};
    for (int d = 0; d < dim; ++d) {
      const double v = x[i * dim + d];
      if (v != std::floor(v) || std::fabs(v) > 1e15)
        throw std::invalid_argument("hm_build: stencil sources need integer lattice coordinates");
      k[d] = (int64_t)v;
    }
    if (!at.emplace(k, i).second) throw std::invalid_argument("hm_build: two points at the same lattice site");
    key[(size_t)i] = k;
  }
  rowptr.assign((size_t)n + 1, 0);
  colind.clear();
  vals.clear();
  for (int64_t i = 0; i < n; ++i) {
    std::vector<int64_t> nb;
    for (int d = 0; d < dim; ++d)
      for (int s = -1; s <= 1; s += 2) {
        std::array<int64_t, 3> k = key[(size_t)i];
        k[d] += s;
        auto it = at.find(k);
        if (it != at.end()) nb.push_back(it->second);
      }
    nb.push_back(i);
    std::sort(nb.begin(), nb.end());
    for (int64_t j : nb) {
      colind.push_back((int32_t)j);
      vals.push_back(j == i ? 2.0 * dim : -1.0);
    }
    rowptr[(size_t)i + 1] = (int64_t)colind.size();
  }
}

struct DevBuf {
  AllocRef alloc;
  void* p = nullptr;
  DevBuf(const AllocRef& a, size_t bytes) : alloc(a) { check(alloc->get(&p, bytes), "allocate(build)"); }
  ~DevBuf() { alloc->put(p); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  template <class T>
  T* as() const {
    return (T*)p;
  }
};

// One truncation item with a single part (A B^T, A m x k, B n x k) into (C, D)
// of capacity cap.
void one_part_item(std::vector<DTrunc>& dt, std::vector<DTruncPart>& dp, double* C, double* D, int* rank, int m, int n,
                   int cap, const DTruncPart& part, int level) {
  DTrunc d{};
  d.C = C;
  d.D = D;
  d.rank = rank;
  d.m = m;
  d.n = n;
  d.ldc = m;
  d.ldd = n;
  d.cap = cap;
  d.part0 = (int)dp.size();
  d.nparts = 1;
  d.lmax = part.k.stat;
  d.flags = 0;
  d.log_idx = (int)dt.size();
  d.level = level;
  d.kfix = -1;
  dp.push_back(part);
  dt.push_back(d);
}

// Runs the items in groups whose truncation workspace stays within the budget.
int run_items_bounded(hm_ctx* ctx, std::vector<DTrunc>& dt, std::vector<DTruncPart>& dp, double eps) {
  int bits = 0;
  size_t i = 0;
  while (i < dt.size()) {
    int64_t ws = 0;
    size_t j = i;
    while (j < dt.size() && (j == i || ws + trunc_ws_doubles(dt[j].m, dt[j].n, dt[j].lmax) * 8 <= kBuildWsBudget)) {
      ws += trunc_ws_doubles(dt[j].m, dt[j].n, dt[j].lmax) * 8;
      ++j;
    }
    std::vector<DTrunc> part(dt.begin() + i, dt.begin() + j);
    bits |= run_trunc_items(ctx, part, dp, eps, HM_FP64, nullptr, nullptr, nullptr, nullptr);
    i = j;
  }
  return bits;
}

// Kernel matrix 1/|x_i - x_j| (diagonal `diag`): dense leaves evaluated on the
// device; every admissible block evaluated densely and truncated at eps.  A
// block with min(m, n) <= 64 is truncated in one item (its dense block as a
// factor pair with an identity).  A larger block is cut into 64-column
// slices, each truncated at kSliceTol, and the slices are merged pairwise by
// truncations at kSliceTol up to one factor pair of the whole block, which is
// then truncated at eps.
void build_kernel_matrix(hm_ctx* ctx, DevHMatrix& M, const double* x, int dim, double diag, double eps,
                         const double* tri9, int layer) {
  const ClusterTree& ct = *M.ct;
  const int64_t n = (int64_t)ct.perm.size();
  // two distinct points at one place would give an infinite entry
  if (!tri9) {
    std::vector<std::array<double, 3>> pts((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
      std::array<double, 3> p{0.0, 0.0, 0.0};
      for (int d = 0; d < dim; ++d) p[d] = x[i * dim + d];
      pts[(size_t)i] = p;
    }
    std::sort(pts.begin(), pts.end());
    if (std::adjacent_find(pts.begin(), pts.end()) != pts.end())
      throw std::invalid_argument("hm_build: two points at the same place (the kernel is infinite there)");
  }
  const AllocRef& al = ctx->alloc;
  std::unique_ptr<DevBuf> tridev;
  if (tri9) {
    std::vector<double> table((size_t)n * BEM_TRI_DOUBLES);
    bem_triangle_table(tri9, ct.perm.data(), n, table.data());
    for (int64_t p = 0; p < n; ++p) {
      const double* nrm = table.data() + (size_t)p * BEM_TRI_DOUBLES + 28;
      if (!(std::fabs(nrm[0]) + std::fabs(nrm[1]) + std::fabs(nrm[2]) > 0.5))
        throw std::invalid_argument("hm_build: a degenerate triangle (zero area)");
    }
    tridev = std::make_unique<DevBuf>(al, table.size() * sizeof(double));
    check(hipMemcpyAsync(tridev->p, table.data(), table.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream),
          "upload triangles");
    check(hipStreamSynchronize(ctx->stream), "upload triangles");
  }
  std::vector<double> xs((size_t)n * dim);
  for (int64_t p = 0; p < n; ++p)
    for (int d = 0; d < dim; ++d) xs[(size_t)d * n + p] = x[(int64_t)ct.perm[p] * dim + d];
  DevBuf xdev(al, xs.size() * sizeof(double));
  check(hipMemcpyAsync(xdev.p, xs.data(), xs.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream),
        "upload points");
  std::vector<double> ident((size_t)kSliceWidth * kSliceWidth, 0.0);
  for (int q = 0; q < kSliceWidth; ++q) ident[(size_t)q * (kSliceWidth + 1)] = 1.0;
  DevBuf idev(al, ident.size() * sizeof(double));
  check(hipMemcpyAsync(idev.p, ident.data(), ident.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream),
        "upload identity");
  auto eval = [&](const std::vector<KEvalTile>& tiles) {
    if (tiles.empty()) return;
    DevBuf tdev(al, tiles.size() * sizeof(KEvalTile));
    check(hipMemcpyAsync(tdev.p, tiles.data(), tiles.size() * sizeof(KEvalTile), hipMemcpyHostToDevice, ctx->stream),
          "upload tiles");
    if (tri9)
      check(launch_bem_eval(tdev.as<KEvalTile>(), (int64_t)tiles.size(), tridev->as<double>(), layer, ctx->stream),
            "boundary-element evaluation");
    else
      check(launch_kmat_eval(tdev.as<KEvalTile>(), (int64_t)tiles.size(), xdev.as<double>(), n, dim, diag,
                             ctx->stream),
            "kernel evaluation");
    check(hipStreamSynchronize(ctx->stream), "kernel evaluation");
  };
  auto add_tiles = [&](std::vector<KEvalTile>& tiles, double* out, int ro, int co, int m, int nn) {
    for (int c0 = 0; c0 < nn; c0 += 64)
      for (int r0 = 0; r0 < m; r0 += 64) tiles.push_back({out, m, ro, co, m, nn, r0, c0, 0});
  };
  // dense leaves
  {
    std::vector<KEvalTile> tiles;
    for (size_t i = 0; i < M.bt.b.size(); ++i) {
      const Block& b = M.bt.b[i];
      if (b.kind != BLK_DENSE) continue;
      add_tiles(tiles, M.N[i], ct.c[b.t].off, ct.c[b.s].off, ct.c[b.t].size, ct.c[b.s].size);
    }
    eval(tiles);
  }
  // admissible blocks, in groups that fit the budget
  std::vector<size_t> adm;
  for (size_t i = 0; i < M.bt.b.size(); ++i)
    if (M.bt.b[i].kind == BLK_RK) adm.push_back(i);
  size_t g0 = 0;
  int bits = 0;
  while (g0 < adm.size()) {
    size_t g1 = g0;
    int64_t elems = 0;
    while (g1 < adm.size()) {
      const Block& b = M.bt.b[adm[g1]];
      const int64_t e = (int64_t)ct.c[b.t].size * ct.c[b.s].size;
      if (g1 > g0 && (elems + e) * 8 > kBuildBlockBudget) break;
      elems += e;
      ++g1;
    }
    DevBuf dbuf(al, (size_t)elems * sizeof(double));
    std::vector<double*> Dptr;
    {
      std::vector<KEvalTile> tiles;
      int64_t o = 0;
      for (size_t q = g0; q < g1; ++q) {
        const Block& b = M.bt.b[adm[q]];
        double* D = dbuf.as<double>() + o;
        Dptr.push_back(D);
        add_tiles(tiles, D, ct.c[b.t].off, ct.c[b.s].off, ct.c[b.t].size, ct.c[b.s].size);
        o += (int64_t)ct.c[b.t].size * ct.c[b.s].size;
      }
      eval(tiles);
    }
    // slices of the blocks with min(m, n) > 64: (A, B, rank, columns, capacity)
    struct Piece {
      double* A;
      double* B;
      int* rank;
      int cols, cap;
    };
    std::vector<std::vector<Piece>> pieces(g1 - g0);
    std::vector<std::unique_ptr<DevBuf>> keep;  // storage of the current and the previous level
    // level 0: one truncation per slice
    {
      std::vector<DTrunc> dt;
      std::vector<DTruncPart> dp;
      int64_t doubles = 0, ints = 0;
      for (size_t q = g0; q < g1; ++q) {
        const Block& b = M.bt.b[adm[q]];
        const int m = ct.c[b.t].size, nn = ct.c[b.s].size;
        if (std::min(m, nn) <= kSliceWidth) continue;
        for (int c0 = 0; c0 < nn; c0 += kSliceWidth) {
          const int w = std::min(kSliceWidth, nn - c0), cap = std::min(m, w);
          doubles += (int64_t)(m + w) * cap;
          ++ints;
        }
      }
      if (ints > 0) {
        keep.push_back(std::make_unique<DevBuf>(al, (size_t)doubles * sizeof(double)));
        keep.push_back(std::make_unique<DevBuf>(al, (size_t)ints * sizeof(int)));
        double* pd = keep[keep.size() - 2]->as<double>();
        int* pr = keep.back()->as<int>();
        for (size_t q = g0; q < g1; ++q) {
          const Block& b = M.bt.b[adm[q]];
          const int m = ct.c[b.t].size, nn = ct.c[b.s].size;
          if (std::min(m, nn) <= kSliceWidth) continue;
          for (int c0 = 0; c0 < nn; c0 += kSliceWidth) {
            const int w = std::min(kSliceWidth, nn - c0), cap = std::min(m, w);
            Piece pc{pd, pd + (int64_t)m * cap, pr, w, cap};
            pd += (int64_t)(m + w) * cap;
            ++pr;
            DTruncPart u{};
            u.A = Dptr[q - g0] + (int64_t)c0 * m;
            u.B = idev.as<double>();
            u.alpha = 1.0;
            u.lda = m;
            u.ldb = kSliceWidth;
            u.rows = m;
            u.cols = w;
            u.k = {w, 0, nullptr};
            one_part_item(dt, dp, pc.A, pc.B, pc.rank, m, w, cap, u, ct.c[b.t].level);
            pieces[q - g0].push_back(pc);
          }
        }
        bits |= run_items_bounded(ctx, dt, dp, kSliceTol);
      }
    }
    // merge levels: neighbouring slices pairwise
    for (;;) {
      std::vector<DTrunc> dt;
      std::vector<DTruncPart> dp;
      int64_t doubles = 0, ints = 0;
      for (size_t q = g0; q < g1; ++q) {
        const Block& b = M.bt.b[adm[q]];
        const int m = ct.c[b.t].size;
        const auto& P = pieces[q - g0];
        for (size_t j = 0; j + 1 < P.size(); j += 2) {
          const int w = P[j].cols + P[j + 1].cols;
          doubles += (int64_t)(m + w) * std::min(std::min(m, w), kSliceCap);
          ++ints;
        }
      }
      if (ints == 0) break;
      auto bd = std::make_unique<DevBuf>(al, (size_t)doubles * sizeof(double));
      auto bi = std::make_unique<DevBuf>(al, (size_t)ints * sizeof(int));
      double* pd = bd->as<double>();
      int* pr = bi->as<int>();
      std::vector<std::vector<Piece>> next(g1 - g0);
      for (size_t q = g0; q < g1; ++q) {
        const Block& b = M.bt.b[adm[q]];
        const int m = ct.c[b.t].size;
        const auto& P = pieces[q - g0];
        for (size_t j = 0; j < P.size(); j += 2) {
          if (j + 1 == P.size()) {
            next[q - g0].push_back(P[j]);  // odd slice: carried to the next level
            continue;
          }
          const int w = P[j].cols + P[j + 1].cols, cap = std::min(std::min(m, w), kSliceCap);
          Piece pc{pd, pd + (int64_t)m * cap, pr, w, cap};
          pd += (int64_t)(m + w) * cap;
          ++pr;
          DTrunc d{};
          d.C = pc.A;
          d.D = pc.B;
          d.rank = pc.rank;
          d.m = m;
          d.n = w;
          d.ldc = m;
          d.ldd = w;
          d.cap = cap;
          d.part0 = (int)dp.size();
          d.nparts = 2;
          d.lmax = P[j].cap + P[j + 1].cap;
          d.flags = 0;
          d.log_idx = (int)dt.size();
          d.level = ct.c[b.t].level;
          d.kfix = -1;
          for (int h = 0; h < 2; ++h) {
            const Piece& s = P[j + h];
            DTruncPart u{};
            u.A = s.A;
            u.B = s.B;
            u.alpha = 1.0;
            u.lda = m;
            u.ldb = s.cols;
            u.row_off = 0;
            u.rows = m;
            u.col_off = h == 0 ? 0 : P[j].cols;
            u.cols = s.cols;
            u.k = {s.cap, 0, s.rank};
            dp.push_back(u);
          }
          dt.push_back(d);
          next[q - g0].push_back(pc);
        }
      }
      bits |= run_items_bounded(ctx, dt, dp, kSliceTol);
      pieces.swap(next);
      // the carried slices may live in any earlier level's storage: keep it all
      keep.push_back(std::move(bd));
      keep.push_back(std::move(bi));
    }
    // final truncation at eps into the matrix
    {
      std::vector<DTrunc> dt;
      std::vector<DTruncPart> dp;
      for (size_t q = g0; q < g1; ++q) {
        const size_t i = adm[q];
        const Block& b = M.bt.b[i];
        const int m = ct.c[b.t].size, nn = ct.c[b.s].size;
        DTruncPart u{};
        u.alpha = 1.0;
        u.rows = m;
        u.cols = nn;
        if (std::min(m, nn) > kSliceWidth) {
          const Piece& s = pieces[q - g0][0];
          u.A = s.A;
          u.B = s.B;
          u.lda = m;
          u.ldb = nn;
          u.k = {s.cap, 0, s.rank};
        } else if (nn <= kSliceWidth) {
          u.A = Dptr[q - g0];  // D I^T
          u.B = idev.as<double>();
          u.lda = m;
          u.ldb = kSliceWidth;
          u.k = {nn, 0, nullptr};
        } else {
          u.A = idev.as<double>();  // I (D^T)^T
          u.B = Dptr[q - g0];
          u.tb = 1;  // B(i, c) = D(c, i)
          u.lda = kSliceWidth;
          u.ldb = m;
          u.k = {m, 0, nullptr};
        }
        one_part_item(dt, dp, M.A[i], M.B[i], M.R[i], m, nn, M.cap[i], u, ct.c[b.t].level);
      }
      bits |= run_items_bounded(ctx, dt, dp, eps);
    }
    g0 = g1;
  }
  if (bits) {
    hm_status s = status_to_error(bits);
    if (s != HM_OK) throw std::runtime_error(std::string("hm_build: ") + hm_last_error());
  }
}

}  // namespace

extern "C" {

void hm_options_init(hm_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->eps = 1e-6;
  o->eta = 2.0;
  o->leaf_size = 64;
  o->kmax = 64;
  o->mode = HM_ACCUMULATED;
  o->precision = HM_FP64;
  o->schedule = -1;
  o->use_graph = 0;
  o->rank_override = nullptr;
  o->rank_override_count = 0;
}

hm_status hm_build(hm_ctx* ctx, int32_t dim, int64_t n, const double* coords, const hm_source* src,
                   const hm_options* opt, hm_matrix** out) {
  hm_options o;
  hm_options_init(&o);
  if (opt) o = *opt;
  if (!ctx || !coords || !src || !out || dim < 1 || dim > 3 || n < 1 || n > INT32_MAX || o.leaf_size < 1 ||
      o.kmax < 1 || !(o.eta > 0) || !(o.eps >= 0))
    return fail(HM_ERR_ARG, "hm_build: invalid argument");
  const double t0 = now_seconds();
  hm_status st = HM_OK;
  switch (src->kind) {
    case HM_SRC_CSR:
      if (!src->rowptr || !src->colind || !src->vals) return fail(HM_ERR_ARG, "hm_build: CSR arrays missing");
      st = hm_build_csr(ctx, dim, n, coords, src->rowptr, src->colind, src->vals, o.leaf_size, o.eta, o.kmax, out);
      break;
    case HM_SRC_STENCIL_5PT:
    case HM_SRC_STENCIL_7PT: {
      if ((src->kind == HM_SRC_STENCIL_5PT) != (dim == 2) || (src->kind == HM_SRC_STENCIL_7PT) != (dim == 3))
        return fail(HM_ERR_ARG, "hm_build: the 5-point stencil needs dim 2, the 7-point stencil dim 3");
      std::vector<int64_t> rp;
      std::vector<int32_t> ci;
      std::vector<double> v;
      st = guard([&] {
        stencil_csr(dim, n, coords, rp, ci, v);
        return HM_OK;
      });
      if (st != HM_OK) return st;
      st = hm_build_csr(ctx, dim, n, coords, rp.data(), ci.data(), v.data(), o.leaf_size, o.eta, o.kmax, out);
      break;
    }
    case HM_SRC_KERNEL_INVDIST:
    case HM_SRC_BEM_SINGLE:
    case HM_SRC_BEM_DOUBLE: {
      const bool bem = src->kind != HM_SRC_KERNEL_INVDIST;
      if (bem && (!src->tri || dim != 3)) return fail(HM_ERR_ARG, "hm_build: boundary elements need dim 3 and triangles");
      st = guard([&] {
        auto ct = build_cluster_tree(dim, n, coords, o.leaf_size);
        BlockTree bt = build_block_tree(*ct, o.eta);
        auto M = allocate(ctx->alloc, ct, bt, o.kmax, nullptr);
        build_kernel_matrix(ctx, *M, coords, dim, src->diag, o.eps, bem ? src->tri : nullptr,
                            src->kind == HM_SRC_BEM_DOUBLE ? 1 : 0);
        *out = new hm_matrix{M};
        return HM_OK;
      });
      break;
    }
    default:
      return fail(HM_ERR_ARG, "hm_build: unknown source kind");
  }
  if (st == HM_OK) {
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->builds++;
    ctx->build_seconds += now_seconds() - t0;
  }
  return st;
}

hm_status hm_plan_set_rank_override(hm_plan* plan, const int32_t* ranks, int64_t count) {
  return guard([&] {
    if (!plan || !plan->P) return fail(HM_ERR_ARG, "hm_plan_set_rank_override: NULL plan");
    if (ranks && count != (int64_t)plan->P->trunc_items())
      return fail(HM_ERR_ARG, "hm_plan_set_rank_override: " + std::to_string(count) + " ranks for " +
                                  std::to_string(plan->P->trunc_items()) + " truncation items");
    hipStream_t s = nullptr;
    check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "stream");
    hipError_t e = plan->P->set_rank_override(ranks, s);
    (void)hipStreamDestroy(s);
    check(e, "hm_plan_set_rank_override");
    return HM_OK;
  });
}

namespace {
hm_status run_with_options(hm_ctx* ctx, int kind, double alpha, hm_matrix* X, hm_matrix* Y, hm_matrix* Z,
                           const hm_options* opt, hm_run_info* info) {
  hm_options o;
  hm_options_init(&o);
  if (opt) o = *opt;
  if (!ctx || (o.schedule != -1 && o.schedule != HM_SCHEDULE_WAVES && o.schedule != HM_SCHEDULE_DATAFLOW))
    return fail(HM_ERR_ARG, "options: invalid schedule");
  const int saved = ctx->schedule;
  if (o.schedule >= 0) ctx->schedule = o.schedule;
  hm_plan* p = nullptr;
  hm_status s = kind == 0 ? hm_plan_lu(ctx, Z, o.mode, &p) : hm_plan_addmul(ctx, alpha, X, Y, Z, o.mode, &p);
  ctx->schedule = saved;
  if (s != HM_OK) return s;
  s = hm_plan_set_precision(p, o.precision);
  if (s == HM_OK && o.use_graph) s = hm_plan_use_graph(p, 1);
  if (s == HM_OK && o.rank_override) s = hm_plan_set_rank_override(p, o.rank_override, o.rank_override_count);
  if (s == HM_OK) s = hm_plan_run(ctx, p, o.eps, info);
  hm_plan_free(p);
  return s;
}
}  // namespace

hm_status hm_lu_opt(hm_ctx* ctx, hm_matrix* G, const hm_options* opt, hm_run_info* info) {
  return run_with_options(ctx, 0, 0.0, nullptr, nullptr, G, opt, info);
}

hm_status hm_addmul_opt(hm_ctx* ctx, double alpha, hm_matrix* X, hm_matrix* Y, hm_matrix* Z, const hm_options* opt,
                        hm_run_info* info) {
  return run_with_options(ctx, 1, alpha, X, Y, Z, opt, info);
}

hm_status hm_get_stats(const hm_ctx* ctx, hm_stats* out) {
  if (!ctx || !out) return fail(HM_ERR_ARG, "hm_get_stats: NULL argument");
  std::memset(out, 0, sizeof(*out));
  std::lock_guard<std::mutex> g(ctx->mu);
  out->plans = ctx->plans;
  out->plan_seconds = ctx->plan_seconds;
  out->runs = ctx->runs;
  out->run_seconds = ctx->run_seconds;
  out->truncations = ctx->truncations;
  out->trunc_bytes = ctx->trunc_bytes;
  out->builds = ctx->builds;
  out->build_seconds = ctx->build_seconds;
  out->device_bytes_in_use = ctx->alloc->in_use();
  out->device_bytes_peak = ctx->alloc->peak();
  out->device_allocations = ctx->alloc->allocations();
  return HM_OK;
}

hm_status hm_trunc_batch_device(hm_ctx* ctx, int32_t count, const hm_trunc_desc* descs, int32_t max_rows,
                                int32_t max_stack, double eps, int32_t precision, int64_t* executed) {
  return guard([&] {
    if (!ctx || count < 0 || (count > 0 && !descs) || max_rows < 1 || max_stack < 0 || !(eps >= 0) ||
        precision < HM_FP64 || precision > HM_BF16X3)
      return fail(HM_ERR_ARG, "hm_trunc_batch_device: invalid argument");
    if (executed) *executed = 0;
    if (count == 0) return HM_OK;
    const AllocRef& al = ctx->alloc;
    const int64_t per = trunc_ws_doubles(max_rows, max_rows, max_stack);
    const int64_t pool_doubles = std::max<int64_t>(per * count, 1024);
    const size_t bt = (size_t)count * sizeof(DTrunc), bp = 2 * (size_t)count * sizeof(DTruncPart);
    DevBuf buf(al, bt + bp), pool(al, (size_t)pool_doubles * sizeof(double)), counter(al, sizeof(unsigned long long)),
        done(al, sizeof(int) * (size_t)count);
    DTrunc* dt = buf.as<DTrunc>();
    DTruncPart* dp = (DTruncPart*)(buf.as<char>() + bt);
    hipStream_t s = ctx->stream;
    check(hipMemsetAsync(ctx->status, 0, STATUS_INTS * sizeof(int), s), "status reset");
    check(hipMemsetAsync(counter.p, 0, sizeof(unsigned long long), s), "counter reset");
    check(hipMemsetAsync(done.p, 0, sizeof(int) * (size_t)count, s), "done reset");
    check(launch_lower_trunc_descs(descs, count, max_rows, max_stack, dt, dp, ctx->status, s), "lower descriptors");
    check(launch_trunc_small(dt, dp, count, ctx->status, eps, nullptr, 4, nullptr, nullptr, precision, s,
                             tiny_path_enabled() ? -1 : 0),
          "small truncations");
    check(launch_trunc_tall(dt, dp, count, pool.as<double>(), pool_doubles, counter.as<int>(), ctx->status, eps,
                            nullptr, done.as<int>(), 1, s, thin_path_enabled()),
          "tall truncations");
    check(launch_trunc(dt, dp, count, pool.as<double>(), pool_doubles, counter.as<int>(), ctx->status, eps, nullptr,
                       done.as<int>(), 1, s),
          "truncations");
    int st[STATUS_INTS] = {0};
    check(hipMemcpyAsync(st, ctx->status, sizeof(st), hipMemcpyDeviceToHost, s), "status read");
    check(hipStreamSynchronize(s), "hm_trunc_batch_device");
    int64_t ex = 0, by = 0;
    std::memcpy(&ex, st + 2, sizeof(ex));
    std::memcpy(&by, st + 4, sizeof(by));
    if (executed) *executed = ex;
    {
      std::lock_guard<std::mutex> g(ctx->mu);
      ctx->truncations += ex;
      ctx->trunc_bytes += by;
    }
    if (st[0] & ST_BAD_DESC) return fail(HM_ERR_ARG, "hm_trunc_batch_device: invalid descriptor or beyond the bounds");
    return status_to_error(st[0]);
  });
}

}  // extern "C"
