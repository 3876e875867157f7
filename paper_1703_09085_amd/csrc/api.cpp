// C ABI of the library (declared in include/hm.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/hm.h"
#include "api_internal.h"

using namespace hm;

double hm::now_seconds() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

std::shared_ptr<DevHMatrix> hm::allocate(const AllocRef& alloc, std::shared_ptr<ClusterTree> ct, const BlockTree& bt,
                                     int kmax, std::vector<size_t>* dense_off) {
  auto M = std::make_shared<DevHMatrix>();
  M->alloc = alloc;
  M->ct = ct;
  M->bt = bt;
  M->kmax = kmax;
  const size_t nb = bt.b.size();
  M->N.assign(nb, nullptr);
  M->A.assign(nb, nullptr);
  M->B.assign(nb, nullptr);
  M->R.assign(nb, nullptr);
  M->cap.assign(nb, 0);
  size_t dense = 0, lowrank = 0;
  std::vector<size_t> off(nb, 0);
  int leafmax = 1;
  for (const Cluster& c : ct->c)
    if (c.nsons == 0) leafmax = std::max(leafmax, c.size);
  M->leafmax = leafmax;
  for (size_t i = 0; i < nb; ++i) {
    const Block& b = bt.b[i];
    const int r = ct->c[b.t].size, c = ct->c[b.s].size;
    if (b.kind == BLK_DENSE) {
      off[i] = dense;
      dense += (size_t)r * c;
    }
  }
  for (size_t i = 0; i < nb; ++i) {
    const Block& b = bt.b[i];
    if (b.kind != BLK_RK) continue;
    const int r = ct->c[b.t].size, c = ct->c[b.s].size;
    M->cap[i] = std::min(std::min(r, c), kmax);
    off[i] = dense + lowrank;
    lowrank += (size_t)(r + c) * M->cap[i];
  }
  const size_t total = std::max<size_t>(dense + lowrank, 1);
  M->pool_bytes = total * sizeof(double);
  check(alloc->get(&M->pool, M->pool_bytes), "allocate(matrix)");
  // unused rank capacity is never read, but is kept finite
  check(hipMemset(M->pool, 0, M->pool_bytes), "zero matrix");
  check(alloc->get(&M->ranks, sizeof(int) * std::max<size_t>(nb, 1)), "allocate(ranks)");
  check(alloc->get(&M->ident, sizeof(double) * leafmax * leafmax), "allocate(identity)");
  std::vector<double> I((size_t)leafmax * leafmax, 0.0);
  for (int q = 0; q < leafmax; ++q) I[q + (size_t)q * leafmax] = 1.0;
  check(hipMemcpy(M->ident, I.data(), I.size() * sizeof(double), hipMemcpyHostToDevice), "identity upload");
  double* base = (double*)M->pool;
  for (size_t i = 0; i < nb; ++i) {
    const Block& b = bt.b[i];
    const int r = ct->c[b.t].size;
    if (b.kind == BLK_DENSE) M->N[i] = base + off[i];
    if (b.kind == BLK_RK) {
      M->A[i] = base + off[i];
      M->B[i] = base + off[i] + (size_t)r * M->cap[i];
      M->R[i] = M->ranks + i;
    }
  }
  if (dense_off) *dense_off = off;
  return M;
}

namespace {

double now() { return now_seconds(); }

void dfs_order(const BlockTree& bt, int i, std::vector<int>& out) {
  out.push_back(i);
  const Block& b = bt.b[i];
  if (b.kind != BLK_NONLEAF) return;
  for (int q = 0; q < b.nt * b.ns; ++q) dfs_order(bt, b.son0 + q, out);
}

void fill_info(hm_run_info* info, const hm_plan* plan, double run_s, int64_t executed, int bits) {
  if (!info) return;
  std::memset(info, 0, sizeof(*info));
  info->plan_seconds = plan->plan_seconds;
  for (int q = 0; q < 3; ++q) info->plan_phase_seconds[q] = plan->phase_seconds[q];
  info->run_seconds = run_s;
  info->truncations = executed;
  info->planned_truncations = plan->P->stats.items[OP_TRUNC];
  for (int q = 0; q < 5; ++q) info->items[q] = plan->P->stats.items[q];
  info->waves = plan->P->stats.waves;
  info->launches = plan->P->stats.launches;
  info->temp_bytes = plan->P->stats.temp_bytes;
  info->workspace_bytes = plan->P->stats.ws_bytes;
  const PlanCounts& c = plan->counts;
  int64_t v[9] = {c.trunc_update, c.trunc_accum, c.trunc_merge, c.dense_updates, c.addproduct,
                  c.pending,      c.products,    c.leaf_lu,     c.merges};
  for (int q = 0; q < 9; ++q) info->counts[q] = v[q];
  info->status_bits = bits;
  info->schedule = plan->P->stats.dataflow ? HM_SCHEDULE_DATAFLOW : HM_SCHEDULE_WAVES;
}

}  // namespace

hm_status hm::status_to_error(int bits) {
  if (bits & ST_ZERO_PIVOT) return fail(HM_ERR_SINGULAR, "zero pivot in a leaf LU");
  if (bits & ST_NONFINITE) return fail(HM_ERR_NUMERIC, "non-finite values in a truncation");
  if (bits & ST_RANK_OVERFLOW) return fail(HM_ERR_NUMERIC, "a truncation needed more columns than its capacity (raise kmax)");
  if (bits & ST_WS_OVERFLOW) return fail(HM_ERR_NUMERIC, "truncation workspace pool exhausted");
  return HM_OK;
}

namespace {

bool same_structure(const DevHMatrix& a, const DevHMatrix& b) {
  return a.ct == b.ct && a.bt.b.size() == b.bt.b.size() && a.kmax == b.kmax;
}

}  // namespace

namespace {
// File format of hm_save / hm_load (little-endian, as written by this host):
// "HMATRIX1", dim, kmax (int32); n, perm[n] (int32); cluster count, clusters
// (off, size, level, nsons, son0, son1, parent as int32, lo[3], hi[3] as
// double); block count, blocks (t, s, kind, nt, ns, son0, parent as int32);
// ranks[blocks] (int32); pool doubles (int64) and the device pool (dense
// leaves, then the low-rank factors at capacity, in the layout that the
// structure and kmax fix).
constexpr char kMagic[8] = {'H', 'M', 'A', 'T', 'R', 'I', 'X', '1'};

struct File {
  FILE* f;
  explicit File(FILE* p) : f(p) {}
  ~File() {
    if (f) fclose(f);
  }
};

template <class T>
void put(FILE* f, const T* p, size_t n) {
  if (n && fwrite(p, sizeof(T), n, f) != n) throw std::runtime_error("hm_save: write failed");
}
template <class T>
void get(FILE* f, T* p, size_t n) {
  if (n && fread(p, sizeof(T), n, f) != n) throw std::invalid_argument("hm_load: file too short");
}

[[noreturn]] void bad_file(const char* what) { throw std::invalid_argument(std::string("hm_load: ") + what); }

// Everything of a checkpoint but the values.
struct FileContents {
  std::shared_ptr<ClusterTree> ct;
  BlockTree bt;
  int kmax = 0;
  std::vector<int> ranks;
  int64_t pool_doubles = 0;  // the size that the structure and kmax fix
};

// Reads the structure of a checkpoint and checks that it is one the library
// could have written: perm a permutation; the cluster tree rooted at 0 with
// every son after its father, the sons' ranges splitting the father's; every
// non-leaf block (t, s) with sons(t) x sons(s) stored row-major after it;
// every block reached once from the root; ranks within capacity.  The planner
// and the tree walks rely on all of this (a cycle or a son out of range would
// make them recurse without end or index out of bounds).  Leaves the file
// positioned at the values.
void read_structure(FILE* f, FileContents& fc) {
  char magic[8];
  get(f, magic, 8);
  if (std::memcmp(magic, kMagic, 8) != 0) bad_file("not an H-matrix file");
  int32_t hdr[2];
  get(f, hdr, 2);
  int64_t n = 0, nc = 0, nbl = 0;
  get(f, &n, 1);
  if (hdr[0] < 1 || hdr[0] > 3 || hdr[1] < 1 || n < 1 || n > INT32_MAX) bad_file("bad header");
  auto ct = std::make_shared<ClusterTree>();
  ct->dim = hdr[0];
  ct->perm.resize((size_t)n);
  get(f, ct->perm.data(), ct->perm.size());
  {
    std::vector<char> seen((size_t)n, 0);
    for (int p : ct->perm) {
      if (p < 0 || p >= n || seen[p]) bad_file("perm is not a permutation");
      seen[p] = 1;
    }
  }
  get(f, &nc, 1);
  if (nc < 1 || nc > 2 * n) bad_file("bad cluster count");
  ct->c.resize((size_t)nc);
  for (Cluster& c : ct->c) {
    int32_t v[7];
    get(f, v, 7);
    c.off = v[0], c.size = v[1], c.level = v[2], c.nsons = v[3], c.son[0] = v[4], c.son[1] = v[5], c.parent = v[6];
    get(f, c.lo, 3);
    get(f, c.hi, 3);
  }
  for (int64_t i = 0; i < nc; ++i) {
    const Cluster& c = ct->c[i];
    if (c.off < 0 || c.size < 1 || (int64_t)c.off + c.size > n || c.level < 0 || c.nsons < 0 || c.nsons > 2)
      bad_file("bad cluster");
    if (i == 0 && (c.off != 0 || c.size != n || c.parent != -1 || c.level != 0)) bad_file("bad root cluster");
    if (i > 0 && (c.parent < 0 || c.parent >= i)) bad_file("bad cluster parent");
    int next = c.off;
    for (int q = 0; q < c.nsons; ++q) {
      const int so = c.son[q];
      if (so <= i || so >= nc) bad_file("cluster son out of range");
      const Cluster& d = ct->c[so];
      if (d.parent != i || d.off != next || d.level != c.level + 1) bad_file("cluster son inconsistent");
      next += d.size;
    }
    if (c.nsons > 0 && next != c.off + c.size) bad_file("cluster sons do not split their father");
  }
  get(f, &nbl, 1);
  if (nbl < 1 || nbl > (int64_t)1 << 31) bad_file("bad block count");
  BlockTree bt;
  bt.b.resize((size_t)nbl);
  for (Block& b : bt.b) {
    int32_t v[7];
    get(f, v, 7);
    b.t = v[0], b.s = v[1], b.kind = v[2], b.nt = v[3], b.ns = v[4], b.son0 = v[5], b.parent = v[6];
  }
  std::vector<char> reached((size_t)nbl, 0);
  reached[0] = 1;
  for (int64_t i = 0; i < nbl; ++i) {
    const Block& b = bt.b[i];
    if (b.t < 0 || b.t >= nc || b.s < 0 || b.s >= nc || b.kind < BLK_NONLEAF || b.kind > BLK_DENSE)
      bad_file("bad block");
    if (i == 0 && (b.t != 0 || b.s != 0 || b.parent != -1)) bad_file("bad root block");
    if (!reached[i]) bad_file("block not reached from the root");
    if (b.kind != BLK_NONLEAF) continue;
    const Cluster &t = ct->c[b.t], &s = ct->c[b.s];
    if (t.nsons < 1 || s.nsons < 1 || b.nt != t.nsons || b.ns != s.nsons) bad_file("block sons do not match the clusters");
    if (b.son0 <= i || (int64_t)b.son0 + b.nt * b.ns > nbl) bad_file("block son out of range");
    for (int a = 0; a < b.nt; ++a)
      for (int c = 0; c < b.ns; ++c) {
        const int64_t q = (int64_t)b.son0 + a * b.ns + c;
        const Block& d = bt.b[q];
        if (reached[q] || d.parent != i || d.t != t.son[a] || d.s != s.son[c]) bad_file("block son inconsistent");
        reached[q] = 1;
      }
  }
  fc.ranks.resize((size_t)nbl);
  get(f, fc.ranks.data(), fc.ranks.size());
  get(f, &fc.pool_doubles, 1);
  // the layout of allocate(): dense leaves, then factors at capacity
  int64_t expect = 0;
  for (int64_t i = 0; i < nbl; ++i) {
    const Block& b = bt.b[i];
    const int64_t r = ct->c[b.t].size, c = ct->c[b.s].size;
    const int cap = (int)std::min<int64_t>(std::min(r, c), hdr[1]);
    if (b.kind == BLK_DENSE) expect += r * c;
    if (b.kind == BLK_RK) expect += (r + c) * cap;
    const int rk = fc.ranks[i];
    if (rk < 0 || rk > (b.kind == BLK_RK ? cap : 0)) bad_file("bad rank");
  }
  if (fc.pool_doubles != std::max<int64_t>(expect, 1)) bad_file("values do not match the structure");
  fc.ct = ct;
  fc.bt = std::move(bt);
  fc.kmax = hdr[1];
}
}  // namespace

extern "C" {

const char* hm_version(void) { return "hm-gfx950 0.1"; }

const char* hm_last_error(void) { return g_err.c_str(); }

hm_status hm_ctx_create_with_allocator(void* hip_stream, hm_alloc_fn alloc, hm_free_fn free_fn, void* user,
                                       hm_ctx** out) {
  return guard([&] {
    if (!out || (!alloc) != (!free_fn)) return fail(HM_ERR_ARG, "hm_ctx_create: invalid argument");
    auto* c = new hm_ctx;
    c->stream = (hipStream_t)hip_stream;
    c->alloc = alloc ? std::make_shared<DevAlloc>(alloc, free_fn, user) : std::make_shared<DevAlloc>();
    hipError_t e = c->alloc->get(&c->status, STATUS_INTS * sizeof(int));
    if (e != hipSuccess) {
      delete c;
      return fail(HM_ERR_HIP, std::string("allocate(status): ") + hipGetErrorString(e));
    }
    *out = c;
    return HM_OK;
  });
}

hm_status hm_ctx_create(void* hip_stream, hm_ctx** out) {
  return hm_ctx_create_with_allocator(hip_stream, nullptr, nullptr, nullptr, out);
}

hm_status hm_schedule_check(int32_t dim, int32_t side, int32_t leaf_size, double eta, int32_t kmax, int32_t mode,
                            int32_t schedule, int64_t* out) {
  return guard([&] {
    if (dim < 1 || dim > 3 || side < 1 || leaf_size < 1 || !(eta > 0) || kmax < 1 || mode < 0 || mode > 2 ||
        (schedule != HM_SCHEDULE_WAVES && schedule != HM_SCHEDULE_DATAFLOW) || !out)
      return fail(HM_ERR_ARG, "hm_schedule_check: invalid argument");
    int64_t n = 1;
    for (int d = 0; d < dim; ++d) n *= side;
    if (n > (int64_t)1 << 22) return fail(HM_ERR_ARG, "hm_schedule_check: grid too large");
    std::vector<double> x((size_t)n * dim);
    for (int64_t i = 0; i < n; ++i) {
      int64_t r = i;
      for (int d = 0; d < dim; ++d) {
        x[(size_t)i * dim + d] = (double)(r % side);
        r /= side;
      }
    }
    // the structure of an H-matrix with placeholder addresses: the plan is
    // recorded and scheduled, never uploaded or run, so no address is used
    DevHMatrix M;
    M.ct = build_cluster_tree(dim, n, x.data(), leaf_size);
    M.bt = build_block_tree(*M.ct, eta);
    M.kmax = kmax;
    const size_t nb = M.bt.b.size();
    M.N.assign(nb, nullptr);
    M.A.assign(nb, nullptr);
    M.B.assign(nb, nullptr);
    M.R.assign(nb, nullptr);
    M.cap.assign(nb, 0);
    M.leafmax = 1;
    for (const auto& c : M.ct->c)
      if (c.nsons == 0) M.leafmax = std::max(M.leafmax, c.size);
    uintptr_t next = 0x10000;
    auto placeholder = [&]() { return (next += 4096); };
    for (size_t i = 0; i < nb; ++i) {
      const Block& b = M.bt.b[i];
      const int r = M.ct->c[b.t].size, c = M.ct->c[b.s].size;
      if (b.kind == BLK_DENSE) M.N[i] = reinterpret_cast<double*>(placeholder());
      if (b.kind == BLK_RK) {
        M.cap[i] = std::min(std::min(r, c), kmax);
        M.A[i] = reinterpret_cast<double*>(placeholder());
        M.B[i] = reinterpret_cast<double*>(placeholder());
        M.R[i] = reinterpret_cast<int*>(placeholder());
      }
    }
    M.ident = reinterpret_cast<double*>(placeholder());
    struct Release {  // the destructor must not free the placeholders
      DevHMatrix& m;
      ~Release() {
        m.pool = nullptr;
        m.ranks = nullptr;
        m.ident = nullptr;
      }
    } release{M};
    Program P;
    P.schedule = schedule;
    Planner pl(P, *M.ct, M.kmax, M.ident, M.leafmax);
    auto root = pl.attach(M);
    pl.lu(root.get(), mode);
    P.finalize(0);
    P.verify_schedule(out);
    return HM_OK;
  });
}

hm_status hm_set_schedule(hm_ctx* ctx, int32_t schedule) {
  if (!ctx || (schedule != HM_SCHEDULE_WAVES && schedule != HM_SCHEDULE_DATAFLOW))
    return fail(HM_ERR_ARG, "hm_set_schedule: invalid argument");
  ctx->schedule = schedule;
  return HM_OK;
}

void hm_ctx_destroy(hm_ctx* ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  ctx->alloc->put(ctx->status);
  delete ctx;
}

hm_status hm_build_csr(hm_ctx* ctx, int32_t dim, int64_t n, const double* x, const int64_t* rowptr,
                       const int32_t* colind, const double* vals, int32_t leaf_size, double eta, int32_t kmax,
                       hm_matrix** out) {
  return guard([&] {
    if (!ctx || !x || !rowptr || !colind || !vals || !out || n < 1 || n > INT32_MAX || leaf_size < 1 || kmax < 1 ||
        !(eta > 0))
      return fail(HM_ERR_ARG, "hm_build_csr: invalid argument");
    auto ct = build_cluster_tree(dim, n, x, leaf_size);
    BlockTree bt = build_block_tree(*ct, eta);
    std::vector<size_t> off;
    auto M = allocate(ctx->alloc, ct, bt, kmax, &off);
    const size_t nb = bt.b.size();
    std::vector<int> inv(n);
    for (int64_t i = 0; i < n; ++i) inv[ct->perm[i]] = (int)i;
    size_t dense_total = 0;
    for (size_t i = 0; i < nb; ++i)
      if (bt.b[i].kind == BLK_DENSE)
        dense_total += (size_t)ct->c[bt.b[i].t].size * ct->c[bt.b[i].s].size;
    std::vector<double> host(dense_total, 0.0);
    std::vector<int> ranks(nb, 0);
    for (size_t i = 0; i < nb; ++i) {
      const Block& b = bt.b[i];
      if (b.kind == BLK_NONLEAF) continue;
      const Cluster &ctc = ct->c[b.t], &csc = ct->c[b.s];
      std::vector<std::pair<int, std::pair<int, double>>> nz;  // admissible entries (col, row, val)
      for (int r = 0; r < ctc.size; ++r) {
        const int gi = ct->perm[ctc.off + r];
        for (int64_t e = rowptr[gi]; e < rowptr[gi + 1]; ++e) {
          const int pj = inv[colind[e]];
          if (pj < csc.off || pj >= csc.off + csc.size) continue;
          if (b.kind == BLK_DENSE)
            host[off[i] + r + (size_t)(pj - csc.off) * ctc.size] += vals[e];
          else if (vals[e] != 0.0)
            nz.push_back({pj - csc.off, {r, vals[e]}});
        }
      }
      if (b.kind == BLK_RK && !nz.empty()) {
        std::vector<int> cols;
        for (auto& q : nz) cols.push_back(q.first);
        std::sort(cols.begin(), cols.end());
        cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
        const int k = (int)cols.size();
        if (k > M->cap[i]) return fail(HM_ERR_ARG, "admissible block entries exceed the rank capacity");
        std::vector<double> A((size_t)ctc.size * M->cap[i], 0.0), B((size_t)csc.size * M->cap[i], 0.0);
        for (int q = 0; q < k; ++q) B[cols[q] + (size_t)q * csc.size] = 1.0;
        for (auto& q : nz) {
          const int c = (int)(std::lower_bound(cols.begin(), cols.end(), q.first) - cols.begin());
          A[q.second.first + (size_t)c * ctc.size] += q.second.second;
        }
        check(hipMemcpy(M->A[i], A.data(), A.size() * 8, hipMemcpyHostToDevice), "upload A");
        check(hipMemcpy(M->B[i], B.data(), B.size() * 8, hipMemcpyHostToDevice), "upload B");
        ranks[i] = k;
      }
    }
    if (dense_total) check(hipMemcpy(M->pool, host.data(), dense_total * 8, hipMemcpyHostToDevice), "upload dense");
    check(hipMemcpy(M->ranks, ranks.data(), nb * sizeof(int), hipMemcpyHostToDevice), "upload ranks");
    *out = new hm_matrix{M};
    return HM_OK;
  });
}

hm_status hm_clone(hm_ctx* ctx, const hm_matrix* src, hm_matrix** out) {
  return guard([&] {
    if (!ctx || !src || !out) return fail(HM_ERR_ARG, "hm_clone: NULL argument");
    auto M = allocate(ctx->alloc, src->M->ct, src->M->bt, src->M->kmax, nullptr);
    check(hipMemcpy(M->pool, src->M->pool, M->pool_bytes, hipMemcpyDeviceToDevice), "copy pool");
    check(hipMemcpy(M->ranks, src->M->ranks, sizeof(int) * std::max<size_t>(M->bt.b.size(), 1),
                    hipMemcpyDeviceToDevice),
          "copy ranks");
    *out = new hm_matrix{M};
    return HM_OK;
  });
}

hm_status hm_save(hm_ctx* ctx, const hm_matrix* m, const char* path) {
  return guard([&] {
    if (!ctx || !m || !path) return fail(HM_ERR_ARG, "hm_save: NULL argument");
    const DevHMatrix& M = *m->M;
    check(hipStreamSynchronize(ctx->stream), "hm_save: synchronize");
    const size_t nb = M.bt.b.size();
    std::vector<int> ranks(nb, 0);
    if (nb) check(hipMemcpy(ranks.data(), M.ranks, nb * sizeof(int), hipMemcpyDeviceToHost), "hm_save: ranks");
    const int64_t pool_doubles = (int64_t)(M.pool_bytes / sizeof(double));
    std::vector<double> pool((size_t)pool_doubles);
    check(hipMemcpy(pool.data(), M.pool, M.pool_bytes, hipMemcpyDeviceToHost), "hm_save: values");
    File out(fopen(path, "wb"));
    if (!out.f) return fail(HM_ERR_ARG, std::string("hm_save: cannot open ") + path);
    const ClusterTree& ct = *M.ct;
    put(out.f, kMagic, 8);
    const int32_t hdr[2] = {ct.dim, M.kmax};
    put(out.f, hdr, 2);
    const int64_t n = (int64_t)ct.perm.size(), nc = (int64_t)ct.c.size(), nbl = (int64_t)nb;
    put(out.f, &n, 1);
    put(out.f, ct.perm.data(), ct.perm.size());
    put(out.f, &nc, 1);
    for (const Cluster& c : ct.c) {
      const int32_t v[7] = {c.off, c.size, c.level, c.nsons, c.son[0], c.son[1], c.parent};
      put(out.f, v, 7);
      put(out.f, c.lo, 3);
      put(out.f, c.hi, 3);
    }
    put(out.f, &nbl, 1);
    for (const Block& b : M.bt.b) {
      const int32_t v[7] = {b.t, b.s, b.kind, b.nt, b.ns, b.son0, b.parent};
      put(out.f, v, 7);
    }
    put(out.f, ranks.data(), nb);
    put(out.f, &pool_doubles, 1);
    put(out.f, pool.data(), pool.size());
    if (fflush(out.f) != 0) return fail(HM_ERR_ARG, "hm_save: write failed");
    return HM_OK;
  });
}

hm_status hm_load(hm_ctx* ctx, const char* path, hm_matrix** out) {
  return guard([&] {
    if (!ctx || !path || !out) return fail(HM_ERR_ARG, "hm_load: NULL argument");
    FileContents fc;
    File in(fopen(path, "rb"));
    if (!in.f) return fail(HM_ERR_ARG, std::string("hm_load: cannot open ") + path);
    read_structure(in.f, fc);  // throws std::invalid_argument (HM_ERR_ARG) on a bad file
    auto M = allocate(ctx->alloc, fc.ct, fc.bt, fc.kmax, nullptr);
    if (fc.pool_doubles != (int64_t)(M->pool_bytes / sizeof(double)))
      return fail(HM_ERR_ARG, "hm_load: values do not match the structure");
    std::vector<double> pool((size_t)fc.pool_doubles);
    get(in.f, pool.data(), pool.size());
    check(hipMemcpy(M->pool, pool.data(), M->pool_bytes, hipMemcpyHostToDevice), "hm_load: values");
    check(hipMemcpy(M->ranks, fc.ranks.data(), fc.ranks.size() * sizeof(int), hipMemcpyHostToDevice),
          "hm_load: ranks");
    *out = new hm_matrix{M};
    return HM_OK;
  });
}

hm_status hm_file_info(const char* path, int64_t* n, int32_t* nclusters, int32_t* nblocks) {
  return guard([&] {
    if (!path) return fail(HM_ERR_ARG, "hm_file_info: NULL path");
    FileContents fc;
    File in(fopen(path, "rb"));
    if (!in.f) return fail(HM_ERR_ARG, std::string("hm_file_info: cannot open ") + path);
    read_structure(in.f, fc);
    // the values must follow in full, and nothing after them
    const long at = ftell(in.f);
    if (at < 0 || fseek(in.f, 0, SEEK_END) != 0) return fail(HM_ERR_ARG, "hm_file_info: cannot seek");
    const long end = ftell(in.f);
    if (end - at != (long)(fc.pool_doubles * (int64_t)sizeof(double)))
      return fail(HM_ERR_ARG, "hm_file_info: the values do not match the structure");
    if (n) *n = (int64_t)fc.ct->perm.size();
    if (nclusters) *nclusters = (int32_t)fc.ct->c.size();
    if (nblocks) *nblocks = (int32_t)fc.bt.b.size();
    return HM_OK;
  });
}

hm_status hm_zeros_like(hm_ctx* ctx, const hm_matrix* src, hm_matrix** out) {
  return guard([&] {
    if (!ctx || !src || !out) return fail(HM_ERR_ARG, "hm_zeros_like: NULL argument");
    auto M = allocate(ctx->alloc, src->M->ct, src->M->bt, src->M->kmax, nullptr);
    check(hipMemset(M->pool, 0, M->pool_bytes), "zero pool");
    check(hipMemset(M->ranks, 0, sizeof(int) * std::max<size_t>(M->bt.b.size(), 1)), "zero ranks");
    *out = new hm_matrix{M};
    return HM_OK;
  });
}

hm_status hm_copy_values(hm_ctx* ctx, const hm_matrix* src, hm_matrix* dst) {
  return guard([&] {
    if (!ctx || !src || !dst || !same_structure(*src->M, *dst->M))
      return fail(HM_ERR_ARG, "hm_copy_values: structures differ");
    check(hipMemcpyAsync(dst->M->pool, src->M->pool, dst->M->pool_bytes, hipMemcpyDeviceToDevice, ctx->stream),
          "copy pool");
    check(hipMemcpyAsync(dst->M->ranks, src->M->ranks, sizeof(int) * std::max<size_t>(dst->M->bt.b.size(), 1),
                         hipMemcpyDeviceToDevice, ctx->stream),
          "copy ranks");
    check(hipStreamSynchronize(ctx->stream), "sync");
    return HM_OK;
  });
}

void hm_matrix_free(hm_matrix* m) { delete m; }

// Run-time options from the environment, schedule, upload.
static void finish_plan(hm_ctx* ctx, hm_plan* plan, double t0) {
  const char* prof = getenv("HM_PROFILE_OPS");
  const char* dbg = getenv("HM_DEBUG");
  plan->P->debug = dbg && dbg[0] == '1';
  plan->P->profile_ops = prof && prof[0] == '1';
  const char* flog = getenv("HM_FEATURE_LOG");
  plan->P->feature_logging = flog && flog[0] == '1';
  const char* tpc = getenv("HM_SMALL_TPC");
  plan->P->small_tpc = (tpc && tpc[0] == '8') ? 8 : 4;
  const char* slog = getenv("HM_TRUNC_LOG");
  plan->P->size_logging = slog && slog[0] == '1';
  plan->P->schedule = ctx->schedule;
  const char* lanes = getenv("HM_WAVE_LANES");
  plan->P->lanes = (lanes && lanes[0] == '2') ? 2 : 4;
  const double t1 = now();
  plan->P->finalize(0);
  const double t2 = now();
  {
    const ProgramStats& ps = plan->P->stats;
    char what[200];
    snprintf(what, sizeof what, "upload plan (temporaries %.3f GB, at most %.3f GB alive at once; workspace %.3f GB)",
             ps.temp_bytes / 1e9, ps.temp_live_peak / 1e9, ps.ws_bytes / 1e9);
    check(plan->P->upload(ctx->stream), what);
  }
  plan->uploaded = true;
  plan->plan_seconds = now() - t0;
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->plans++;
    ctx->plan_seconds += plan->plan_seconds;
  }
  plan->phase_seconds[0] = t1 - t0;
  plan->phase_seconds[1] = t2 - t1;
  plan->phase_seconds[2] = now() - t2;
}

static void add_counts(PlanCounts& a, const PlanCounts& b) {
  a.trunc_update += b.trunc_update;
  a.trunc_accum += b.trunc_accum;
  a.trunc_merge += b.trunc_merge;
  a.dense_updates += b.dense_updates;
  a.addproduct += b.addproduct;
  a.pending += b.pending;
  a.products += b.products;
  a.leaf_lu += b.leaf_lu;
  a.merges += b.merges;
}

// Host threads for planning: HM_PLAN_THREADS, else the hardware threads,
// at most 16.
static int plan_threads() {
  if (const char* e = getenv("HM_PLAN_THREADS"))
    if (atoi(e) > 0) return atoi(e);
  const unsigned hw = std::thread::hardware_concurrency();
  return (int)std::max(1u, std::min(hw, 16u));
}

static hm_status make_plan(hm_ctx* ctx, int kind, double alpha, hm_matrix* X, hm_matrix* Y, hm_matrix* Z,
                           int32_t mode, hm_plan** out) {
  return guard([&] {
    if (!ctx || !Z || !out || (mode < HM_STANDARD || mode > HM_ACCUMULATED_FUSED))
      return fail(HM_ERR_ARG, "plan: invalid argument");
    if (kind == 1 && (!X || !Y || X->M->ct != Z->M->ct || Y->M->ct != Z->M->ct))
      return fail(HM_ERR_ARG, "hm_addmul: X, Y and Z must share one cluster tree");
    if (kind == 1 && (X == Z || Y == Z)) return fail(HM_ERR_ARG, "hm_addmul: Z must not alias X or Y");
    const double t0 = now();
    auto plan = std::make_unique<hm_plan>();
    plan->P = std::make_unique<Program>();
    plan->P->alloc = ctx->alloc;
    plan->targets.push_back(Z->M);
    DevHMatrix& MZ = *Z->M;
    Planner pl(*plan->P, *MZ.ct, MZ.kmax, MZ.ident, MZ.leafmax);
    if (kind == 0 || kind == 2 || kind == 3) {
      plan->roots.push_back(pl.attach(MZ));
      if (kind == 0)
        pl.lu(plan->roots[0].get(), mode);
      else if (kind == 2)
        pl.inv(plan->roots[0].get(), mode);
      else
        pl.chol(plan->roots[0].get(), mode);
    } else {
      auto rz = pl.attach(MZ);
      auto rx = (X == Z) ? nullptr : pl.attach(*X->M);
      auto ry = (Y == Z || Y == X) ? nullptr : pl.attach(*Y->M);
      PNode* px = rx ? rx.get() : rz.get();
      PNode* py = ry ? ry.get() : (Y == X ? px : rz.get());
      pl.mul(alpha, px, py, rz.get(), mode);
      plan->roots.push_back(std::move(rz));
      if (rx) plan->roots.push_back(std::move(rx));
      if (ry) plan->roots.push_back(std::move(ry));
    }
    plan->counts = pl.counts;
    finish_plan(ctx, plan.get(), t0);
    *out = plan.release();
    return HM_OK;
  });
}

hm_status hm_plan_lu_solve(hm_ctx* ctx, hm_matrix* G, double* X, int64_t ldx, int32_t c, hm_plan** out) {
  return guard([&] {
    if (!ctx || !G || !out || !X || c < 1) return fail(HM_ERR_ARG, "hm_plan_lu_solve: invalid argument");
    DevHMatrix& M = *G->M;
    const int64_t n = (int64_t)M.ct->perm.size();
    if (ldx < n || ldx > INT32_MAX) return fail(HM_ERR_ARG, "hm_plan_lu_solve: ldx smaller than n");
    const double t0 = now();
    auto plan = std::make_unique<hm_plan>();
    plan->P = std::make_unique<Program>();
    plan->P->alloc = ctx->alloc;
    Planner pl(*plan->P, *M.ct, M.kmax, M.ident, M.leafmax);
    plan->roots.push_back(pl.attach(M));
    View x;
    x.obj = plan->P->add_persistent(X, ldx * (int64_t)c, (int)n);
    x.off = 0;
    x.ld = (int)ldx;
    x.trans = 0;
    x.rows = (int)n;
    x.cols = {c, -1};
    x.rlo = 0;
    pl.lu_solve(plan->roots[0].get(), x);
    finish_plan(ctx, plan.get(), t0);
    *out = plan.release();
    return HM_OK;
  });
}

hm_status hm_lu_solve(hm_ctx* ctx, hm_matrix* G, double* X, int64_t ldx, int32_t c) {
  hm_plan* p = nullptr;
  hm_status s = hm_plan_lu_solve(ctx, G, X, ldx, c, &p);
  if (s != HM_OK) return s;
  hm_run_info info;
  s = hm_plan_run(ctx, p, 0.0, &info);
  hm_plan_free(p);
  return s;
}

hm_status hm_plan_lu_batch(hm_ctx* ctx, hm_matrix* const* G, int32_t count, int32_t mode, hm_plan** out) {
  return guard([&] {
    if (!ctx || !out || count < 1 || !G || (mode < HM_STANDARD || mode > HM_ACCUMULATED_FUSED))
      return fail(HM_ERR_ARG, "hm_plan_lu_batch: invalid argument");
    for (int i = 0; i < count; ++i) {
      if (!G[i]) return fail(HM_ERR_ARG, "hm_plan_lu_batch: NULL matrix " + std::to_string(i));
      for (int j = 0; j < i; ++j)
        if (G[j]->M == G[i]->M) return fail(HM_ERR_ARG, "hm_plan_lu_batch: a matrix appears twice");
    }
    const double t0 = now();
    auto plan = std::make_unique<hm_plan>();
    plan->P = std::make_unique<Program>();
    plan->P->alloc = ctx->alloc;
    // one planner and one program per instance, recorded on parallel host
    // threads, then appended in order: the instances touch disjoint
    // objects, so the scheduler puts their independent items into the same
    // waves, exactly as if they had been recorded one after another
    const int threads = plan_threads();
    std::vector<std::unique_ptr<Program>> parts(count);
    std::vector<std::unique_ptr<PNode>> roots(count);
    std::vector<PlanCounts> counts(count);
    for (int i = 0; i < count; ++i) plan->targets.push_back(G[i]->M);
    // the largest instances are handed out first, so that the threads finish
    // together; each program keeps its place in the batch's order
    std::vector<int> by_size(count);
    for (int i = 0; i < count; ++i) by_size[i] = i;
    std::stable_sort(by_size.begin(), by_size.end(), [&](int a, int b) {
      return G[a]->M->ct->perm.size() > G[b]->M->ct->perm.size();
    });
    parallel_for(count, threads, [&](size_t k) {
      const int i = by_size[k];
      DevHMatrix& M = *G[i]->M;
      parts[i] = std::make_unique<Program>();
      Planner pl(*parts[i], *M.ct, M.kmax, M.ident, M.leafmax);
      roots[i] = pl.attach(M);
      pl.lu(roots[i].get(), mode);
      counts[i] = pl.counts;
    });
    plan->P->absorb(parts, threads);
    for (int i = 0; i < count; ++i) {
      plan->roots.push_back(std::move(roots[i]));
      add_counts(plan->counts, counts[i]);
    }
    finish_plan(ctx, plan.get(), t0);
    *out = plan.release();
    return HM_OK;
  });
}

hm_status hm_plan_lu(hm_ctx* ctx, hm_matrix* G, int32_t mode, hm_plan** out) {
  return make_plan(ctx, 0, 0.0, nullptr, nullptr, G, mode, out);
}

hm_status hm_plan_addmul(hm_ctx* ctx, double alpha, hm_matrix* X, hm_matrix* Y, hm_matrix* Z, int32_t mode,
                         hm_plan** out) {
  return make_plan(ctx, 1, alpha, X, Y, Z, mode, out);
}

hm_status hm_plan_inv(hm_ctx* ctx, hm_matrix* G, int32_t mode, hm_plan** out) {
  return make_plan(ctx, 2, 0.0, nullptr, nullptr, G, mode, out);
}

hm_status hm_plan_chol(hm_ctx* ctx, hm_matrix* G, int32_t mode, hm_plan** out) {
  return make_plan(ctx, 3, 0.0, nullptr, nullptr, G, mode, out);
}

hm_status hm_chol(hm_ctx* ctx, hm_matrix* G, double eps, int32_t mode, hm_run_info* info) {
  hm_plan* p = nullptr;
  hm_status s = hm_plan_chol(ctx, G, mode, &p);
  if (s != HM_OK) return s;
  s = hm_plan_run(ctx, p, eps, info);
  hm_plan_free(p);
  return s;
}

hm_status hm_inv(hm_ctx* ctx, hm_matrix* G, double eps, int32_t mode, hm_run_info* info) {
  hm_plan* p = nullptr;
  hm_status s = hm_plan_inv(ctx, G, mode, &p);
  if (s != HM_OK) return s;
  s = hm_plan_run(ctx, p, eps, info);
  hm_plan_free(p);
  return s;
}

hm_status hm_plan_run(hm_ctx* ctx, hm_plan* plan, double eps, hm_run_info* info) {
  return guard([&] {
    if (!ctx || !plan || !(eps >= 0)) return fail(HM_ERR_ARG, "hm_plan_run: invalid argument");
    hipEvent_t e0, e1;
    check(hipEventCreate(&e0), "event");
    check(hipEventCreate(&e1), "event");
    check(hipMemsetAsync(ctx->status, 0, STATUS_INTS * sizeof(int), ctx->stream), "status reset");
    check(hipEventRecord(e0, ctx->stream), "event record");
    plan->P->replayed = false;
    if (plan->P->debug) {
      check(plan->P->run_checked(ctx->stream, ctx->status, eps), "run");
      if (!plan->P->error.empty()) return fail(HM_ERR_NUMERIC, "debug: " + plan->P->error);
    } else if (plan->P->use_graph && !plan->P->profile_ops) {
      check(plan->P->run_graph(ctx->stream, ctx->status, eps), "graph run");
    } else {
      check(plan->P->run(ctx->stream, ctx->status, eps), "run");
    }
    check(hipEventRecord(e1, ctx->stream), "event record");
    check(hipEventSynchronize(e1), "event sync");
    float ms = 0;
    check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    int st[STATUS_INTS];
    check(hipMemcpy(st, ctx->status, sizeof(st), hipMemcpyDeviceToHost), "status read");
    int64_t executed = 0, tbytes = 0, sbytes = 0;
    std::memcpy(&executed, st + 2, sizeof(executed));
    std::memcpy(&tbytes, st + 4, sizeof(tbytes));
    std::memcpy(&sbytes, st + 6, sizeof(sbytes));
    fill_info(info, plan, ms * 1e-3, executed, st[0]);
    {
      std::lock_guard<std::mutex> g(ctx->mu);
      ctx->runs++;
      ctx->run_seconds += ms * 1e-3;
      ctx->truncations += executed;
      ctx->trunc_bytes += tbytes;
    }
    if (info) {
      info->trunc_bytes = tbytes;
      for (int q = 0; q < 5; ++q) info->op_seconds[q] = plan->P->op_seconds[q];
      info->small_trunc_bytes = sbytes;
      info->small_trunc_seconds = plan->P->small_seconds;
      info->small_trunc_launches = plan->P->small_launches;
      info->general_trunc_launches = plan->P->general_launches;
      std::memcpy(&info->predicted, st + 8, sizeof(int64_t));
      std::memcpy(&info->predicted_fallback, st + 10, sizeof(int64_t));
      info->graph_replay = plan->P->replayed ? 1 : 0;
    }
    return status_to_error(st[0]);
  });
}

namespace {
struct Snapshot {
  const DevHMatrix* M;
  void* pool;
  void* ranks;
};
struct Snapshots {
  std::vector<Snapshot> v;
  hipStream_t s;
  AllocRef alloc;
};
size_t rank_bytes(const DevHMatrix& M) { return sizeof(int) * std::max<size_t>(M.bt.b.size(), 1); }
hipError_t restore_snapshots(void* p) {
  const Snapshots& S = *(const Snapshots*)p;
  hipError_t e = hipSuccess;
  for (const Snapshot& x : S.v) {
    if (e == hipSuccess) e = hipMemcpyAsync(x.M->pool, x.pool, x.M->pool_bytes, hipMemcpyDeviceToDevice, S.s);
    if (e == hipSuccess) e = hipMemcpyAsync(x.M->ranks, x.ranks, rank_bytes(*x.M), hipMemcpyDeviceToDevice, S.s);
  }
  return e;
}
}  // namespace

hm_status hm_plan_autotune(hm_ctx* ctx, hm_plan* plan, double eps, int64_t* chosen) {
  return guard([&] {
    if (!ctx || !plan || !plan->P || plan->targets.empty() || !chosen || !(eps >= 0))
      return fail(HM_ERR_ARG, "hm_plan_autotune: invalid argument");
    Snapshots S;
    S.s = ctx->stream;
    S.alloc = ctx->alloc;
    hipError_t e = hipSuccess;
    for (const auto& t : plan->targets) {
      Snapshot x{t.get(), nullptr, nullptr};
      e = S.alloc->get(&x.pool, std::max<size_t>(t->pool_bytes, 1));
      if (e == hipSuccess) e = S.alloc->get(&x.ranks, rank_bytes(*t));
      S.v.push_back(x);
      if (e != hipSuccess) break;
      e = hipMemcpyAsync(x.pool, t->pool, t->pool_bytes, hipMemcpyDeviceToDevice, ctx->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(x.ranks, t->ranks, rank_bytes(*t), hipMemcpyDeviceToDevice, ctx->stream);
      if (e != hipSuccess) break;
    }
    if (e == hipSuccess) e = hipMemsetAsync(ctx->status, 0, STATUS_INTS * sizeof(int), ctx->stream);
    if (e == hipSuccess) e = plan->P->autotune(ctx->stream, ctx->status, eps, restore_snapshots, &S, chosen);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    int st[STATUS_INTS] = {0};
    if (e == hipSuccess) e = hipMemcpy(st, ctx->status, sizeof(st), hipMemcpyDeviceToHost);
    (void)hipStreamSynchronize(ctx->stream);
    for (const Snapshot& x : S.v) {
      S.alloc->put(x.pool);
      S.alloc->put(x.ranks);
    }
    check(e, "hm_plan_autotune");
    return status_to_error(st[0]);
  });
}

hm_status hm_plan_set_predictor(hm_plan* plan, const hm_mlp* mlp, const double* omega, int32_t oversample,
                                int32_t mode) {
  return guard([&] {
    if (!plan || !plan->P || (mlp && (!omega || oversample < 0 || (mode != 0 && mode != 1))))
      return fail(HM_ERR_ARG, "hm_plan_set_predictor: invalid argument");
    plan->P->invalidate_graph();
    if (!mlp) {
      plan->P->pred = nullptr;
      return HM_OK;
    }
    DPredictor d{};
    d.w = hm_mlp_weights(mlp);
    d.omega = omega;
    d.oversample = oversample;
    d.mode = mode;
    if (!plan->pred_dev) check(plan->P->alloc->get(&plan->pred_dev, sizeof(DPredictor)), "allocate(predictor)");
    check(hipMemcpy(plan->pred_dev, &d, sizeof(d), hipMemcpyHostToDevice), "predictor upload");
    plan->P->pred = plan->pred_dev;
    if (plan->P->feature_logging && !plan->P->feat_log) {
      const size_t bytes = sizeof(float) * 10 * std::max<size_t>(plan->P->trunc_items(), 1);
      check(plan->P->alloc->get(&plan->P->feat_log, bytes), "allocate(feature log)");
      check(hipMemset(plan->P->feat_log, 0xff, bytes), "feature log");
    }
    return HM_OK;
  });
}

int64_t hm_plan_feature_log(const hm_plan* plan, float* out, int64_t cap) {
  if (!plan || !plan->P) return -1;
  const int64_t n = (int64_t)plan->P->trunc_items();
  if (!plan->P->feat_log) return 0;
  if (out && cap > 0) {
    const int64_t k = std::min(n, cap);
    if (hipMemcpy(out, plan->P->feat_log, sizeof(float) * 10 * (size_t)k, hipMemcpyDeviceToHost) != hipSuccess)
      return -1;
  }
  return n;
}

hm_status hm_plan_set_precision(hm_plan* plan, int32_t precision) {
  if (!plan || !plan->P || precision < HM_FP64 || precision > HM_BF16X3)
    return fail(HM_ERR_ARG, "hm_plan_set_precision: invalid argument");
  plan->P->invalidate_graph();
  plan->P->prec = precision;
  return HM_OK;
}

hm_status hm_plan_use_graph(hm_plan* plan, int32_t enable) {
  if (!plan || !plan->P) return fail(HM_ERR_ARG, "hm_plan_use_graph: NULL plan");
  plan->P->use_graph = enable != 0;
  return HM_OK;
}

int64_t hm_plan_launch_log(const hm_plan* plan, double* out, int64_t cap) {
  if (!plan || !plan->P) return -1;
  const int64_t n = plan->P->launch_count();
  if (out)
    for (int64_t i = 0; i < std::min(n, cap); ++i) plan->P->launch_entry(i, out + 5 * i);
  return n;
}

int64_t hm_plan_trunc_log(const hm_plan* plan, int32_t* out, int64_t cap) {
  if (!plan || !plan->P) return -1;
  std::vector<int> v = plan->P->read_size_log();
  const int64_t n = (int64_t)v.size() / 9;
  if (out)
    for (int64_t i = 0; i < std::min(n, cap) * 9; ++i) out[i] = v[i];
  return n;
}

void hm_plan_free(hm_plan* plan) {
  if (!plan) return;
  if (plan->P) {
    plan->P->release();
    plan->P->alloc->put(plan->pred_dev);
  }
  delete plan;
}

hm_status hm_lu(hm_ctx* ctx, hm_matrix* G, double eps, int32_t mode, hm_run_info* info) {
  hm_plan* p = nullptr;
  hm_status s = hm_plan_lu(ctx, G, mode, &p);
  if (s != HM_OK) return s;
  s = hm_plan_run(ctx, p, eps, info);
  hm_plan_free(p);
  return s;
}

hm_status hm_addmul(hm_ctx* ctx, double alpha, hm_matrix* X, hm_matrix* Y, hm_matrix* Z, double eps, int32_t mode,
                    hm_run_info* info) {
  hm_plan* p = nullptr;
  hm_status s = hm_plan_addmul(ctx, alpha, X, Y, Z, mode, &p);
  if (s != HM_OK) return s;
  s = hm_plan_run(ctx, p, eps, info);
  hm_plan_free(p);
  return s;
}

}  // extern "C"

// The larger of what the two kernels claim for stacked rank at most l: the
// general kernel the stacks, the core and R_A^T U_k when they do not fit its
// LDS; the register-resident kernel the stacks, plus the TSQR parts when a
// stack is taller than one register block (at the actual rank the blocks are
// no smaller than at l, so the TSQR part is needed only if it is at l).
int64_t hm::trunc_ws_doubles(int m, int n, int l) {
  if (m <= TRUNC_SMALL_MAX && n <= TRUNC_SMALL_MAX) return 0;
  const int64_t st = (int64_t)(m + n) * l;
  const int64_t qa = std::min(m, l), qb = std::min(n, l), qm = std::max(qa, qb);
  const int64_t general = st + (qm | 1) * qm + (int64_t)l * qb;
  int64_t tall = st;
  int p2 = 8;
  while (p2 < std::min(std::max(l, 1), 64)) p2 *= 2;
  const int rb = 32 * (512 / p2);
  if (std::max(m, n) > rb) tall += 3 * 16384 + 64 * ((m + rb - 1) / rb + (n + rb - 1) / rb);
  return (std::max(general, tall) + 31) / 32 * 32;
}

int hm::run_trunc_items(hm_ctx* ctx, std::vector<DTrunc>& dt, const std::vector<DTruncPart>& dp, double eps, int prec,
                        const DPredictor* pred, int64_t* executed, int64_t* accepted, int64_t* fell_back) {
  const int count = (int)dt.size();
  if (count == 0) return 0;
  int64_t ws = 0;
  for (const DTrunc& d : dt) ws += trunc_ws_doubles(d.m, d.n, d.lmax);
  // small blocks first (dense-core kernel), then the other kernels
  std::stable_partition(dt.begin(), dt.end(),
                        [](const DTrunc& d) { return d.m <= TRUNC_SMALL_MAX && d.n <= TRUNC_SMALL_MAX; });
  int nsmall = 0;
  while (nsmall < count && dt[nsmall].m <= TRUNC_SMALL_MAX && dt[nsmall].n <= TRUNC_SMALL_MAX) ++nsmall;
  // inside them, the blocks of at most 32 x 32 first (one per wavefront)
  int ntiny = 0;
  if (tiny_path_enabled()) {
    std::stable_partition(dt.begin(), dt.begin() + nsmall, [](const DTrunc& d) { return trunc_is_tiny(d.m, d.n); });
    while (ntiny < nsmall && trunc_is_tiny(dt[ntiny].m, dt[ntiny].n)) ++ntiny;
  }
  const AllocRef& al = ctx->alloc;
  char* buf = nullptr;
  const size_t bt = dt.size() * sizeof(DTrunc), bp = std::max<size_t>(dp.size(), 1) * sizeof(DTruncPart);
  double* pool = nullptr;
  unsigned long long* counter = nullptr;
  int* done = nullptr;
  int* slog = nullptr;
  DPredictor* pdev = nullptr;
  const int64_t pool_doubles = std::max<int64_t>(ws, 1024);
  const char* logpath = getenv("HM_TRUNC_BATCH_LOG");
  hipError_t e = al->get(&buf, bt + bp);
  if (e == hipSuccess) e = al->get(&pool, (size_t)pool_doubles * sizeof(double));
  if (e == hipSuccess) e = al->get(&counter, sizeof(unsigned long long));
  if (e == hipSuccess) e = al->get(&done, sizeof(int) * (size_t)count);
  if (e == hipSuccess) e = hipMemcpyAsync(buf, dt.data(), bt, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess && !dp.empty())
    e = hipMemcpyAsync(buf + bt, dp.data(), dp.size() * sizeof(DTruncPart), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipMemsetAsync(counter, 0, sizeof(unsigned long long), ctx->stream);
  if (e == hipSuccess) e = hipMemsetAsync(done, 0, sizeof(int) * (size_t)count, ctx->stream);
  if (e == hipSuccess) e = hipMemsetAsync(ctx->status, 0, STATUS_INTS * sizeof(int), ctx->stream);
  if (e == hipSuccess && logpath) e = al->get(&slog, sizeof(int) * 8 * (size_t)count);
  if (e == hipSuccess && logpath) e = hipMemsetAsync(slog, 0xff, sizeof(int) * 8 * (size_t)count, ctx->stream);
  if (e == hipSuccess && pred) e = al->get(&pdev, sizeof(DPredictor));
  if (e == hipSuccess && pred) e = hipMemcpyAsync(pdev, pred, sizeof(DPredictor), hipMemcpyHostToDevice, ctx->stream);
  const DTrunc* dd = (const DTrunc*)buf;
  const DTruncPart* pd = (const DTruncPart*)(buf + bt);
  if (e == hipSuccess)
    e = launch_trunc_small(dd, pd, nsmall, ctx->status, eps, slog, 4, pdev, nullptr, prec, ctx->stream, ntiny);
  if (e == hipSuccess)
    e = launch_trunc_tall(dd + nsmall, pd, count - nsmall, pool, pool_doubles, (int*)counter, ctx->status, eps, slog,
                          done, 1, ctx->stream, thin_path_enabled());
  if (e == hipSuccess)
    e = launch_trunc(dd + nsmall, pd, count - nsmall, pool, pool_doubles, (int*)counter, ctx->status, eps, slog, done,
                     1, ctx->stream);
  int st[STATUS_INTS] = {0};
  if (e == hipSuccess) e = hipMemcpyAsync(st, ctx->status, sizeof(st), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (slog && e == hipSuccess) {
    std::vector<int> hl(8 * (size_t)count);
    e = hipMemcpy(hl.data(), slog, hl.size() * sizeof(int), hipMemcpyDeviceToHost);
    if (FILE* f = fopen(logpath, "wb")) {
      fwrite(hl.data(), sizeof(int), hl.size(), f);
      fclose(f);
    }
  }
  (void)hipStreamSynchronize(ctx->stream);
  al->put(buf);
  al->put(pool);
  al->put(counter);
  al->put(done);
  al->put(slog);
  al->put(pdev);
  check(e, "truncation batch");
  int64_t v = 0;
  std::memcpy(&v, st + 2, sizeof(v));
  if (executed) *executed += v;
  if (accepted) std::memcpy(accepted, st + 8, sizeof(int64_t));
  if (fell_back) std::memcpy(fell_back, st + 10, sizeof(int64_t));
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    int64_t b = 0;
    std::memcpy(&b, st + 4, sizeof(b));
    ctx->truncations += v;
    ctx->trunc_bytes += b;
  }
  return st[0];
}

namespace {

// Both batch entry points: prec is the arithmetic of the small-block
// contractions, pred (host struct, may be NULL) attaches the rank predictor to
// the small-block kernel, level is the items' level feature; the executed,
// accepted and fallen-back counts go to the last three (any may be NULL).
hm_status trunc_batch_impl(hm_ctx* ctx, int32_t count, const hm_trunc_desc* descs, double eps, int prec,
                           const DPredictor* pred, int level, int64_t* executed, int64_t* accepted,
                           int64_t* fell_back) {
  return guard([&] {
    if (!ctx || count < 0 || (count > 0 && !descs) || !(eps >= 0) || prec < HM_FP64 || prec > HM_BF16X3)
      return fail(HM_ERR_ARG, "hm_trunc_batch: invalid argument");
    if (count == 0) {
      for (int64_t* o : {executed, accepted, fell_back})
        if (o) *o = 0;
      return HM_OK;
    }
    std::vector<DTrunc> dt(count);
    std::vector<DTruncPart> dp(2 * (size_t)count);
    for (int i = 0; i < count; ++i) {
      const hm_trunc_desc& h = descs[i];
      if (h.m < 1 || h.n < 1 || h.k1 < 0 || h.k2 < 0 || h.kcap < 0 || !h.Cout || !h.Dout || !h.rank_out ||
          (h.k1 > 0 && (!h.A || !h.B || h.lda < h.m || h.ldb < h.n)) ||
          (h.k2 > 0 && (!h.C || !h.D || h.ldc < h.m || h.ldd < h.n)))
        return fail(HM_ERR_ARG, "hm_trunc_batch: invalid descriptor " + std::to_string(i));
      DTruncPart& u = dp[2 * (size_t)i];
      u = DTruncPart{};
      u.A = h.A;
      u.B = h.B;
      u.alpha = h.alpha;
      u.lda = h.lda;
      u.ldb = h.ldb;
      u.rows = h.m;
      u.cols = h.n;
      u.k = {h.k1, 0, nullptr};
      DTruncPart& z = dp[2 * (size_t)i + 1];
      z = DTruncPart{};
      z.A = h.C;
      z.B = h.D;
      z.alpha = 1.0;
      z.lda = h.ldc;
      z.ldb = h.ldd;
      z.rows = h.m;
      z.cols = h.n;
      z.k = {h.k2, 0, nullptr};
      DTrunc& d = dt[i];
      d = DTrunc{};
      d.C = h.Cout;
      d.D = h.Dout;
      d.rank = h.rank_out;
      d.m = h.m;
      d.n = h.n;
      d.ldc = h.m;
      d.ldd = h.n;
      d.cap = h.kcap;
      d.part0 = 2 * i;
      d.nparts = 2;
      d.lmax = h.k1 + h.k2;
      d.flags = TRUNC_SKIP_IF_PART0_EMPTY;
      d.log_idx = i;
      d.level = level;
      d.kfix = -1;
    }
    int64_t ex = 0;
    const int bits = run_trunc_items(ctx, dt, dp, eps, prec, pred, &ex, accepted, fell_back);
    if (executed) *executed = ex;
    return status_to_error(bits);
  });
}

}  // namespace

extern "C" {

hm_status hm_trunc_batch(hm_ctx* ctx, int32_t count, const hm_trunc_desc* descs, double eps, int32_t precision,
                         int64_t* executed) {
  return trunc_batch_impl(ctx, count, descs, eps, precision, nullptr, 0, executed, nullptr, nullptr);
}

hm_status hm_trunc_batch_predicted(hm_ctx* ctx, int32_t count, const hm_trunc_desc* descs, double eps,
                                   const hm_mlp* mlp, const double* omega, int32_t oversample, int32_t level,
                                   int64_t* counts) {
  if (!mlp || !omega || oversample < 0 || !counts)
    return fail(HM_ERR_ARG, "hm_trunc_batch_predicted: invalid argument");
  DPredictor d{};
  d.w = hm_mlp_weights(mlp);
  d.omega = omega;
  d.oversample = oversample;
  d.mode = 1;
  return trunc_batch_impl(ctx, count, descs, eps, HM_FP64, &d, level, counts, counts + 1, counts + 2);
}

int64_t hm_n(const hm_matrix* m) { return m ? (int64_t)m->M->ct->perm.size() : -1; }

hm_status hm_perm(const hm_matrix* m, int32_t* perm) {
  if (!m || !perm) return fail(HM_ERR_ARG, "hm_perm: NULL argument");
  for (size_t i = 0; i < m->M->ct->perm.size(); ++i) perm[i] = m->M->ct->perm[i];
  return HM_OK;
}

int32_t hm_num_clusters(const hm_matrix* m) { return m ? (int32_t)m->M->ct->c.size() : -1; }

hm_status hm_clusters(const hm_matrix* m, int32_t* off, int32_t* size, int32_t* level, int32_t* son0, int32_t* son1) {
  if (!m || !off || !size || !level || !son0 || !son1) return fail(HM_ERR_ARG, "hm_clusters: NULL argument");
  const auto& c = m->M->ct->c;
  for (size_t i = 0; i < c.size(); ++i) {
    off[i] = c[i].off;
    size[i] = c[i].size;
    level[i] = c[i].level;
    son0[i] = c[i].son[0];
    son1[i] = c[i].son[1];
  }
  return HM_OK;
}

int32_t hm_num_blocks(const hm_matrix* m) { return m ? (int32_t)m->M->bt.b.size() : -1; }

hm_status hm_blocks(hm_ctx* ctx, const hm_matrix* m, int32_t* t, int32_t* s, int32_t* kind, int32_t* rank,
                    int32_t* parent) {
  return guard([&] {
    if (!ctx || !m || !t || !s || !kind || !rank || !parent) return fail(HM_ERR_ARG, "hm_blocks: NULL argument");
    const BlockTree& bt = m->M->bt;
    std::vector<int> ranks(bt.b.size());
    check(hipMemcpy(ranks.data(), m->M->ranks, sizeof(int) * bt.b.size(), hipMemcpyDeviceToHost), "ranks");
    std::vector<int> order;
    dfs_order(bt, 0, order);
    std::vector<int> pos(bt.b.size());
    for (size_t q = 0; q < order.size(); ++q) pos[order[q]] = (int)q;
    for (size_t q = 0; q < order.size(); ++q) {
      const Block& b = bt.b[order[q]];
      t[q] = b.t;
      s[q] = b.s;
      kind[q] = b.kind;
      rank[q] = b.kind == BLK_RK ? ranks[order[q]] : -1;
      parent[q] = b.parent >= 0 ? pos[b.parent] : -1;
    }
    return HM_OK;
  });
}

hm_status hm_to_dense(hm_ctx* ctx, const hm_matrix* m, double* out) {
  return guard([&] {
    if (!ctx || !m || !out) return fail(HM_ERR_ARG, "hm_to_dense: NULL argument");
    const DevHMatrix& M = *m->M;
    const int64_t n = (int64_t)M.ct->perm.size();
    std::vector<double> pool(M.pool_bytes / sizeof(double));
    std::vector<int> ranks(M.bt.b.size());
    check(hipMemcpy(pool.data(), M.pool, M.pool_bytes, hipMemcpyDeviceToHost), "pool");
    check(hipMemcpy(ranks.data(), M.ranks, sizeof(int) * ranks.size(), hipMemcpyDeviceToHost), "ranks");
    std::fill(out, out + n * n, 0.0);
    const double* base = (const double*)M.pool;
    for (size_t i = 0; i < M.bt.b.size(); ++i) {
      const Block& b = M.bt.b[i];
      const Cluster &ct = M.ct->c[b.t], &cs = M.ct->c[b.s];
      if (b.kind == BLK_DENSE) {
        const double* N = pool.data() + (M.N[i] - base);
        for (int c = 0; c < cs.size; ++c)
          for (int r = 0; r < ct.size; ++r) out[(ct.off + r) + (cs.off + c) * n] = N[r + (size_t)c * ct.size];
      } else if (b.kind == BLK_RK) {
        const double* A = pool.data() + (M.A[i] - base);
        const double* B = pool.data() + (M.B[i] - base);
        const int k = std::min(ranks[i], M.cap[i]);
        for (int c = 0; c < cs.size; ++c)
          for (int r = 0; r < ct.size; ++r) {
            double v = 0;
            for (int q = 0; q < k; ++q) v += A[r + (size_t)q * ct.size] * B[c + (size_t)q * cs.size];
            out[(ct.off + r) + (cs.off + c) * n] = v;
          }
      }
    }
    return HM_OK;
  });
}

hm_status hm_block_to_dense(hm_ctx* ctx, const hm_matrix* m, int64_t block, double* out, int64_t ld) {
  return guard([&] {
    if (!ctx || !m || !out) return fail(HM_ERR_ARG, "hm_block_to_dense: NULL argument");
    const DevHMatrix& M = *m->M;
    if (block < 0 || block >= (int64_t)M.bt.b.size()) return fail(HM_ERR_ARG, "hm_block_to_dense: no such block");
    std::vector<int> order;  // pre-order position -> storage index
    dfs_order(M.bt, 0, order);
    block = order[block];
    const Block& b = M.bt.b[block];
    const Cluster &ct = M.ct->c[b.t], &cs = M.ct->c[b.s];
    if (ld < ct.size) return fail(HM_ERR_ARG, "hm_block_to_dense: ld smaller than the block's rows");
    for (int c = 0; c < cs.size; ++c) std::fill(out + (size_t)c * ld, out + (size_t)c * ld + ct.size, 0.0);
    if (b.kind == BLK_DENSE) {
      std::vector<double> N((size_t)ct.size * cs.size);
      check(hipMemcpy(N.data(), M.N[block], N.size() * sizeof(double), hipMemcpyDeviceToHost), "block");
      for (int c = 0; c < cs.size; ++c)
        for (int r = 0; r < ct.size; ++r) out[r + (size_t)c * ld] = N[r + (size_t)c * ct.size];
    } else if (b.kind == BLK_RK) {
      int rank = 0;
      check(hipMemcpy(&rank, M.R[block], sizeof(int), hipMemcpyDeviceToHost), "rank");
      const int k = std::min(rank, M.cap[block]);
      std::vector<double> A((size_t)ct.size * std::max(k, 1)), B((size_t)cs.size * std::max(k, 1));
      if (k > 0) {
        check(hipMemcpy(A.data(), M.A[block], (size_t)ct.size * k * sizeof(double), hipMemcpyDeviceToHost), "A");
        check(hipMemcpy(B.data(), M.B[block], (size_t)cs.size * k * sizeof(double), hipMemcpyDeviceToHost), "B");
      }
      for (int c = 0; c < cs.size; ++c)
        for (int r = 0; r < ct.size; ++r) {
          double v = 0;
          for (int q = 0; q < k; ++q) v += A[r + (size_t)q * ct.size] * B[c + (size_t)q * cs.size];
          out[r + (size_t)c * ld] = v;
        }
    }
    return HM_OK;
  });
}

}  // extern "C"
