#include "program.h"

#include <algorithm>
#include <set>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <stdexcept>

namespace hm {

hipError_t launch_gemm(const DGemm* items, const DGemmTerm* terms, int count, int prec, hipStream_t s);
hipError_t launch_lu(const DLu* items, int count, int nmax, int* status, hipStream_t s);
hipError_t launch_trsm(const DTrsm* items, int count, int nmax, hipStream_t s);
hipError_t launch_copy(const DCopy* items, int count, hipStream_t s);
hipError_t launch_nan_scan(const double* p, int64_t n, int* flag, hipStream_t s);
hipError_t launch_fill_u32(unsigned int* p, int64_t n, unsigned int v, hipStream_t s);
hipError_t launch_trunc(const DTrunc* descs, const DTruncPart* parts, int count, double* pool, int64_t pool_doubles,
                        int* counter, int* status, double eps, int* size_log, const int* done, int run_id,
                        hipStream_t stream);
hipError_t launch_trunc_tall(const DTrunc* descs, const DTruncPart* parts, int count, double* pool,
                             int64_t pool_doubles, int* counter, int* status, double eps, int* size_log,
                             int* done, int run_id, hipStream_t stream);
hipError_t launch_trunc_small(const DTrunc* descs, const DTruncPart* parts, int count, int* status, double eps,
                              int* size_log, int tpc, const DPredictor* pred, float* feat_log, int prec,
                              hipStream_t stream);

int Program::add_persistent(void* ptr, int64_t elems, int rows, bool is_int) {
  Obj o;
  o.ptr = ptr;
  o.elems = elems;
  o.rows = rows;
  o.is_int = is_int;
  objs.push_back(o);
  track_.emplace_back();
  return (int)objs.size() - 1;
}

int Program::add_temp(int64_t elems, int rows, bool is_int) {
  Obj o;
  o.temp = true;
  o.elems = elems;
  o.rows = rows;
  o.is_int = is_int;
  objs.push_back(o);
  track_.emplace_back();
  return (int)objs.size() - 1;
}

int Program::record(int op, int idx, const std::vector<Region>& reads, const std::vector<Region>& writes) {
  int wave = 0;
  for (const Region& r : reads)
    for (const Access& a : track_[r.obj])
      if (a.w && a.lo < r.hi && r.lo < a.hi) wave = std::max(wave, a.wave + 1);
  for (const Region& r : writes)
    for (const Access& a : track_[r.obj])
      if (a.lo < r.hi && r.lo < a.hi) wave = std::max(wave, a.wave + 1);
  for (const Region& r : reads) {
    auto& tr = track_[r.obj];
    bool merged = false;
    for (Access& a : tr)
      if (!a.w && a.lo == r.lo && a.hi == r.hi) {
        a.wave = std::max(a.wave, wave);
        merged = true;
        break;
      }
    if (!merged) tr.push_back({wave, r.lo, r.hi, false});
  }
  for (const Region& r : writes) {
    auto& tr = track_[r.obj];
    tr.erase(std::remove_if(tr.begin(), tr.end(), [&](const Access& a) { return a.lo >= r.lo && a.hi <= r.hi; }),
             tr.end());
    tr.push_back({wave, r.lo, r.hi, true});
  }
  auto touch = [&](int o) {
    Obj& ob = objs[o];
    if (!ob.temp) return;
    if (ob.first_wave < 0 || wave < ob.first_wave) ob.first_wave = wave;
    ob.last_wave = std::max(ob.last_wave, wave);
  };
  for (const Region& r : reads) touch(r.obj);
  for (const Region& r : writes) touch(r.obj);
  Record rc{wave, (int)rec_regions_.size(), (int)reads.size(), (int)writes.size(), false};
  rec_regions_.insert(rec_regions_.end(), reads.begin(), reads.end());
  rec_regions_.insert(rec_regions_.end(), writes.begin(), writes.end());
  for (const Region& r : writes) rc.persistent_write |= !objs[r.obj].temp;
  recs_.push_back(rc);
  items.push_back({op, idx, wave, (int)recs_.size() - 1});
  nwaves = std::max(nwaves, wave + 1);
  stats.items[op]++;
  return wave;
}

void* Program::ptr_of(int obj) const {
  const Obj& o = objs[obj];
  if (!o.temp) return o.ptr;
  return arena_ + o.off;
}

namespace {
constexpr int64_t kAlign = 256;
int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }
}  // namespace

// Second scheduling pass, backwards: an operation that writes only
// temporaries (a product, a merge piece) moves to the latest wave before its
// first dependent operation, so that its temporaries live only as long as
// they are needed; operations that write the matrices keep their earliest
// wave.  The number of waves and every dependency are unchanged.  Conflicts
// are tracked as in record(), for the later operations.
void Program::schedule_late() {
  const int nrec = (int)recs_.size();
  std::vector<int> late(nrec);
  struct Late {
    int wave, lo, hi;
    bool w;
  };
  std::vector<std::vector<Late>> tr(objs.size());
  for (int i = nrec - 1; i >= 0; --i) {
    const Record& R = recs_[i];
    const Region* rd = rec_regions_.data() + R.r0;
    const Region* wr = rd + R.nr;
    int bound = nwaves;
    for (int q = 0; q < R.nr; ++q)
      for (const Late& a : tr[rd[q].obj])
        if (a.w && a.lo < rd[q].hi && rd[q].lo < a.hi) bound = std::min(bound, a.wave - 1);
    for (int q = 0; q < R.nw; ++q)
      for (const Late& a : tr[wr[q].obj])
        if (a.lo < wr[q].hi && wr[q].lo < a.hi) bound = std::min(bound, a.wave - 1);
    if (bound < R.wave) throw std::runtime_error("schedule: inconsistent dependencies");
    const int L = (R.persistent_write || bound == nwaves) ? R.wave : bound;
    late[i] = L;
    for (int q = 0; q < R.nw; ++q) {
      auto& t = tr[wr[q].obj];
      t.erase(std::remove_if(t.begin(), t.end(), [&](const Late& a) { return a.lo >= wr[q].lo && a.hi <= wr[q].hi; }),
              t.end());
      t.push_back({L, wr[q].lo, wr[q].hi, true});
    }
    for (int q = 0; q < R.nr; ++q) {
      auto& t = tr[rd[q].obj];
      bool merged = false;
      for (Late& a : t)
        if (!a.w && a.lo == rd[q].lo && a.hi == rd[q].hi) {
          a.wave = std::min(a.wave, L);
          merged = true;
          break;
        }
      if (!merged) t.push_back({L, rd[q].lo, rd[q].hi, false});
    }
  }
  for (Item& it : items) it.wave = late[it.rec];
  for (Obj& o : objs) o.first_wave = o.last_wave = -1;
  for (int i = 0; i < nrec; ++i) {
    const Record& R = recs_[i];
    for (int q = 0; q < R.nr + R.nw; ++q) {
      Obj& o = objs[rec_regions_[R.r0 + q].obj];
      if (!o.temp) continue;
      if (o.first_wave < 0 || late[i] < o.first_wave) o.first_wave = late[i];
      o.last_wave = std::max(o.last_wave, late[i]);
    }
  }
}

// Temporary memory over wave lifetimes: temporaries are placed in order of
// their first wave, best fit among the free ranges (freed ranges are merged
// with their neighbours, and a range at the end lowers the top); a
// temporary's range is free again after the last wave that uses it.  Sets the
// objects' offsets; returns the arena size.
int64_t Program::layout_temps() {
  arena_top_peak_ = 0;
  // temporaries in order of their first wave (a stable counting sort)
  std::vector<int> start(nwaves + 1, 0);
  int ntemp = 0;
  for (const Obj& o : objs)
    if (o.temp && o.first_wave >= 0) {
      start[o.first_wave + 1]++;
      ++ntemp;
    }
  for (int w = 0; w < nwaves; ++w) start[w + 1] += start[w];
  std::vector<int> temps(ntemp);
  for (int i = 0; i < (int)objs.size(); ++i)
    if (objs[i].temp && objs[i].first_wave >= 0) temps[start[objs[i].first_wave]++] = i;
  // ranges to free after each wave, in order of allocation
  std::vector<std::vector<std::pair<int64_t, int64_t>>> ends(nwaves);
  int freed = -1;                                          // waves whose ranges are free again
  std::map<int64_t, int64_t> free_off;                     // off -> size
  std::set<std::pair<int64_t, int64_t>> free_size;         // (size, off)
  int64_t top = 0, live = 0, live_peak = 0;
  auto release = [&](int64_t off, int64_t size) {
    auto nx = free_off.lower_bound(off);
    if (nx != free_off.end() && off + size == nx->first) {
      size += nx->second;
      free_size.erase({nx->second, nx->first});
      nx = free_off.erase(nx);
    }
    if (nx != free_off.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {
        off = pv->first;
        size += pv->second;
        free_size.erase({pv->second, pv->first});
        free_off.erase(pv);
      }
    }
    if (off + size == top) {
      top = off;
    } else {
      free_off[off] = size;
      free_size.insert({size, off});
    }
  };
  for (int id : temps) {
    Obj& o = objs[id];
    while (freed + 1 < o.first_wave) {
      ++freed;
      for (const auto& r : ends[freed]) {
        live -= r.second;
        release(r.first, r.second);
      }
      std::vector<std::pair<int64_t, int64_t>>().swap(ends[freed]);
    }
    const int64_t need = align_up(std::max<int64_t>(o.elems * (o.is_int ? 4 : 8), 1), kAlign);
    int64_t off;
    auto it = free_size.lower_bound({need, (int64_t)-1});
    if (it != free_size.end()) {
      off = it->second;
      const int64_t size = it->first;
      free_size.erase(it);
      free_off.erase(off);
      if (size > need) {
        free_off[off + need] = size - need;
        free_size.insert({size - need, off + need});
      }
    } else {
      off = top;
      top += need;
    }
    arena_top_peak_ = std::max(arena_top_peak_, top);
    live += need;
    live_peak = std::max(live_peak, live);
    o.off = off;
    ends[o.last_wave].push_back({off, need});
  }
  stats.temp_live_peak = live_peak;
  return arena_top_peak_;
}

void Program::finalize(int /*kmax_lds*/) {
  // 1. temporaries: the earliest-wave schedule, or, when its temporaries
  // exceed the budget (HM_TEMP_BUDGET_GB, default 64), the late schedule of
  // the operations that only write temporaries (fewer bytes alive at once,
  // more launches)
  int64_t top = layout_temps();
  const char* sched = getenv("HM_SCHEDULE");
  const char* budget_env = getenv("HM_TEMP_BUDGET_GB");
  const double budget = (budget_env && *budget_env ? atof(budget_env) : 64.0) * 1e9;
  const bool late = sched ? std::strcmp(sched, "late") == 0 : top > budget;
  if (late) {
    schedule_late();
    top = layout_temps();
  }
  stats.late_schedule = late;
  arena_bytes_ = (size_t)std::max<int64_t>(top, kAlign);
  stats.temp_bytes = top;

  // 2. order items by wave, per kind; launch list
  std::vector<std::vector<int>> per_op(OP_COUNT);
  // items in order of their wave (a stable counting sort)
  std::vector<int> item_order(items.size());
  {
    std::vector<int> first(nwaves + 1, 0);
    for (const Item& it : items) first[it.wave + 1]++;
    for (int w = 0; w < nwaves; ++w) first[w + 1] += first[w];
    for (size_t i = 0; i < items.size(); ++i) item_order[first[items[i].wave]++] = (int)i;
  }
  launches_.clear();
  size_t i = 0;
  int64_t ws_max = 0;
  while (i < item_order.size()) {
    int w = items[item_order[i]].wave;
    size_t j = i;
    int first[OP_COUNT], count[OP_COUNT];
    for (int op = 0; op < OP_COUNT; ++op) {
      first[op] = (int)per_op[op].size();
      count[op] = 0;
    }
    int64_t ws_wave = 0;
    std::vector<int> general;  // truncations for the general kernel, after the small ones
    while (j < item_order.size() && items[item_order[j]].wave == w) {
      const Item& it = items[item_order[j]];
      if (it.op == OP_TRUNC) {
        const HTrunc& t = truncs[it.idx];
        if (!trunc_is_small(t)) {
          general.push_back(it.idx);
          // the general kernel's need, or the register-resident kernel's (at
          // most (m + n) l plus four TSQR parts of 16384 doubles)
          ws_wave += align_up((int64_t)(t.m + t.n) * t.lmax + 2 * (int64_t)t.lmax * t.lmax + 4 * t.lmax + 64, 32) +
                     4 * 16384;
          ++j;
          continue;
        }
      }
      per_op[it.op].push_back(it.idx);
      count[it.op]++;
      ++j;
    }
    const int nsmall = count[OP_TRUNC];
    for (int idx : general) per_op[OP_TRUNC].push_back(idx);
    count[OP_TRUNC] += (int)general.size();
    ws_max = std::max(ws_max, ws_wave);
    static const int op_order[OP_COUNT] = {OP_COPY, OP_LU, OP_TRSM, OP_GEMM, OP_TRUNC};
    for (int q = 0; q < OP_COUNT; ++q) {
      int op = op_order[q];
      if (op == OP_TRUNC) {
        if (!general.empty()) launches_.push_back({op, first[op] + nsmall, (int)general.size(), 0, w});
        if (nsmall > 0) launches_.push_back({op, first[op], nsmall, small_tpc == 8 ? 2 : 1, w});
      } else if (count[op] > 0) {
        launches_.push_back({op, first[op], count[op], 0, w});
      }
    }
    i = j;
  }
  // workspace pool: the static bound, capped; truncations claim their actual
  // need from it on the device and flag an overflow if it runs out
  const int64_t cap = (int64_t)1 << 28;  // 2 GiB of doubles
  ws_doubles_ = (size_t)std::max<int64_t>(std::min(ws_max, cap), 1024);
  stats.ws_bytes = (int64_t)ws_doubles_ * 8;
  stats.waves = nwaves;
  stats.launches = (int64_t)launches_.size();
  emit_order_ = per_op;
  n_trunc_launches_ = 0;
  small_launches = general_launches = 0;
  for (const Launch& L : launches_) {
    if (L.op == OP_TRUNC && L.variant == 0) n_trunc_launches_++;
    if (L.op == OP_TRUNC) (L.variant >= 1 ? small_launches : general_launches)++;
  }
}

DDim Program::ddim(const Dim& d) const {
  DDim r;
  r.stat = d.stat;
  r.pad = 0;
  r.dyn = d.rank_obj >= 0 ? (const int*)ptr_of(d.rank_obj) : nullptr;
  return r;
}

namespace {
template <class T>
size_t put(std::vector<char>& buf, const std::vector<T>& v) {
  size_t off = align_up((int64_t)buf.size(), 256);
  buf.resize(off + v.size() * sizeof(T));
  if (!v.empty()) std::memcpy(buf.data() + off, v.data(), v.size() * sizeof(T));
  return off;
}
}  // namespace

hipError_t Program::upload(hipStream_t s) {
  hipError_t e;
  if ((e = hipMalloc(&arena_, arena_bytes_)) != hipSuccess) return e;
  if ((e = hipMalloc(&ws_, ws_doubles_ * sizeof(double))) != hipSuccess) return e;
  if (debug) {
    if ((e = hipMemset(arena_, 0, arena_bytes_)) != hipSuccess) return e;
    if ((e = hipMemset(ws_, 0, ws_doubles_ * sizeof(double))) != hipSuccess) return e;
  }
  if ((e = hipMalloc(&counters_, sizeof(unsigned long long) * (size_t)std::max(1, n_trunc_launches_))) != hipSuccess)
    return e;
  if ((e = hipMalloc(&done_, sizeof(int) * std::max<size_t>(truncs.size(), 1))) != hipSuccess) return e;
  if ((e = hipStreamCreateWithFlags(&side_, hipStreamNonBlocking)) != hipSuccess) return e;
  if ((e = hipEventCreateWithFlags(&ev_main_, hipEventDisableTiming)) != hipSuccess) return e;
  if ((e = hipEventCreateWithFlags(&ev_side_, hipEventDisableTiming)) != hipSuccess) return e;
  auto P = [&](const View& v) -> double* { return (double*)ptr_of(v.obj) + v.off; };
  std::vector<DGemmTerm> dterms(terms.size());
  for (size_t i = 0; i < terms.size(); ++i) {
    const HTerm& t = terms[i];
    DGemmTerm d;
    d.A = P(t.A);
    d.B = P(t.B);
    d.alpha = t.alpha;
    d.lda = t.A.ld;
    d.ldb = t.B.ld;
    d.ta = t.ta ^ t.A.trans;  // op() of a view whose storage is itself transposed
    d.tb = t.tb ^ t.B.trans;
    d.k = ddim(t.k);
    dterms[i] = d;
  }
  std::vector<DTruncPart> dparts(parts.size());
  for (size_t i = 0; i < parts.size(); ++i) {
    const HPart& p = parts[i];
    DTruncPart d;
    d.A = P(p.A);
    d.B = P(p.B);
    d.alpha = p.alpha;
    d.lda = p.A.ld;
    d.ldb = p.B.ld;
    d.ta = p.A.trans;
    d.tb = p.B.trans;
    d.row_off = p.row_off;
    d.rows = p.rows;
    d.col_off = p.col_off;
    d.cols = p.cols;
    d.k = ddim(p.k);
    dparts[i] = d;
  }
  std::vector<DGemm> dg;
  for (int idx : emit_order_[OP_GEMM]) {
    const HGemm& g = gemms[idx];
    DGemm d;
    d.C = P(g.C);
    d.m = ddim(g.m);
    d.n = ddim(g.C.cols);
    d.ldc = g.C.ld;
    d.ctrans = g.C.trans;
    d.beta = g.beta;
    d.pad = 0;
    d.term0 = g.term0;
    d.nterms = g.nterms;
    d.row0 = g.row0;
    d.col0 = g.col0;
    dg.push_back(d);
  }
  std::vector<DTrunc> dt;
  for (int idx : emit_order_[OP_TRUNC]) {
    const HTrunc& t = truncs[idx];
    DTrunc d;
    d.C = (double*)ptr_of(t.objA);
    d.D = (double*)ptr_of(t.objB);
    d.rank = (int*)ptr_of(t.objR);
    d.m = t.m;
    d.n = t.n;
    d.ldc = t.m;
    d.ldd = t.n;
    d.cap = t.cap;
    d.part0 = t.part0;
    d.nparts = t.nparts;
    d.lmax = t.lmax;
    d.flags = t.flags;
    d.log_idx = idx;  // record order: the order of the recursion
    d.level = t.level;
    dt.push_back(d);
  }
  std::vector<DLu> dl;
  for (int idx : emit_order_[OP_LU]) {
    const HLu& u = lus[idx];
    dl.push_back({(double*)ptr_of(u.obj), u.n, u.n});
  }
  std::vector<DTrsm> ds;
  for (int idx : emit_order_[OP_TRSM]) {
    const HTrsm& t = trsms[idx];
    DTrsm d;
    d.T = P(t.T);
    d.X = P(t.X);
    d.n = t.n;
    d.ldt = t.T.ld;
    d.ldx = t.X.ld;
    d.kind = t.kind;
    d.xtrans = t.X.trans;
    d.col0 = t.col0;
    d.c = ddim(t.X.cols);
    ds.push_back(d);
  }
  std::vector<DCopy> dc;
  for (int idx : emit_order_[OP_COPY]) {
    const HCopy& c = copies[idx];
    DCopy d;
    d.src = c.src.obj >= 0 ? P(c.src) : nullptr;
    d.dst = c.dst.obj >= 0 ? P(c.dst) : nullptr;
    d.rank_src = c.rank_src >= 0 ? (const int*)ptr_of(c.rank_src) : nullptr;
    d.rank_dst = c.rank_dst >= 0 ? (int*)ptr_of(c.rank_dst) : nullptr;
    d.alpha = c.alpha;
    d.lds = c.src.ld;
    d.ldd = c.dst.ld;
    d.strans = c.src.trans;
    d.mode = c.mode;
    d.m = ddim(c.m);
    d.n = ddim(c.n);
    dc.push_back(d);
  }
  std::vector<char> host;
  off_term_ = put(host, dterms);
  off_part_ = put(host, dparts);
  off_[OP_GEMM] = put(host, dg);
  off_[OP_TRUNC] = put(host, dt);
  off_[OP_LU] = put(host, dl);
  off_[OP_TRSM] = put(host, ds);
  off_[OP_COPY] = put(host, dc);
  desc_bytes_ = std::max<size_t>(host.size(), 256);
  stats.desc_bytes = (int64_t)desc_bytes_;
  if ((e = hipMalloc(&desc_, desc_bytes_)) != hipSuccess) return e;
  if (size_logging) {
    if ((e = hipMalloc(&size_log_, sizeof(int) * 8 * std::max<size_t>(dt.size(), 1))) != hipSuccess) return e;
    if ((e = hipMemset(size_log_, 0xff, sizeof(int) * 8 * std::max<size_t>(dt.size(), 1))) != hipSuccess) return e;
  }
  if ((e = hipMemcpyAsync(desc_, host.data(), host.size(), hipMemcpyHostToDevice, s)) != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

hipError_t Program::reset_counters(hipStream_t s) {
  hipError_t e = launch_fill_u32((unsigned int*)counters_, 2 * (int64_t)std::max(1, n_trunc_launches_), 0u, s);
  if (e == hipSuccess) e = launch_fill_u32((unsigned int*)done_, (int64_t)std::max<size_t>(truncs.size(), 1), 0u, s);
  return e;
}

hipError_t Program::run_graph(hipStream_t s, int* status, double eps) {
  // capture and replay on a stream of the plan (the caller's stream may be the
  // legacy default stream, which cannot be captured), ordered by events
  hipError_t e;
  if (!cap_) {
    if ((e = hipStreamCreateWithFlags(&cap_, hipStreamNonBlocking)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&ev_cap_, hipEventDisableTiming)) != hipSuccess) return e;
  }
  if ((e = hipEventRecord(ev_cap_, s)) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(cap_, ev_cap_, 0)) != hipSuccess) return e;
  if (!gexec_ || graph_eps_ != eps || graph_status_ != status) {
    if (gexec_) (void)hipGraphExecDestroy(gexec_);
    gexec_ = nullptr;
    if ((e = hipStreamBeginCapture(cap_, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
    const hipError_t er = run(cap_, status, eps);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cap_, &g);
    if (er != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return er;
    }
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&gexec_, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      gexec_ = nullptr;
      return e;
    }
    graph_eps_ = eps;
    graph_status_ = status;
  }
  if ((e = hipGraphLaunch(gexec_, cap_)) != hipSuccess) return e;
  if ((e = hipEventRecord(ev_cap_, cap_)) != hipSuccess) return e;
  return hipStreamWaitEvent(s, ev_cap_, 0);
}

hipError_t Program::autotune(hipStream_t s, int* status, double eps, hipError_t (*restore)(void*), void* ctx,
                             int64_t* chosen) {
  const bool saved = profile_ops;
  profile_ops = true;
  std::vector<float> t[2];
  hipError_t e = hipSuccess;
  for (int v = 0; v < 2 && e == hipSuccess; ++v) {
    for (Launch& L : launches_)
      if (L.op == OP_TRUNC && L.variant >= 1) L.variant = v + 1;
    if ((e = restore(ctx)) != hipSuccess) break;
    if ((e = run(s, status, eps)) != hipSuccess) break;
    t[v] = launch_ms;
  }
  chosen[0] = chosen[1] = 0;
  for (size_t li = 0; li < launches_.size(); ++li) {
    Launch& L = launches_[li];
    if (L.op != OP_TRUNC || L.variant < 1) continue;
    const int v = (e == hipSuccess && t[1][li] < t[0][li]) ? 1 : 0;
    L.variant = v + 1;
    chosen[v]++;
  }
  profile_ops = saved;
  if (gexec_) (void)hipGraphExecDestroy(gexec_);  // the launches changed: capture again
  gexec_ = nullptr;
  if (e == hipSuccess) e = restore(ctx);
  return e;
}

hipError_t Program::run(hipStream_t s, int* status, double eps) {
  hipError_t e = reset_counters(s);
  if (e != hipSuccess) return e;
  const DGemmTerm* terms_d = (const DGemmTerm*)(desc_ + off_term_);
  const DTruncPart* parts_d = (const DTruncPart*)(desc_ + off_part_);
  int tl = 0;
  std::vector<hipEvent_t> ev;
  if (profile_ops) {
    ev.resize(2 * launches_.size());
    for (auto& x : ev)
      if ((e = hipEventCreate(&x)) != hipSuccess) return e;
  }
  // main_dirty / side_dirty: launches not yet published by an event record;
  // side_wait / main_wait: the other stream has published work this one has
  // not waited for.  Records happen at wave boundaries only, so the launches
  // of one wave on the two streams overlap.
  bool main_dirty = true, side_dirty = false, side_wait = false, main_wait = false;
  int cur_wave = -1;
  for (size_t li = 0; li < launches_.size(); ++li) {
    const Launch& L = launches_[li];
    if (L.wave != cur_wave) {
      cur_wave = L.wave;
      if (main_dirty) {
        if ((e = hipEventRecord(ev_main_, s)) != hipSuccess) return e;
        main_dirty = false;
        side_wait = true;
      }
      if (side_dirty) {
        if ((e = hipEventRecord(ev_side_, side_)) != hipSuccess) return e;
        side_dirty = false;
        main_wait = true;
      }
    }
    const bool on_side = L.op == OP_TRUNC && L.variant >= 1;
    hipStream_t st = on_side ? side_ : s;
    if (on_side && side_wait) {
      if ((e = hipStreamWaitEvent(side_, ev_main_, 0)) != hipSuccess) return e;
      side_wait = false;
    }
    if (!on_side && main_wait) {
      if ((e = hipStreamWaitEvent(s, ev_side_, 0)) != hipSuccess) return e;
      main_wait = false;
    }
    if (profile_ops) (void)hipEventRecord(ev[2 * li], st);
    switch (L.op) {
      case OP_GEMM:
        e = launch_gemm((const DGemm*)(desc_ + off_[OP_GEMM]) + L.first, terms_d, L.count, prec, st);
        break;
      case OP_TRUNC:
        if (L.variant >= 1) {
          e = launch_trunc_small((const DTrunc*)(desc_ + off_[OP_TRUNC]) + L.first, parts_d, L.count, status, eps,
                                 size_log_, L.variant == 2 ? 8 : 4, pred, feat_log, prec, st);
        } else {
          // register-resident kernel, then the general kernel: each skips the other's items
          int* ctr = (int*)((unsigned long long*)counters_ + tl);
          e = launch_trunc_tall((const DTrunc*)(desc_ + off_[OP_TRUNC]) + L.first, parts_d, L.count, ws_,
                                (int64_t)ws_doubles_, ctr, status, eps, size_log_, done_ + L.first, 1, st);
          if (e == hipSuccess)
            e = launch_trunc((const DTrunc*)(desc_ + off_[OP_TRUNC]) + L.first, parts_d, L.count, ws_,
                             (int64_t)ws_doubles_, ctr, status, eps, size_log_, done_ + L.first, 1, st);
          tl++;
        }
        break;
      case OP_LU:
        e = launch_lu((const DLu*)(desc_ + off_[OP_LU]) + L.first, L.count, lu_nmax, status, st);
        break;
      case OP_TRSM:
        e = launch_trsm((const DTrsm*)(desc_ + off_[OP_TRSM]) + L.first, L.count, trsm_nmax, st);
        break;
      case OP_COPY:
        e = launch_copy((const DCopy*)(desc_ + off_[OP_COPY]) + L.first, L.count, st);
        break;
    }
    if (e != hipSuccess) return e;
    if (profile_ops) (void)hipEventRecord(ev[2 * li + 1], st);
    if (on_side)
      side_dirty = true;
    else
      main_dirty = true;
  }
  // the caller's stream sees the end of the side stream's work
  if (side_dirty) {
    if ((e = hipEventRecord(ev_side_, side_)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(s, ev_side_, 0)) != hipSuccess) return e;
  }
  if (profile_ops) {
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    for (int q = 0; q < OP_COUNT; ++q) op_seconds[q] = 0;
    small_seconds = 0;
    launch_ms.assign(launches_.size(), 0.0f);
    for (size_t li = 0; li < launches_.size(); ++li) {
      float ms = 0;
      (void)hipEventElapsedTime(&ms, ev[2 * li], ev[2 * li + 1]);
      op_seconds[launches_[li].op] += ms * 1e-3;
      launch_ms[li] = ms;
      if (launches_[li].op == OP_TRUNC && launches_[li].variant >= 1) small_seconds += ms * 1e-3;
    }
    for (auto& x : ev) (void)hipEventDestroy(x);
  }
  return hipSuccess;
}

hipError_t Program::run_checked(hipStream_t s, int* status, double eps) {
  hipError_t e = reset_counters(s);
  if (e != hipSuccess) return e;
  // memory spans to scan: the arena and every persistent double object
  std::vector<std::pair<const double*, int64_t>> spans;
  spans.push_back({(const double*)arena_, (int64_t)(arena_bytes_ / 8)});
  for (const Obj& o : objs)
    if (!o.temp && !o.is_int && o.ptr) spans.push_back({(const double*)o.ptr, o.elems});
  int* flag = nullptr;
  if ((e = hipMalloc(&flag, sizeof(int))) != hipSuccess) return e;
  const DGemmTerm* terms_d = (const DGemmTerm*)(desc_ + off_term_);
  const DTruncPart* parts_d = (const DTruncPart*)(desc_ + off_part_);
  int tl = 0;
  const char* names[OP_COUNT] = {"GEMM", "TRUNC", "LU", "TRSM", "COPY"};
  for (size_t li = 0; li < launches_.size(); ++li) {
    const Launch& L = launches_[li];
    switch (L.op) {
      case OP_GEMM: e = launch_gemm((const DGemm*)(desc_ + off_[OP_GEMM]) + L.first, terms_d, L.count, prec, s); break;
      case OP_TRUNC:
        if (L.variant >= 1) {
          e = launch_trunc_small((const DTrunc*)(desc_ + off_[OP_TRUNC]) + L.first, parts_d, L.count, status, eps,
                                 size_log_, L.variant == 2 ? 8 : 4, pred, feat_log, prec, s);
        } else {
          // register-resident kernel, then the general kernel: each skips the other's items
          int* ctr = (int*)((unsigned long long*)counters_ + tl);
          e = launch_trunc_tall((const DTrunc*)(desc_ + off_[OP_TRUNC]) + L.first, parts_d, L.count, ws_,
                                (int64_t)ws_doubles_, ctr, status, eps, size_log_, done_ + L.first, 1, s);
          if (e == hipSuccess)
            e = launch_trunc((const DTrunc*)(desc_ + off_[OP_TRUNC]) + L.first, parts_d, L.count, ws_,
                             (int64_t)ws_doubles_, ctr, status, eps, size_log_, done_ + L.first, 1, s);
          tl++;
        }
        break;
      case OP_LU: e = launch_lu((const DLu*)(desc_ + off_[OP_LU]) + L.first, L.count, lu_nmax, status, s); break;
      case OP_TRSM: e = launch_trsm((const DTrsm*)(desc_ + off_[OP_TRSM]) + L.first, L.count, trsm_nmax, s); break;
      case OP_COPY: e = launch_copy((const DCopy*)(desc_ + off_[OP_COPY]) + L.first, L.count, s); break;
    }
    if (e != hipSuccess) break;
    if ((e = hipMemsetAsync(flag, 0, sizeof(int), s)) != hipSuccess) break;
    for (auto& sp : spans)
      if ((e = launch_nan_scan(sp.first, sp.second, flag, s)) != hipSuccess) break;
    int h = 0;
    if ((e = hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) break;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) break;
    int stv[2] = {0, 0};
    (void)hipMemcpy(stv, status, sizeof(stv), hipMemcpyDeviceToHost);
    const int st = stv[0];
    if (h || st) {
      const char* dump = getenv("HM_DEBUG_DUMP");
      if (dump && L.op == OP_TRUNC && stv[1] > 0) {
        // replayable inputs of the failing truncation (its inputs are unchanged
        // unless it updates a block in place)
        const DTrunc* dd = (const DTrunc*)(desc_ + off_[OP_TRUNC]) + L.first + (stv[1] - 1);
        DTrunc d;
        (void)hipMemcpy(&d, dd, sizeof(d), hipMemcpyDeviceToHost);
        FILE* f = fopen(dump, "wb");
        if (f) {
          int hd[4] = {d.m, d.n, d.nparts, d.cap};
          fwrite(hd, sizeof(int), 4, f);
          fwrite(&eps, sizeof(double), 1, f);
          for (int q = 0; q < d.nparts; ++q) {
            DTruncPart P;
            (void)hipMemcpy(&P, (const DTruncPart*)(desc_ + off_part_) + d.part0 + q, sizeof(P), hipMemcpyDeviceToHost);
            int k = P.k.stat;
            if (P.k.dyn) {
              int r = 0;
              (void)hipMemcpy(&r, P.k.dyn, sizeof(int), hipMemcpyDeviceToHost);
              k = std::min(std::max(r, 0), k);
            }
            int ph[8] = {P.row_off, P.rows, P.col_off, P.cols, k, P.lda, P.ldb, P.ta * 2 + P.tb};
            fwrite(ph, sizeof(int), 8, f);
            fwrite(&P.alpha, sizeof(double), 1, f);
            std::vector<double> a((size_t)P.rows * k), b((size_t)P.cols * k);
            for (int c = 0; c < k; ++c)
              for (int r = 0; r < P.rows; ++r)
                (void)hipMemcpy(&a[r + (size_t)c * P.rows], P.ta ? P.A + c + (size_t)r * P.lda : P.A + r + (size_t)c * P.lda,
                                sizeof(double), hipMemcpyDeviceToHost);
            for (int c = 0; c < k; ++c)
              for (int r = 0; r < P.cols; ++r)
                (void)hipMemcpy(&b[r + (size_t)c * P.cols], P.tb ? P.B + c + (size_t)r * P.ldb : P.B + r + (size_t)c * P.ldb,
                                sizeof(double), hipMemcpyDeviceToHost);
            fwrite(a.data(), sizeof(double), a.size(), f);
            fwrite(b.data(), sizeof(double), b.size(), f);
          }
          fclose(f);
        }
        error += "[dumped item " + std::to_string(stv[1] - 1) + "] ";
      }
      error += "launch " + std::to_string(li) + " of " + std::to_string(launches_.size()) + " (" + names[L.op] +
              ", " + std::to_string(L.count) + " items, first item " + std::to_string(emit_order_[L.op][L.first]) +
              ") left " + (h ? "non-finite values" : "") + (st ? " status " + std::to_string(st) : "");
      if (L.op == OP_TRUNC) {
        for (int q = 0; q < std::min(L.count, 4); ++q) {
          const HTrunc& t = truncs[emit_order_[L.op][L.first + q]];
          error += "; trunc m=" + std::to_string(t.m) + " n=" + std::to_string(t.n) + " cap=" + std::to_string(t.cap) +
                   " parts=" + std::to_string(t.nparts);
          for (int pp = 0; pp < t.nparts; ++pp) {
            const HPart& hp = parts[t.part0 + pp];
            error += " [A obj " + std::to_string(hp.A.obj) + (objs[hp.A.obj].temp ? "t" : "p") + " tr" +
                     std::to_string(hp.A.trans) + " B obj " + std::to_string(hp.B.obj) +
                     (objs[hp.B.obj].temp ? "t" : "p") + " tr" + std::to_string(hp.B.trans) + " k " +
                     std::to_string(hp.k.stat) + "/" + std::to_string(hp.k.rank_obj) + " rows " +
                     std::to_string(hp.rows) + "@" + std::to_string(hp.row_off) + " cols " + std::to_string(hp.cols) +
                     "@" + std::to_string(hp.col_off) + "]";
          }
        }
      }
      break;
    }
  }
  (void)hipFree(flag);
  return e;
}

std::vector<int> Program::read_size_log() const {
  std::vector<int> out;
  if (!size_log_) return out;
  std::vector<int> dev(8 * std::max<size_t>(truncs.size(), 1));
  (void)hipMemcpy(dev.data(), size_log_, sizeof(int) * dev.size(), hipMemcpyDeviceToHost);
  // 9 ints per item: the 8 the kernel wrote, then the wave of the item
  out.assign(9 * truncs.size(), -1);
  for (size_t i = 0; i < truncs.size(); ++i)
    for (int j = 0; j < 8; ++j) out[9 * i + j] = dev[8 * i + j];
  for (const Item& it : items)
    if (it.op == OP_TRUNC) out[9 * (size_t)it.idx + 8] = it.wave;
  return out;
}

void Program::release() {
  if (gexec_) (void)hipGraphExecDestroy(gexec_);
  gexec_ = nullptr;
  if (feat_log) (void)hipFree(feat_log);
  feat_log = nullptr;
  if (cap_) {
    (void)hipStreamSynchronize(cap_);
    (void)hipStreamDestroy(cap_);
    (void)hipEventDestroy(ev_cap_);
    cap_ = nullptr;
  }
  if (side_) {
    (void)hipStreamSynchronize(side_);
    (void)hipStreamDestroy(side_);
    (void)hipEventDestroy(ev_main_);
    (void)hipEventDestroy(ev_side_);
    side_ = nullptr;
  }
  if (arena_) (void)hipFree(arena_);
  if (ws_) (void)hipFree(ws_);
  if (desc_) (void)hipFree(desc_);
  if (counters_) (void)hipFree(counters_);
  if (size_log_) (void)hipFree(size_log_);
  if (done_) (void)hipFree(done_);
  size_log_ = nullptr;
  done_ = nullptr;
  arena_ = nullptr;
  ws_ = nullptr;
  desc_ = nullptr;
  counters_ = nullptr;
}

}  // namespace hm
