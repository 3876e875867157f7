#include "program.h"

#include <algorithm>
#include <cmath>
#include <set>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <stdexcept>
#include <atomic>
#include <exception>
#include <functional>
#include <mutex>
#include <thread>

namespace hm {

// Host threads for the parallel parts of planning: the hardware threads, at
// most 16.
int host_threads() {
  const unsigned hw = std::thread::hardware_concurrency();
  return (int)std::max(1u, std::min(hw, 16u));
}

// Runs fn(0 .. n-1) on up to `threads` host threads (indices handed out in
// order); the first exception is rethrown after all threads have joined.
void parallel_for(int n, int threads, const std::function<void(size_t)>& fn) {
  threads = std::max(1, std::min(threads, n));
  if (threads == 1) {
    for (int i = 0; i < n; ++i) fn((size_t)i);
    return;
  }
  std::atomic<int> next{0};
  std::exception_ptr err;
  std::mutex mu;
  std::vector<std::thread> pool;
  for (int t = 0; t < threads; ++t)
    pool.emplace_back([&] {
      for (int i; (i = next.fetch_add(1)) < n;) {
        try {
          fn((size_t)i);
        } catch (...) {
          std::lock_guard<std::mutex> g(mu);
          if (!err) err = std::current_exception();
        }
      }
    });
  for (auto& th : pool) th.join();
  if (err) std::rethrow_exception(err);
}

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
                             int* done, int run_id, hipStream_t stream, bool thin);
hipError_t launch_trunc_small(const DTrunc* descs, const DTruncPart* parts, int count, int* status, double eps,
                              int* size_log, int tpc, const DPredictor* pred, float* feat_log, int prec,
                              hipStream_t stream, int ntiny = 0);

int Program::add_persistent(void* ptr, int64_t elems, int rows, bool is_int) {
  Obj o;
  o.ptr = ptr;
  o.elems = elems;
  o.rows = rows;
  o.is_int = is_int;
  grow4(objs);
  grow4(track_);
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
  grow4(objs);
  grow4(track_);
  objs.push_back(o);
  track_.emplace_back();
  return (int)objs.size() - 1;
}

void Program::reserve_scaled(double f) {
  auto grow = [f](auto& v) {
    const size_t want = (size_t)((double)v.size() * f) + 16;
    if (want > v.capacity()) v.reserve(want);
  };
  grow(objs);
  grow(track_);
  grow(gemms);
  grow(terms);
  grow(truncs);
  grow(parts);
  grow(lus);
  grow(trsms);
  grow(copies);
  grow(items);
  grow(recs_);
  grow(rec_regions_);
}

void Program::absorb(std::vector<std::unique_ptr<Program>>& parts_in, int threads) {
  struct Off {
    size_t obj, gemm, term, trunc, part, lu, trsm, copy, item, rec, reg;
  };
  const size_t np = parts_in.size();
  std::vector<Off> off(np + 1);
  off[0] = {objs.size(), gemms.size(), terms.size(), truncs.size(), parts.size(), lus.size(), trsms.size(),
            copies.size(), items.size(), recs_.size(), rec_regions_.size()};
  for (size_t i = 0; i < np; ++i) {
    const Program& q = *parts_in[i];
    const Off& a = off[i];
    off[i + 1] = {a.obj + q.objs.size(), a.gemm + q.gemms.size(), a.term + q.terms.size(),
                  a.trunc + q.truncs.size(), a.part + q.parts.size(), a.lu + q.lus.size(),
                  a.trsm + q.trsms.size(), a.copy + q.copies.size(), a.item + q.items.size(),
                  a.rec + q.recs_.size(), a.reg + q.rec_regions_.size()};
    nwaves = std::max(nwaves, q.nwaves);
    lu_nmax = std::max(lu_nmax, q.lu_nmax);
    trsm_nmax = std::max(trsm_nmax, q.trsm_nmax);
    for (int op = 0; op < OP_COUNT; ++op) stats.items[op] += q.stats.items[op];
  }
  // copy the parts' arrays in order (each destination's pages are touched
  // once), freeing each part's array behind it, then shift the object and
  // index references of every part's range in parallel
  const Off& e = off[np];
  auto cat = [&](auto& dst, auto member, size_t total) {
    dst.reserve(total);
    for (size_t i = 0; i < np; ++i) {
      auto& src = (*parts_in[i]).*member;
      dst.insert(dst.end(), src.begin(), src.end());
      std::remove_reference_t<decltype(src)>().swap(src);
    }
  };
  // the eleven arrays are independent: one thread each, largest first
  const std::function<void()> cats[] = {
      [&] { cat(rec_regions_, &Program::rec_regions_, e.reg); }, [&] { cat(terms, &Program::terms, e.term); },
      [&] { cat(gemms, &Program::gemms, e.gemm); },              [&] { cat(objs, &Program::objs, e.obj); },
      [&] { cat(parts, &Program::parts, e.part); },              [&] { cat(items, &Program::items, e.item); },
      [&] { cat(recs_, &Program::recs_, e.rec); },               [&] { cat(copies, &Program::copies, e.copy); },
      [&] { cat(trsms, &Program::trsms, e.trsm); },              [&] { cat(truncs, &Program::truncs, e.trunc); },
      [&] { cat(lus, &Program::lus, e.lu); }};
  parallel_for(11, threads, [&](size_t i) { cats[i](); });
  auto move_part = [&](size_t i) {
    const Off& a = off[i];
    const Off& b = off[i + 1];
    const int O = (int)a.obj;
    auto sd = [O](Dim& d) {
      if (d.rank_obj >= 0) d.rank_obj += O;
    };
    auto sv = [O, &sd](View& v) {
      if (v.obj >= 0) v.obj += O;
      sd(v.cols);
    };
    for (size_t j = a.gemm; j < b.gemm; ++j) {
      HGemm& g = gemms[j];
      sv(g.C);
      sd(g.m);
      g.term0 += (int)a.term;
    }
    for (size_t j = a.term; j < b.term; ++j) {
      HTerm& t = terms[j];
      sv(t.A);
      sv(t.B);
      sd(t.k);
    }
    for (size_t j = a.trunc; j < b.trunc; ++j) {
      HTrunc& t = truncs[j];
      t.objA += O;
      t.objB += O;
      t.objR += O;
      t.part0 += (int)a.part;
    }
    for (size_t j = a.part; j < b.part; ++j) {
      HPart& p = parts[j];
      sv(p.A);
      sv(p.B);
      sd(p.k);
    }
    for (size_t j = a.lu; j < b.lu; ++j) lus[j].obj += O;
    for (size_t j = a.trsm; j < b.trsm; ++j) {
      sv(trsms[j].T);
      sv(trsms[j].X);
    }
    for (size_t j = a.copy; j < b.copy; ++j) {
      HCopy& c = copies[j];
      sv(c.src);
      sv(c.dst);
      sd(c.m);
      sd(c.n);
      if (c.rank_src >= 0) c.rank_src += O;
      if (c.rank_dst >= 0) c.rank_dst += O;
    }
    const size_t base[OP_COUNT] = {a.gemm, a.trunc, a.lu, a.trsm, a.copy};
    for (size_t j = a.item; j < b.item; ++j) {
      Item& it = items[j];
      it.idx += (int)base[it.op];
      it.rec += (int)a.rec;
    }
    for (size_t j = a.rec; j < b.rec; ++j) recs_[j].r0 += (int)a.reg;
    for (size_t j = a.reg; j < b.reg; ++j) rec_regions_[j].obj += O;
  };
  parallel_for((int)np, threads, move_part);
  part_obj_.resize(np + 1);
  part_item_.resize(np + 1);
  for (size_t i = 0; i <= np; ++i) {
    part_obj_[i] = (int)off[i].obj;
    part_item_[i] = off[i].item;
  }
  parts_in.clear();
  std::vector<AccessList>().swap(track_);
  closed_ = true;
}

int Program::record(int op, int idx, const std::vector<Region>& reads, const std::vector<Region>& writes) {
  if (closed_) throw std::logic_error("record() after absorb()");
  int wave = 0;
  for (const Region& r : reads) {
    const AccessList& tr = track_[r.obj];
    for (int i = 0; i < tr.n; ++i) {
      const Access& a = tr.at(i);
      if (a.w && a.lo < r.hi && r.lo < a.hi) wave = std::max(wave, a.wave + 1);
    }
  }
  for (const Region& r : writes) {
    const AccessList& tr = track_[r.obj];
    for (int i = 0; i < tr.n; ++i) {
      const Access& a = tr.at(i);
      if (a.lo < r.hi && r.lo < a.hi) wave = std::max(wave, a.wave + 1);
    }
  }
  for (const Region& r : reads) {
    AccessList& tr = track_[r.obj];
    bool merged = false;
    for (int i = 0; i < tr.n; ++i) {
      Access& a = tr.at(i);
      if (!a.w && a.lo == r.lo && a.hi == r.hi) {
        a.wave = std::max(a.wave, wave);
        merged = true;
        break;
      }
    }
    if (!merged) tr.push({wave, r.lo, r.hi, false});
  }
  for (const Region& r : writes) {
    AccessList& tr = track_[r.obj];
    tr.drop_inside(r.lo, r.hi);
    tr.push({wave, r.lo, r.hi, true});
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
  grow4(rec_regions_, reads.size() + writes.size());
  rec_regions_.insert(rec_regions_.end(), reads.begin(), reads.end());
  rec_regions_.insert(rec_regions_.end(), writes.begin(), writes.end());
  for (const Region& r : writes) rc.persistent_write |= !objs[r.obj].temp;
  grow4(recs_);
  recs_.push_back(rc);
  grow4(items);
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

// Temporary memory over the lifetimes of the temporaries in nslots waves (or
// epochs): temporaries are placed in order of their first wave, best fit among the free ranges (freed ranges are merged
// with their neighbours, and a range at the end lowers the top); a
// temporary's range is free again after the last wave that uses it.  Sets the
// objects' offsets; returns the arena size.
namespace {

// Open-addressing hash map from int64 keys (>= 0) to int64 values, linear
// probing with backward-shift deletion (no tombstones).
class OffMap {
 public:
  explicit OffMap(size_t expect) {
    size_t cap = 1024;
    while (cap < 2 * expect) cap <<= 1;
    keys_.assign(cap, -1);
    vals_.assign(cap, 0);
    mask_ = cap - 1;
  }
  bool find(int64_t k, int64_t* v) const {
    for (size_t i = slot(k);; i = (i + 1) & mask_) {
      if (keys_[i] == k) {
        *v = vals_[i];
        return true;
      }
      if (keys_[i] < 0) return false;
    }
  }
  void put(int64_t k, int64_t v) {
    if (2 * (count_ + 1) > keys_.size()) grow();
    size_t i = slot(k);
    while (keys_[i] >= 0 && keys_[i] != k) i = (i + 1) & mask_;
    if (keys_[i] < 0) ++count_;
    keys_[i] = k;
    vals_[i] = v;
  }
  void erase(int64_t k) {
    size_t i = slot(k);
    while (keys_[i] != k) {
      if (keys_[i] < 0) return;
      i = (i + 1) & mask_;
    }
    --count_;
    // backward shift: move later entries of the cluster into the hole when
    // their home slot does not lie cyclically in (hole, j]
    size_t hole = i;
    for (size_t j = (i + 1) & mask_; keys_[j] >= 0; j = (j + 1) & mask_) {
      const size_t home = slot(keys_[j]);
      const bool stays = hole <= j ? (home > hole && home <= j) : (home > hole || home <= j);
      if (!stays) {
        keys_[hole] = keys_[j];
        vals_[hole] = vals_[j];
        hole = j;
      }
    }
    keys_[hole] = -1;
  }

 private:
  size_t slot(int64_t k) const { return (size_t)(((uint64_t)k * 0x9E3779B97F4A7C15ull) >> 20) & mask_; }
  void grow() {
    std::vector<int64_t> k, v;
    k.swap(keys_);
    v.swap(vals_);
    keys_.assign(k.size() * 2, -1);
    vals_.assign(k.size() * 2, 0);
    mask_ = keys_.size() - 1;
    count_ = 0;
    for (size_t i = 0; i < k.size(); ++i)
      if (k[i] >= 0) put(k[i], v[i]);
  }
  std::vector<int64_t> keys_, vals_;
  size_t mask_ = 0, count_ = 0;
};

}  // namespace

// Device memory of the temporaries: a range of the arena for the span of
// slots (waves or epochs) in which each one is used.  Free ranges are
// coalesced with their neighbours (boundary maps: start -> size and
// end -> start) and kept in per-size lists; an allocation takes a free range
// of the smallest size that fits (the most recently freed one of that size),
// else grows the arena.  List entries of ranges that were merged or taken are
// dropped lazily, when they are met.
// Sets of small integers with "smallest member >= i": a tree of 64-bit
// words, each bit of a level telling whether the word below it is not empty.
class BitTree {
 public:
  explicit BitTree(uint64_t n) { ensure(n); }
  // room for members below n (the members so far are kept)
  void ensure(uint64_t n) {
    if (n <= cap_) return;
    uint64_t c = cap_ ? cap_ : 4096;
    while (c < n) c *= 2;
    cap_ = c;
    size_t L = 0;
    do {
      c = (c + 63) / 64;
      if (L == lv_.size()) {
        // a new top level: its bit 0 tells whether the old top word is set
        std::vector<uint64_t> top(c, 0ULL);
        if (L > 0 && lv_[L - 1][0] != 0) top[0] = 1;
        lv_.push_back(std::move(top));
      } else {
        lv_[L].resize(c, 0ULL);
      }
      ++L;
    } while (c > 1);
  }
  void set(uint64_t i) {
    for (auto& w : lv_) {
      const bool had = w[i >> 6] != 0;
      w[i >> 6] |= 1ULL << (i & 63);
      if (had) return;
      i >>= 6;
    }
  }
  void clear(uint64_t i) {
    for (auto& w : lv_) {
      w[i >> 6] &= ~(1ULL << (i & 63));
      if (w[i >> 6] != 0) return;
      i >>= 6;
    }
  }
  // smallest member >= i, or -1
  int64_t next(uint64_t i) const {
    size_t L = 0;
    for (;; ++L) {
      if (L >= lv_.size()) return -1;
      const uint64_t wi = i >> 6;
      if (wi < lv_[L].size()) {
        const uint64_t w = lv_[L][wi] & (~0ULL << (i & 63));
        if (w) {
          i = (wi << 6) | (uint64_t)__builtin_ctzll(w);
          break;
        }
      }
      i = wi + 1;  // the next word of this level, as a bit of the level above
    }
    while (L > 0) {
      --L;
      i = (i << 6) | (uint64_t)__builtin_ctzll(lv_[L][i]);
    }
    return (int64_t)i;
  }

 private:
  std::vector<std::vector<uint64_t>> lv_;
  uint64_t cap_ = 0;
};

int64_t Program::layout_objs(int lo, int hi, int nslots) {
  int64_t top_peak = 0;
  // temporaries in order of their first wave (a stable counting sort)
  std::vector<int> start(nslots + 1, 0);
  int ntemp = 0;
  for (int i = lo; i < hi; ++i) {
    const Obj& o = objs[i];
    if (o.temp && o.first_wave >= 0) {
      start[o.first_wave + 1]++;
      ++ntemp;
    }
  }
  for (int w = 0; w < nslots; ++w) start[w + 1] += start[w];
  std::vector<int> temps(ntemp);
  for (int i = lo; i < hi; ++i)
    if (objs[i].temp && objs[i].first_wave >= 0) temps[start[objs[i].first_wave]++] = i;
  std::vector<int>().swap(start);
  // ranges to free after each slot: (offset, size) pairs in one array, by
  // last slot (a counting sort over the allocation order)
  std::vector<int64_t> end_pos(nslots + 1, 0);
  for (int id : temps) end_pos[objs[id].last_wave + 1]++;
  for (int w = 0; w < nslots; ++w) end_pos[w + 1] += end_pos[w];
  std::vector<int64_t> end_fill(end_pos.begin(), end_pos.end() - 1);
  std::vector<std::pair<int64_t, int64_t>> ends(ntemp);
  OffMap by_start(1 << 16), by_end(1 << 16);
  // free ranges by size (a multiple of kAlign): per size unit a stack of
  // offsets, possibly stale (head node in `head`, nodes in one pool), and the
  // set of units whose stacks are not empty; a request takes the smallest
  // size that fits and, among ranges of that size, the last one freed
  BitTree sizes(1 << 16);
  OffMap head(1 << 12);
  std::vector<int64_t> node_off;
  std::vector<int64_t> node_next;
  int64_t node_free = -1;
  auto push_size = [&](int64_t u, int64_t off) {
    int64_t nd;
    if (node_free >= 0) {
      nd = node_free;
      node_free = node_next[nd];
    } else {
      nd = (int64_t)node_off.size();
      node_off.push_back(0);
      node_next.push_back(-1);
    }
    int64_t h = -1;
    const bool had = head.find(u, &h);
    node_off[nd] = off;
    node_next[nd] = had ? h : -1;
    head.put(u, nd);
    if (!had) {
      sizes.ensure((uint64_t)u + 1);
      sizes.set((uint64_t)u);
    }
  };
  // pop the stack of unit u (not empty); true when it is empty afterwards
  auto pop_size = [&](int64_t u, int64_t* off) {
    int64_t h = -1;
    head.find(u, &h);
    *off = node_off[h];
    const int64_t nx = node_next[h];
    node_next[h] = node_free;
    node_free = h;
    if (nx < 0) {
      head.erase(u);
      sizes.clear((uint64_t)u);
      return true;
    }
    head.put(u, nx);
    return false;
  };
  int64_t top = 0;
  auto add_free = [&](int64_t off, int64_t size) {
    by_start.put(off, size);
    by_end.put(off + size, off);
    push_size(size / kAlign, off);
  };
  auto take_free = [&](int64_t off, int64_t size) {
    by_start.erase(off);
    by_end.erase(off + size);
  };
  auto release = [&](int64_t off, int64_t size) {
    int64_t po = 0, ps = 0, ns = 0;
    if (by_end.find(off, &po)) {  // a free range ends where this one starts
      by_start.find(po, &ps);
      take_free(po, ps);
      off = po;
      size += ps;
    }
    if (by_start.find(off + size, &ns)) {  // a free range starts where this one ends
      take_free(off + size, ns);
      size += ns;
    }
    if (off + size == top)
      top = off;
    else
      add_free(off, size);
  };
  int freed = -1;  // slots whose ranges are free again
  for (int id : temps) {
    Obj& o = objs[id];
    while (freed + 1 < o.first_wave) {
      ++freed;
      for (int64_t e = end_pos[freed]; e < end_fill[freed]; ++e) release(ends[e].first, ends[e].second);
    }
    const int64_t need = align_up(std::max<int64_t>(o.elems * (o.is_int ? 4 : 8), 1), kAlign);
    int64_t off = -1;
    for (int64_t u = sizes.next((uint64_t)(need / kAlign)); u >= 0 && off < 0; u = sizes.next((uint64_t)u + 1)) {
      const int64_t size = u * kAlign;
      bool empty = false;
      while (!empty) {
        int64_t c, sz;
        empty = pop_size(u, &c);
        if (by_start.find(c, &sz) && sz == size) {
          off = c;
          break;
        }
      }
      if (off >= 0) {
        take_free(off, size);
        if (size > need) add_free(off + need, size - need);
      }
    }
    if (off < 0) {
      off = top;
      top += need;
    }
    top_peak = std::max(top_peak, top);
    o.off = off;
    ends[end_fill[o.last_wave]++] = {off, need};
  }
  return top_peak;
}

// Device memory of the temporaries.  A plan appended from separately
// recorded parts (absorb) lays out each part's temporaries in a region of
// its own, the parts on parallel host threads; the regions follow one
// another in the arena.  The parts' objects are disjoint, so two
// temporaries of different parts never share memory.
int64_t Program::layout_temps(int nslots) {
  const int np = part_obj_.size() > 1 ? (int)part_obj_.size() - 1 : 1;
  std::vector<int64_t> tops(np, 0);
  if (np == 1) {
    tops[0] = layout_objs(0, (int)objs.size(), nslots);
  } else {
    parallel_for(np, host_threads(), [&](size_t p) {
      tops[p] = layout_objs(part_obj_[p], part_obj_[p + 1], nslots);
    });
    std::vector<int64_t> base(np, 0);
    int64_t b = 0;
    for (int p = 0; p < np; ++p) {
      base[p] = b;
      b += align_up(tops[p], kAlign);
    }
    parallel_for(np, host_threads(), [&](size_t p) {
      for (int i = part_obj_[p]; i < part_obj_[p + 1]; ++i)
        if (objs[i].temp && objs[i].first_wave >= 0) objs[i].off += base[p];
    });
    tops[0] = b;
  }
  arena_top_peak_ = tops[0];
  stats.temp_live_peak = live_peak(nslots);
  return arena_top_peak_;
}

// The largest sum of the sizes of the temporaries alive in one slot.
int64_t Program::live_peak(int nslots) const {
  std::vector<int64_t> delta(nslots + 1, 0);
  for (const Obj& o : objs)
    if (o.temp && o.first_wave >= 0) {
      const int64_t need = align_up(std::max<int64_t>(o.elems * (o.is_int ? 4 : 8), 1), kAlign);
      delta[o.first_wave] += need;
      delta[o.last_wave + 1] -= need;
    }
  int64_t live = 0, peak = 0;
  for (int w = 0; w < nslots; ++w) {
    live += delta[w];
    peak = std::max(peak, live);
  }
  return peak;
}

void Program::finalize(int /*kmax_lds*/) {
  const char* sched = getenv("HM_SCHEDULE");
  const char* budget_env = getenv("HM_TEMP_BUDGET_GB");
  const double budget = (budget_env && *budget_env ? atof(budget_env) : 64.0) * 1e9;
  // the dataflow schedule when asked for and its temporaries fit the budget
  // (it keeps temporaries alive longer, about 2.6 times the earliest-wave
  // schedule's bytes on the 32^3 H-LU: a plan of more than 8M items is only
  // tried when the earliest-wave schedule's temporaries take at most a third
  // of the budget, which spares large plans a failing attempt)
  dataflow_ = false;
  const bool want_dataflow = sched && *sched ? std::strcmp(sched, "dataflow") == 0 : schedule == 1;
  int64_t top = -1;  // the earliest-wave layout, once computed and still in place
  // the bytes alive at once in the earliest-wave schedule: a lower bound of
  // its layout's top, known without laying it out
  const int64_t live = live_peak(nwaves);
  if (want_dataflow) {
    bool attempt = true;
    if (items.size() > ((size_t)8 << 20)) {
      if ((double)live * 3.0 > budget) {
        attempt = false;
      } else {
        top = layout_temps(nwaves);
        attempt = (double)top * 3.0 <= budget;
      }
    }
    if (attempt) {
      if (finalize_dataflow(budget)) return;
      top = -1;  // the attempt placed the temporaries by epochs
    }
  }
  // 1. temporaries: the earliest-wave schedule, or, when its temporaries
  // exceed the budget (HM_TEMP_BUDGET_GB, default 64), the late schedule of
  // the operations that only write temporaries (fewer bytes alive at once,
  // more launches); when the bytes alive at once already exceed the budget,
  // the late schedule is certain and the earliest-wave layout is skipped
  if (top < 0 && (double)live <= budget) top = layout_temps(nwaves);
  const bool late = (sched && std::strcmp(sched, "late") == 0) || top < 0 || top > budget;
  if (late) {
    schedule_late();
    top = layout_temps(nwaves);
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
  const int64_t cap = (int64_t)1 << 30;  // 8 GiB
  ws_doubles_ = (size_t)std::max<int64_t>(std::min(ws_max, cap), 1024);
  stats.ws_bytes = (int64_t)ws_doubles_ * 8;
  stats.waves = nwaves;
  stats.launches = (int64_t)launches_.size();
  emit_order_ = per_op;
  order_tiny_first();
  n_trunc_launches_ = 0;
  small_launches = general_launches = 0;
  for (const Launch& L : launches_) {
    if (L.op == OP_TRUNC && L.variant == 0) n_trunc_launches_++;
    if (L.op == OP_TRUNC) (L.variant >= 1 ? small_launches : general_launches)++;
  }
}

// Dataflow schedule.  The waves make every launch wait for all launches of
// the wave before, so a wave lasts as long as its slowest item.  Here each
// operation waits only for the operations it conflicts with:
//   1. every operation gets an estimated duration (by kind and size) and, in
//      record order, an estimated earliest start: the latest estimated end of
//      the operations it conflicts with (as in record());
//   2. operations in order of that start are gathered into launches per
//      stream and kind (the caller's stream: products, leaf LU, triangular
//      solves, copies; the side stream: small-block truncations; two more
//      streams: the larger truncations, split by size, since a launch ends
//      with its slowest item and every dependent waits for the whole launch);
//      a launch takes operations that start within a window after its first
//      one, and is closed when an operation depends on it;
//   3. a launch waits, by events, for the launches of other streams that
//      hold operations it conflicts with (conflicts tracked again, launch by
//      launch; a stream runs its launches in order);
//   4. epochs of a fixed estimated length end with all streams joining; a
//      temporary's memory is reused only in a later epoch than its last use.
// Returns false (nothing changed) when the temporaries exceed the budget.
bool Program::finalize_dataflow(double budget) {
  const char* wenv = getenv("HM_DF_WINDOW_US");
  const char* eenv = getenv("HM_DF_EPOCH_MS");
  const double window = wenv && *wenv ? atof(wenv) : 100.0;
  const double epoch_len = (eenv && *eenv ? atof(eenv) : 25.0) * 1e3;
  // units: the items of one record (column chunks of one operation)
  std::vector<int> ustart;
  for (size_t i = 0; i < items.size(); ++i)
    if (i == 0 || items[i].rec != items[i - 1].rec) ustart.push_back((int)i);
  const int nu = (int)ustart.size();
  ustart.push_back((int)items.size());
  auto est = [&](const Item& it) -> double {  // microseconds
    switch (it.op) {
      case OP_GEMM: return 15.0;
      case OP_LU: return 70.0;
      case OP_TRSM: return 40.0;
      case OP_COPY: return 5.0;
      default: {
        const HTrunc& t = truncs[it.idx];
        if (trunc_is_small(t)) return 60.0;
        return 150.0 * std::pow(std::max(t.m, t.n) / 128.0, 0.75);
      }
    }
  };
  auto overlap = [](int alo, int ahi, int blo, int bhi) { return alo < bhi && blo < ahi; };
  // the parts of an appended batch touch disjoint objects: the passes over
  // units that follow objects run one part per thread
  std::vector<int> urange{0, nu};
  if (part_item_.size() > 2 && part_item_.front() == 0 && part_item_.back() == items.size()) {
    urange.clear();
    for (size_t pi : part_item_)
      urange.push_back((int)(std::lower_bound(ustart.begin(), ustart.end(), (int)pi) - ustart.begin()));
  }
  const int nparts_u = (int)urange.size() - 1;
  // 1. estimated earliest starts
  std::vector<double> t0(nu);
  {
    struct A {
      double fin;
      int lo, hi;
      bool w;
    };
    std::vector<std::vector<A>> tr(objs.size());
    parallel_for(nparts_u, host_threads(), [&](size_t p) {
      for (int u = urange[p]; u < urange[p + 1]; ++u) {
        const Record& R = recs_[items[ustart[u]].rec];
        const Region* rd = rec_regions_.data() + R.r0;
        const Region* wr = rd + R.nr;
        double st = 0.0, d = 0.0;
        for (int i = ustart[u]; i < ustart[u + 1]; ++i) d = std::max(d, est(items[i]));
        for (int q = 0; q < R.nr; ++q)
          for (const A& a : tr[rd[q].obj])
            if (a.w && overlap(a.lo, a.hi, rd[q].lo, rd[q].hi)) st = std::max(st, a.fin);
        for (int q = 0; q < R.nw; ++q)
          for (const A& a : tr[wr[q].obj])
            if (overlap(a.lo, a.hi, wr[q].lo, wr[q].hi)) st = std::max(st, a.fin);
        t0[u] = st;
        const double fin = st + d;
        for (int q = 0; q < R.nr; ++q) {
          auto& t = tr[rd[q].obj];
          bool merged = false;
          for (A& a : t)
            if (!a.w && a.lo == rd[q].lo && a.hi == rd[q].hi) {
              a.fin = std::max(a.fin, fin);
              merged = true;
              break;
            }
          if (!merged) t.push_back({fin, rd[q].lo, rd[q].hi, false});
        }
        for (int q = 0; q < R.nw; ++q) {
          auto& t = tr[wr[q].obj];
          t.erase(std::remove_if(t.begin(), t.end(),
                                 [&](const A& a) { return a.lo >= wr[q].lo && a.hi <= wr[q].hi; }),
                  t.end());
          t.push_back({fin, wr[q].lo, wr[q].hi, true});
        }
      }
    });
  }
  // 2.-4. units in order of their estimated start (ties: record order):
  // chunks sorted on parallel threads, then merged pairwise
  std::vector<int> order(nu);
  {
    using Key = std::pair<double, int>;
    std::vector<Key> key(nu), tmp(nu);
    for (int u = 0; u < nu; ++u) key[u] = {t0[u], u};
    const int nch = std::max(1, std::min(host_threads(), nu / 65536));
    std::vector<size_t> cut(nch + 1);
    for (int c = 0; c <= nch; ++c) cut[c] = (size_t)nu * c / nch;
    parallel_for(nch, nch, [&](size_t c) { std::sort(key.begin() + cut[c], key.begin() + cut[c + 1]); });
    for (size_t w = 1; w < (size_t)nch; w *= 2) {
      const int pairs = (int)((nch + 2 * w - 1) / (2 * w));
      parallel_for(pairs, pairs, [&](size_t j) {
        const size_t a = cut[2 * w * j], b = cut[std::min<size_t>(2 * w * j + w, nch)],
                     e = cut[std::min<size_t>(2 * w * j + 2 * w, nch)];
        std::merge(key.begin() + a, key.begin() + b, key.begin() + b, key.begin() + e, tmp.begin() + a);
      });
      key.swap(tmp);
    }
    for (int u = 0; u < nu; ++u) order[u] = key[u].second;
  }
  // epochs: one starts with the first unit at or after the previous epoch's
  // end, and lasts a fixed estimated length from that unit's start; a
  // temporary lives from the first to the last epoch that touches it.  The
  // bytes alive at once over epochs bound the layout from below: a plan whose
  // bound already exceeds the budget is given up before the launches are built.
  std::vector<int> uepoch(nu);
  int nepochs = 1;
  {
    int e = 0;
    double end = epoch_len;
    for (int u : order) {
      if (t0[u] >= end) {
        ++e;
        end = t0[u] + epoch_len;
      }
      uepoch[u] = e;
    }
    nepochs = e + 1;
  }
  std::vector<int> first_epoch(objs.size(), -1), last_epoch(objs.size(), -1);
  parallel_for(nparts_u, host_threads(), [&](size_t p) {
    for (int u = urange[p]; u < urange[p + 1]; ++u) {
      const Record& R = recs_[items[ustart[u]].rec];
      const Region* rg = rec_regions_.data() + R.r0;
      for (int q = 0; q < R.nr + R.nw; ++q) {
        const int o = rg[q].obj;
        if (!objs[o].temp) continue;
        if (first_epoch[o] < 0 || uepoch[u] < first_epoch[o]) first_epoch[o] = uepoch[u];
        last_epoch[o] = std::max(last_epoch[o], uepoch[u]);
      }
    }
  });
  {
    std::vector<int64_t> delta(nepochs + 1, 0);
    for (size_t o = 0; o < objs.size(); ++o)
      if (first_epoch[o] >= 0) {
        const int64_t need = align_up(std::max<int64_t>(objs[o].elems * (objs[o].is_int ? 4 : 8), 1), kAlign);
        delta[first_epoch[o]] += need;
        delta[last_epoch[o] + 1] -= need;
      }
    int64_t live = 0;
    for (int e = 0; e < nepochs; ++e)
      if ((double)(live += delta[e]) > budget) return false;
  }
  struct Group {
    int op, variant, stream, slot;
    double tfirst;
    std::vector<int> units, deps;
    int launch;
  };
  std::vector<Group> groups;
  std::vector<int> open_slot(4 * OP_COUNT, -1);  // class (main, side, large by size) x kind -> open group
  std::vector<std::vector<int>> per_op(OP_COUNT);
  std::vector<int64_t> ws_need;  // per launch, doubles
  std::vector<Launch> L;
  std::vector<int> waits;
  int epoch = 0;
  const char* senv = getenv("HM_DF_LARGE_SPLIT");
  // the larger truncations go to stream 2 up to this many rows, else to stream 3
  const int large_split = senv && *senv ? atoi(senv) : 256;
  bool epoch_pending = false;
  auto close = [&](int g) {
    Group& G = groups[g];
    open_slot[G.slot] = -1;
    G.launch = (int)L.size();
    Launch ln;
    ln.op = G.op;
    ln.first = (int)per_op[G.op].size();
    ln.variant = G.variant;
    ln.wave = epoch;
    ln.stream = G.stream;
    ln.epoch_start = epoch_pending;
    epoch_pending = false;
    int64_t need = 0;
    for (int u : G.units)
      for (int i = ustart[u]; i < ustart[u + 1]; ++i) {
        per_op[G.op].push_back(items[i].idx);
        if (G.op == OP_TRUNC && G.variant == 0) {
          const HTrunc& t = truncs[items[i].idx];
          need += align_up((int64_t)(t.m + t.n) * t.lmax + 2 * (int64_t)t.lmax * t.lmax + 4 * t.lmax + 64, 32) +
                  4 * 16384;
        }
      }
    ln.count = (int)per_op[G.op].size() - ln.first;
    std::sort(G.deps.begin(), G.deps.end());
    G.deps.erase(std::unique(G.deps.begin(), G.deps.end()), G.deps.end());
    ln.w0 = (int)waits.size();
    for (int d : G.deps) {
      const Group& D = groups[d];
      if (D.launch < 0) throw std::runtime_error("dataflow schedule: a dependency is still open");
      if (D.stream == G.stream) continue;  // the stream's order
      waits.push_back(D.launch);
      L[D.launch].signal = true;
    }
    ln.nw = (int)waits.size() - ln.w0;
    L.push_back(ln);
    ws_need.push_back(need);
    std::vector<int>().swap(G.units);
    std::vector<int>().swap(G.deps);
  };
  auto close_all = [&]() {
    for (int g : open_slot)
      if (g >= 0) close(g);
  };
  // conflicts by launch group; reads of one range are merged per stream (a
  // later launch of the same stream comes after the earlier one)
  struct B {
    int lo, hi;
    bool w;
    int g;
  };
  std::vector<std::vector<B>> tr(objs.size());
  std::vector<int> deps;
  for (int u : order) {
    const Item& it0 = items[ustart[u]];
    const Record& R = recs_[it0.rec];
    const Region* rd = rec_regions_.data() + R.r0;
    const Region* wr = rd + R.nr;
    if (uepoch[u] != epoch) {
      close_all();
      epoch = uepoch[u];
      epoch_pending = true;
    }
    deps.clear();
    auto add_dep = [&](int d) {  // a unit has few dependencies: a linear check
      for (int e : deps)
        if (e == d) return;
      deps.push_back(d);
    };
    for (int q = 0; q < R.nr; ++q)
      for (const B& a : tr[rd[q].obj])
        if (a.w && overlap(a.lo, a.hi, rd[q].lo, rd[q].hi)) add_dep(a.g);
    for (int q = 0; q < R.nw; ++q)
      for (const B& a : tr[wr[q].obj])
        if (overlap(a.lo, a.hi, wr[q].lo, wr[q].hi)) add_dep(a.g);
    int cls = 0, variant = 0;
    if (it0.op == OP_TRUNC) {
      if (trunc_is_small(truncs[it0.idx])) {
        cls = 1;
        variant = small_tpc == 8 ? 2 : 1;
      } else {
        const HTrunc& t = truncs[it0.idx];
        cls = std::max(t.m, t.n) <= large_split ? 2 : 3;
      }
    }
    const int slot = cls * OP_COUNT + it0.op;
    for (int d : deps)
      if (groups[d].launch < 0) close(d);
    int g = open_slot[slot];
    if (g >= 0 && t0[u] - groups[g].tfirst > window) {
      close(g);
      g = -1;
    }
    if (g < 0) {
      Group G;
      G.op = it0.op;
      G.variant = variant;
      G.stream = cls;
      G.slot = slot;
      G.tfirst = t0[u];
      G.launch = -1;
      g = (int)groups.size();
      groups.push_back(std::move(G));
      open_slot[slot] = g;
    }
    groups[g].units.push_back(u);
    groups[g].deps.insert(groups[g].deps.end(), deps.begin(), deps.end());
    const int gs = groups[g].stream;
    for (int q = 0; q < R.nr; ++q) {
      auto& t = tr[rd[q].obj];
      bool merged = false;
      for (B& a : t)
        if (!a.w && a.lo == rd[q].lo && a.hi == rd[q].hi && groups[a.g].stream == gs) {
          a.g = g;
          merged = true;
          break;
        }
      if (!merged) t.push_back({rd[q].lo, rd[q].hi, false, g});
    }
    for (int q = 0; q < R.nw; ++q) {
      auto& t = tr[wr[q].obj];
      t.erase(std::remove_if(t.begin(), t.end(), [&](const B& a) { return a.lo >= wr[q].lo && a.hi <= wr[q].hi; }),
              t.end());
      t.push_back({wr[q].lo, wr[q].hi, true, g});
    }
  }
  close_all();
  // events after the last launch of every stream in an epoch (the joins)
  {
    int last[4] = {-1, -1, -1, -1};
    for (size_t li = 0; li <= L.size(); ++li) {
      if (li == L.size() || L[li].epoch_start) {
        for (int k = 0; k < 4; ++k)
          if (last[k] >= 0) L[last[k]].signal = true;
        for (int k = 0; k < 4; ++k) last[k] = -1;
      }
      if (li < L.size()) last[L[li].stream] = (int)li;
    }
  }
  // temporaries over epochs
  std::vector<std::pair<int, int>> saved(objs.size());
  for (size_t o = 0; o < objs.size(); ++o) {
    saved[o] = {objs[o].first_wave, objs[o].last_wave};
    objs[o].first_wave = first_epoch[o];
    objs[o].last_wave = last_epoch[o];
  }
  const int64_t top = layout_temps(nepochs);
  if ((double)top > budget) {
    for (size_t o = 0; o < objs.size(); ++o) {
      objs[o].first_wave = saved[o].first;
      objs[o].last_wave = saved[o].second;
    }
    return false;
  }
  // workspace: one part per stream that runs large truncations, sized for its
  // largest launch (at most 4 GiB each)
  const int64_t cap = (int64_t)1 << 29;
  int64_t part[4] = {0, 0, 0, 0}, poff[4] = {0, 0, 0, 0};
  for (size_t li = 0; li < L.size(); ++li)
    if (L[li].op == OP_TRUNC && L[li].variant == 0)
      part[L[li].stream] = std::max(part[L[li].stream], std::max<int64_t>(std::min(ws_need[li], cap), 1024));
  int64_t wtot = 0;
  for (int k = 0; k < 4; ++k) {
    poff[k] = wtot;
    wtot += part[k];
  }
  for (Launch& ln : L)
    if (ln.op == OP_TRUNC && ln.variant == 0) {
      ln.ws_off = poff[ln.stream];
      ln.ws_len = part[ln.stream];
    }
  ws_doubles_ = (size_t)std::max<int64_t>(wtot, 1024);
  launches_ = std::move(L);
  waits_ = std::move(waits);
  emit_order_ = per_op;
  order_tiny_first();
  dataflow_ = true;
  stats.late_schedule = false;
  stats.dataflow = true;
  stats.epochs = nepochs;
  arena_bytes_ = (size_t)std::max<int64_t>(top, kAlign);
  stats.temp_bytes = top;
  stats.ws_bytes = (int64_t)ws_doubles_ * 8;
  stats.waves = nwaves;
  stats.launches = (int64_t)launches_.size();
  n_trunc_launches_ = 0;
  small_launches = general_launches = 0;
  for (const Launch& ln : launches_) {
    if (ln.op == OP_TRUNC && ln.variant == 0) n_trunc_launches_++;
    if (ln.op == OP_TRUNC) (ln.variant >= 1 ? small_launches : general_launches)++;
  }
  return true;
}

// Inside every small-block launch, the blocks of at most 32 x 32 first: the
// kernel runs them one per wavefront (Launch::tiny counts them).
void Program::order_tiny_first() {
  const bool on = tiny_path_enabled();
  std::vector<int>& ord = emit_order_[OP_TRUNC];
  for (Launch& L : launches_) {
    L.tiny = 0;
    if (L.op != OP_TRUNC || L.variant < 1 || !on) continue;
    auto b = ord.begin() + L.first, e = b + L.count;
    auto mid = std::stable_partition(b, e, [&](int idx) {
      const HTrunc& t = truncs[idx];
      return trunc_is_tiny(t.m, t.n) && !(t.flags & TRUNC_CLASS_CHECK);
    });
    L.tiny = (int)(mid - b);
  }
}

DDim Program::ddim(const Dim& d) const {
  DDim r;
  r.stat = d.stat;
  r.pad = 0;
  r.dyn = d.rank_obj >= 0 ? (const int*)ptr_of(d.rank_obj) : nullptr;
  return r;
}


hipError_t Program::upload(hipStream_t s) {
  hipError_t e;
  if ((e = alloc->get(&arena_, arena_bytes_)) != hipSuccess) return e;
  if ((e = alloc->get(&ws_, ws_doubles_ * sizeof(double))) != hipSuccess) return e;
  if (debug) {
    if ((e = hipMemset(arena_, 0, arena_bytes_)) != hipSuccess) return e;
    if ((e = hipMemset(ws_, 0, ws_doubles_ * sizeof(double))) != hipSuccess) return e;
  }
  if ((e = alloc->get(&counters_, sizeof(unsigned long long) * (size_t)std::max(1, n_trunc_launches_))) != hipSuccess)
    return e;
  if ((e = alloc->get(&done_, sizeof(int) * std::max<size_t>(truncs.size(), 1))) != hipSuccess) return e;
  if ((e = hipStreamCreateWithFlags(&side_, hipStreamNonBlocking)) != hipSuccess) return e;
  if ((e = hipEventCreateWithFlags(&ev_main_, hipEventDisableTiming)) != hipSuccess) return e;
  if ((e = hipEventCreateWithFlags(&ev_side_, hipEventDisableTiming)) != hipSuccess) return e;
  if (!dataflow_ && lanes > 2)
    for (int q = 0; q < 2; ++q) {
      if ((e = hipStreamCreateWithFlags(&lane_[q], hipStreamNonBlocking)) != hipSuccess) return e;
      if ((e = hipEventCreateWithFlags(&ev_lane_[q], hipEventDisableTiming)) != hipSuccess) return e;
    }
  if (dataflow_) {
    for (auto& x : long_)
      if ((e = hipStreamCreateWithFlags(&x, hipStreamNonBlocking)) != hipSuccess) return e;
    for (auto& x : ev_tail_)
      if ((e = hipEventCreateWithFlags(&x, hipEventDisableTiming)) != hipSuccess) return e;
    lev_.assign(launches_.size(), nullptr);
    for (size_t li = 0; li < launches_.size(); ++li)
      if (launches_[li].signal && (e = hipEventCreateWithFlags(&lev_[li], hipEventDisableTiming)) != hipSuccess)
        return e;
  }
  auto P = [&](const View& v) -> double* { return (double*)ptr_of(v.obj) + v.off; };
  // one host image of every descriptor array (each at a 256-byte offset),
  // lowered on parallel threads, then one copy to the device
  const std::vector<int>& og = emit_order_[OP_GEMM];
  const std::vector<int>& ot = emit_order_[OP_TRUNC];
  const std::vector<int>& ol = emit_order_[OP_LU];
  const std::vector<int>& os = emit_order_[OP_TRSM];
  const std::vector<int>& oc = emit_order_[OP_COPY];
  size_t total = 0;
  auto place = [&](size_t bytes) {
    const size_t off = (size_t)align_up((int64_t)total, 256);
    total = off + bytes;
    return off;
  };
  off_term_ = place(terms.size() * sizeof(DGemmTerm));
  off_part_ = place(parts.size() * sizeof(DTruncPart));
  off_[OP_GEMM] = place(og.size() * sizeof(DGemm));
  off_[OP_TRUNC] = place(ot.size() * sizeof(DTrunc));
  off_[OP_LU] = place(ol.size() * sizeof(DLu));
  off_[OP_TRSM] = place(os.size() * sizeof(DTrsm));
  off_[OP_COPY] = place(oc.size() * sizeof(DCopy));
  std::unique_ptr<char[]> host(new char[std::max<size_t>(total, 256)]);
  DGemmTerm* dterms = (DGemmTerm*)(host.get() + off_term_);
  DTruncPart* dparts = (DTruncPart*)(host.get() + off_part_);
  DGemm* dg = (DGemm*)(host.get() + off_[OP_GEMM]);
  DTrunc* dt = (DTrunc*)(host.get() + off_[OP_TRUNC]);
  DLu* dl = (DLu*)(host.get() + off_[OP_LU]);
  DTrsm* ds = (DTrsm*)(host.get() + off_[OP_TRSM]);
  DCopy* dc = (DCopy*)(host.get() + off_[OP_COPY]);
  // chunks of 64K elements of each array, all arrays in one pool of tasks
  struct Task {
    int kind;
    size_t lo, hi;
  };
  std::vector<Task> tasks;
  const size_t sizes[7] = {terms.size(), parts.size(), og.size(), ot.size(), ol.size(), os.size(), oc.size()};
  for (int k = 0; k < 7; ++k)
    for (size_t lo = 0; lo < sizes[k]; lo += 65536) tasks.push_back({k, lo, std::min(sizes[k], lo + 65536)});
  parallel_for((int)tasks.size(), host_threads(), [&](size_t ti) {
    const Task tk = tasks[ti];
    for (size_t i = tk.lo; i < tk.hi; ++i) {
      switch (tk.kind) {
        case 0: {
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
          break;
        }
        case 1: {
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
          break;
        }
        case 2: {
          const HGemm& g = gemms[og[i]];
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
          dg[i] = d;
          break;
        }
        case 3: {
          const int idx = ot[i];
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
          d.kfix = -1;
          dt[i] = d;
          break;
        }
        case 4: {
          const HLu& u = lus[ol[i]];
          dl[i] = {(double*)ptr_of(u.obj), u.n, u.n, u.kind, 0};
          break;
        }
        case 5: {
          const HTrsm& t = trsms[os[i]];
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
          ds[i] = d;
          break;
        }
        default: {
          const HCopy& c = copies[oc[i]];
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
          dc[i] = d;
          break;
        }
      }
    }
  });
  dt_host_.assign(dt, dt + ot.size());
  desc_bytes_ = std::max<size_t>(total, 256);
  stats.desc_bytes = (int64_t)desc_bytes_;
  if ((e = alloc->get(&desc_, desc_bytes_)) != hipSuccess) return e;
  if (size_logging) {
    if ((e = alloc->get(&size_log_, sizeof(int) * 8 * std::max<size_t>(ot.size(), 1))) != hipSuccess) return e;
    if ((e = hipMemset(size_log_, 0xff, sizeof(int) * 8 * std::max<size_t>(ot.size(), 1))) != hipSuccess) return e;
  }
  if (total > 0 && (e = hipMemcpyAsync(desc_, host.get(), total, hipMemcpyHostToDevice, s)) != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

hipError_t Program::set_rank_override(const int* ranks, hipStream_t s) {
  if (!desc_) return hipErrorNotReady;
  for (DTrunc& d : dt_host_) d.kfix = ranks ? ranks[d.log_idx] : -1;
  invalidate_graph();
  if (dt_host_.empty()) return hipSuccess;
  hipError_t e = hipMemcpyAsync(desc_ + off_[OP_TRUNC], dt_host_.data(), dt_host_.size() * sizeof(DTrunc),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e;
}

hipError_t Program::reset_counters(hipStream_t s) {
  hipError_t e = launch_fill_u32((unsigned int*)counters_, 2 * (int64_t)std::max(1, n_trunc_launches_), 0u, s);
  if (e == hipSuccess) e = launch_fill_u32((unsigned int*)done_, (int64_t)std::max<size_t>(truncs.size(), 1), 0u, s);
  return e;
}

hipError_t Program::run_graph(hipStream_t s, int* status, double eps) {
  replayed = false;
  // A dataflow plan runs on its streams directly: capturing it (about 30,000
  // launches on four streams with about 25,000 cross-stream waits) ended the
  // process at its first capture, so graph replay is not used for it.
  if (dataflow_) return run(s, status, eps);
  // A plan of more launches than any plan whose capture has been seen to
  // complete runs directly: the process ended during or after the capture of
  // a much larger wave plan (the 64^3 Laplacian), and the cause is not known.
  if (launches_.size() > kGraphMaxLaunches) return run(s, status, eps);
  // a wave plan on more than two streams runs directly (its capture would
  // carry several cross-stream waits per wave)
  if (lanes > 2) return run(s, status, eps);
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
  replayed = true;
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

// One launch on stream st: the kernel of its kind (for the general
// truncations, the register-resident kernel and then the general kernel, on
// the launch's part of the workspace).  *tl counts the general launches.
int Program::lane_of(const Launch& L) const {
  const bool small = L.op == OP_TRUNC && L.variant >= 1;
  if (lanes <= 2) return small ? 1 : 0;
  if (L.op == OP_TRUNC) return small ? 1 : 2;
  if (L.op == OP_LU || L.op == OP_TRSM) return 3;
  return 0;
}

hipError_t Program::launch_one(size_t li, hipStream_t st, int* status, double eps, int* tl) {
  const Launch& L = launches_[li];
  const DGemmTerm* terms_d = (const DGemmTerm*)(desc_ + off_term_);
  const DTruncPart* parts_d = (const DTruncPart*)(desc_ + off_part_);
  hipError_t e = hipSuccess;
  switch (L.op) {
    case OP_GEMM:
      e = launch_gemm((const DGemm*)(desc_ + off_[OP_GEMM]) + L.first, terms_d, L.count, prec, st);
      break;
    case OP_TRUNC:
      if (L.variant >= 1) {
        e = launch_trunc_small((const DTrunc*)(desc_ + off_[OP_TRUNC]) + L.first, parts_d, L.count, status, eps,
                               size_log_, L.variant == 2 ? 8 : 4, pred, feat_log, prec, st, L.tiny);
      } else {
        // register-resident kernel, then the general kernel: each skips the other's items
        int* ctr = (int*)((unsigned long long*)counters_ + *tl);
        double* pool = ws_ + L.ws_off;
        const int64_t pool_len = L.ws_len > 0 ? L.ws_len : (int64_t)ws_doubles_;
        e = launch_trunc_tall((const DTrunc*)(desc_ + off_[OP_TRUNC]) + L.first, parts_d, L.count, pool, pool_len,
                              ctr, status, eps, size_log_, done_ + L.first, 1, st, false);
        if (e == hipSuccess)
          e = launch_trunc((const DTrunc*)(desc_ + off_[OP_TRUNC]) + L.first, parts_d, L.count, pool, pool_len, ctr,
                           status, eps, size_log_, done_ + L.first, 1, st);
        ++*tl;
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
  return e;
}

// Dataflow schedule: four streams (the caller's, the side stream, two for the
// larger truncations).  A launch waits by events for the launches of other
// streams named in its wait list, unless its stream has already waited for
// them or for later launches of theirs; at an epoch start every stream joins
// the caller's stream, which first waits for all of them.
hipError_t Program::run_dataflow(hipStream_t s, int* status, double eps) {
  hipError_t e = reset_counters(s);
  if (e != hipSuccess) return e;
  hipStream_t st[4] = {s, side_, long_[0], long_[1]};
  std::vector<hipEvent_t> ev;
  if (profile_ops) {
    ev.resize(2 * launches_.size());
    for (auto& x : ev)
      if ((e = hipEventCreate(&x)) != hipSuccess) return e;
  }
  int waited[4][4];  // waited[k][j]: latest launch of stream j that stream k has waited for
  int last[4] = {-1, -1, -1, -1};
  auto join = [&]() -> hipError_t {
    hipError_t er;
    for (int k = 1; k < 4; ++k)
      if (last[k] >= 0 && waited[0][k] < last[k]) {
        if ((er = hipStreamWaitEvent(st[0], lev_[last[k]], 0)) != hipSuccess) return er;
        waited[0][k] = last[k];
      }
    if ((er = hipEventRecord(ev_main_, st[0])) != hipSuccess) return er;
    for (int k = 1; k < 4; ++k) {
      if ((er = hipStreamWaitEvent(st[k], ev_main_, 0)) != hipSuccess) return er;
      for (int j = 0; j < 4; ++j) waited[k][j] = last[j];
    }
    return hipSuccess;
  };
  for (int k = 0; k < 4; ++k)
    for (int j = 0; j < 4; ++j) waited[k][j] = -1;
  if ((e = join()) != hipSuccess) return e;  // every stream starts after the caller's work so far
  int tl = 0;
  for (size_t li = 0; li < launches_.size(); ++li) {
    const Launch& L = launches_[li];
    if (L.epoch_start && (e = join()) != hipSuccess) return e;
    const int k = L.stream;
    for (int q = L.w0; q < L.w0 + L.nw; ++q) {
      const int d = waits_[q];
      const int j = launches_[d].stream;
      if (waited[k][j] >= d) continue;
      if ((e = hipStreamWaitEvent(st[k], lev_[d], 0)) != hipSuccess) return e;
      waited[k][j] = d;
    }
    if (profile_ops) (void)hipEventRecord(ev[2 * li], st[k]);
    if ((e = launch_one(li, st[k], status, eps, &tl)) != hipSuccess) return e;
    if (profile_ops) (void)hipEventRecord(ev[2 * li + 1], st[k]);
    if (L.signal && (e = hipEventRecord(lev_[li], st[k])) != hipSuccess) return e;
    last[k] = (int)li;
  }
  // the caller's stream sees the end of every stream, also of a stream whose
  // last work is a join (under graph capture every stream that took part
  // must end joined to the capturing stream)
  for (int k = 1; k < 4; ++k) {
    if ((e = hipEventRecord(ev_tail_[k - 1], st[k])) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(st[0], ev_tail_[k - 1], 0)) != hipSuccess) return e;
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

hipError_t Program::run(hipStream_t s, int* status, double eps) {
  if (dataflow_) return run_dataflow(s, status, eps);
  hipError_t e = reset_counters(s);
  if (e != hipSuccess) return e;
  int tl = 0;
  std::vector<hipEvent_t> ev;
  if (profile_ops) {
    ev.resize(2 * launches_.size());
    for (auto& x : ev)
      if ((e = hipEventCreate(&x)) != hipSuccess) return e;
  }
  // Streams ("lanes") of the wave schedule: lane 0 is the caller's stream.
  // dirty[b]: lane b has launches not yet published by an event record;
  // need[a][b]: lane b has published work that lane a has not waited for.
  // Records happen at wave boundaries only, so the launches of one wave on
  // different lanes overlap, and every launch of a wave starts after all
  // launches of the waves before it.
  const int K = lanes > 2 ? 4 : 2;
  hipStream_t ls[4] = {s, side_, lane_[0], lane_[1]};
  hipEvent_t le[4] = {ev_main_, ev_side_, ev_lane_[0], ev_lane_[1]};
  bool dirty[4] = {true, false, false, false};
  bool need[4][4] = {};
  int cur_wave = -1;
  for (size_t li = 0; li < launches_.size(); ++li) {
    const Launch& L = launches_[li];
    if (L.wave != cur_wave) {
      cur_wave = L.wave;
      for (int b = 0; b < K; ++b)
        if (dirty[b]) {
          if ((e = hipEventRecord(le[b], ls[b])) != hipSuccess) return e;
          dirty[b] = false;
          for (int a = 0; a < K; ++a)
            if (a != b) need[a][b] = true;
        }
    }
    const int a = lane_of(L);
    hipStream_t st = ls[a];
    for (int b = 0; b < K; ++b)
      if (need[a][b]) {
        if ((e = hipStreamWaitEvent(st, le[b], 0)) != hipSuccess) return e;
        need[a][b] = false;
      }
    if (profile_ops) (void)hipEventRecord(ev[2 * li], st);
    e = launch_one(li, st, status, eps, &tl);
    if (e != hipSuccess) return e;
    if (profile_ops) (void)hipEventRecord(ev[2 * li + 1], st);
    dirty[a] = true;
  }
  // the caller's stream sees the end of every other lane's work
  for (int b = 1; b < K; ++b) {
    if (dirty[b]) {
      if ((e = hipEventRecord(le[b], ls[b])) != hipSuccess) return e;
      need[0][b] = true;
    }
    if (need[0][b]) {
      if ((e = hipStreamWaitEvent(s, le[b], 0)) != hipSuccess) return e;
      need[0][b] = false;
    }
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
  if ((e = alloc->get(&flag, sizeof(int))) != hipSuccess) return e;
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
                                 size_log_, L.variant == 2 ? 8 : 4, pred, feat_log, prec, s, L.tiny);
        } else {
          // register-resident kernel, then the general kernel: each skips the other's items
          int* ctr = (int*)((unsigned long long*)counters_ + tl);
          e = launch_trunc_tall((const DTrunc*)(desc_ + off_[OP_TRUNC]) + L.first, parts_d, L.count, ws_,
                                (int64_t)ws_doubles_, ctr, status, eps, size_log_, done_ + L.first, 1, s, false);
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
  (void)hipStreamSynchronize(s);
  alloc->put(flag);
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
  for (auto& x : long_)
    if (x) {
      (void)hipStreamSynchronize(x);
      (void)hipStreamDestroy(x);
      x = nullptr;
    }
  for (int q = 0; q < 2; ++q) {
    if (lane_[q]) {
      (void)hipStreamSynchronize(lane_[q]);
      (void)hipStreamDestroy(lane_[q]);
      lane_[q] = nullptr;
    }
    if (ev_lane_[q]) (void)hipEventDestroy(ev_lane_[q]);
    ev_lane_[q] = nullptr;
  }
  for (auto& x : ev_tail_)
    if (x) {
      (void)hipEventDestroy(x);
      x = nullptr;
    }
  for (auto& x : lev_)
    if (x) (void)hipEventDestroy(x);
  lev_.clear();
  alloc->put(feat_log);
  feat_log = nullptr;
  alloc->put(arena_);
  alloc->put(ws_);
  alloc->put(desc_);
  alloc->put(counters_);
  alloc->put(size_log_);
  alloc->put(done_);
  size_log_ = nullptr;
  done_ = nullptr;
  arena_ = nullptr;
  ws_ = nullptr;
  desc_ = nullptr;
  counters_ = nullptr;
}

}  // namespace hm
