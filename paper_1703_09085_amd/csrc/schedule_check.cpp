// Host check of a finished schedule, written apart from the code that makes
// it: it derives the order of the launches from the run rules alone (stream
// order, event waits, joins at epoch starts; or, for waves, the wave order)
// and replays the recorded operations' regions to find every pair that must
// be ordered.
#include <algorithm>
#include <array>
#include <vector>

#include "program.h"

namespace hm {

void Program::verify_schedule(int64_t* out) const {
  for (int q = 0; q < 8; ++q) out[q] = 0;
  const size_t nl = launches_.size();
  out[0] = (int64_t)nl;
  out[7] = dataflow_ ? 1 : 0;
  // the launch of every item
  std::vector<std::vector<int>> pos_launch(OP_COUNT), idx_pos(OP_COUNT);
  for (int op = 0; op < OP_COUNT; ++op) pos_launch[op].assign(emit_order_[op].size(), -1);
  for (size_t li = 0; li < nl; ++li)
    for (int q = 0; q < launches_[li].count; ++q) {
      int& slot = pos_launch[launches_[li].op][launches_[li].first + q];
      if (slot >= 0) ++out[6];
      slot = (int)li;
    }
  for (int op = 0; op < OP_COUNT; ++op) {
    size_t mx = 0;
    for (int v : emit_order_[op]) mx = std::max(mx, (size_t)v + 1);
    idx_pos[op].assign(mx, -1);
    for (size_t p = 0; p < emit_order_[op].size(); ++p) {
      int& slot = idx_pos[op][emit_order_[op][p]];
      if (slot >= 0) ++out[6];
      slot = (int)p;
    }
  }
  std::vector<int> item_launch(items.size(), -1);
  for (size_t i = 0; i < items.size(); ++i) {
    const Item& it = items[i];
    const int p = (size_t)it.idx < idx_pos[it.op].size() ? idx_pos[it.op][it.idx] : -1;
    item_launch[i] = p >= 0 ? pos_launch[it.op][p] : -1;
    if (item_launch[i] < 0) ++out[6];
  }
  if (out[6]) return;
  // vector clocks (dataflow): vc[li][j] = the latest launch of stream j that
  // has ended before launch li starts
  using Clock = std::array<int, 4>;
  std::vector<Clock> vc;
  if (dataflow_) {
    vc.resize(nl);
    std::array<Clock, 4> cur;
    for (auto& c : cur) c.fill(-1);
    int last[4] = {-1, -1, -1, -1};
    auto after = [&](int li) {
      Clock v = vc[li];
      v[launches_[li].stream] = li;
      return v;
    };
    auto merge = [](Clock& a, const Clock& b) {
      for (int j = 0; j < 4; ++j) a[j] = std::max(a[j], b[j]);
    };
    auto join = [&]() {
      for (int k = 1; k < 4; ++k)
        if (last[k] >= 0) {
          if (!launches_[last[k]].signal) ++out[5];
          merge(cur[0], after(last[k]));
        }
      for (int k = 1; k < 4; ++k) merge(cur[k], cur[0]);
    };
    join();
    for (size_t li = 0; li < nl; ++li) {
      const Launch& L = launches_[li];
      if (L.epoch_start) join();
      for (int q = L.w0; q < L.w0 + L.nw; ++q) {
        const int d = waits_[q];
        if (d >= (int)li || !launches_[d].signal) {
          ++out[5];
          continue;
        }
        merge(cur[L.stream], after(d));
      }
      vc[li] = cur[L.stream];
      cur[L.stream][L.stream] = (int)li;
      last[L.stream] = (int)li;
    }
  }
  auto ordered = [&](int a, int b) {  // launch a ends before launch b starts
    if (a == b) return false;
    if (!dataflow_) return launches_[a].wave < launches_[b].wave;
    return vc[b][launches_[a].stream] >= a;
  };
  // every conflicting pair, in record order (all readers kept until a write
  // covers them)
  struct Acc {
    int lo, hi;
    bool w;
    int launch;
  };
  std::vector<std::vector<Acc>> tr(objs.size());
  size_t i = 0;
  while (i < items.size()) {
    size_t j = i;
    while (j < items.size() && items[j].rec == items[i].rec) ++j;
    const int lv = item_launch[i];
    const Record& R = recs_[items[i].rec];
    const Region* rd = rec_regions_.data() + R.r0;
    auto check = [&](const Acc& a) {
      ++out[1];
      if (!ordered(a.launch, lv)) ++out[2];
    };
    for (int q = 0; q < R.nr; ++q)
      for (const Acc& a : tr[rd[q].obj])
        if (a.w && a.lo < rd[q].hi && rd[q].lo < a.hi) check(a);
    for (int q = 0; q < R.nw; ++q) {
      const Region& r = rd[R.nr + q];
      for (const Acc& a : tr[r.obj])
        if (a.lo < r.hi && r.lo < a.hi) check(a);
    }
    for (int q = 0; q < R.nr; ++q) {
      auto& t = tr[rd[q].obj];
      bool dup = false;
      for (const Acc& a : t)
        if (!a.w && a.lo == rd[q].lo && a.hi == rd[q].hi && a.launch == lv) dup = true;
      if (!dup) t.push_back({rd[q].lo, rd[q].hi, false, lv});
    }
    for (int q = 0; q < R.nw; ++q) {
      const Region& r = rd[R.nr + q];
      auto& t = tr[r.obj];
      t.erase(std::remove_if(t.begin(), t.end(), [&](const Acc& a) { return a.lo >= r.lo && a.hi <= r.hi; }),
              t.end());
      t.push_back({r.lo, r.hi, true, lv});
    }
    i = j;
  }
  // temporaries that share memory: every launch that touches the later one
  // starts after every launch that touches the earlier one has ended
  std::vector<std::vector<int>> users(objs.size());
  for (size_t it = 0; it < items.size(); ++it) {
    const Record& R = recs_[items[it].rec];
    for (int q = 0; q < R.nr + R.nw; ++q) {
      const int o = rec_regions_[R.r0 + q].obj;
      if (objs[o].temp) users[o].push_back(item_launch[it]);
    }
  }
  std::vector<int> tmp;
  for (size_t o = 0; o < objs.size(); ++o)
    if (objs[o].temp && !users[o].empty()) {
      auto& u = users[o];
      std::sort(u.begin(), u.end());
      u.erase(std::unique(u.begin(), u.end()), u.end());
      tmp.push_back((int)o);
    }
  std::sort(tmp.begin(), tmp.end(), [&](int a, int b) { return objs[a].off < objs[b].off; });
  for (size_t a = 0; a < tmp.size(); ++a) {
    const Obj& A = objs[tmp[a]];
    const int64_t end = A.off + std::max<int64_t>(A.elems * (A.is_int ? 4 : 8), 1);
    for (size_t b = a + 1; b < tmp.size() && objs[tmp[b]].off < end; ++b) {
      ++out[3];
      // one of the two must come entirely before the other
      auto before = [&](int x, int y) {
        for (int la : users[x])
          for (int lb : users[y])
            if (!ordered(la, lb)) return false;
        return true;
      };
      if (!before(tmp[a], tmp[b]) && !before(tmp[b], tmp[a])) ++out[4];
    }
  }
}

}  // namespace hm
