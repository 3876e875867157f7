// A recorded H-matrix computation: logical arrays ("objects"), primitive work
// items, and their schedule.
//
// The planner replays the paper's recursions on the host and records every
// arithmetic step as a work item that names the rows of the objects it reads
// and writes.  Each item is placed in the earliest wave after every item it
// conflicts with (read-after-write, write-after-read, write-after-write on
// overlapping rows), so one wave holds only independent items and is executed
// as one batched launch per item kind.  Temporary objects get device memory
// only for the span of waves in which they are used.
#pragma once
#include <algorithm>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <functional>
#include <memory>
#include <string>
#include <vector>

#include "devmem.h"
#include "hm_types.h"

namespace hm {

// Make room in one of a plan's arrays before an append: fourfold growth (the
// arrays reach tens of millions of entries, and each doubling copies them
// again; capacity that is never written costs no memory).
template <class V>
inline void grow4(V& v, size_t extra = 1) {
  if (v.size() + extra > v.capacity()) v.reserve(std::max<size_t>(4096, 4 * (v.size() + extra)));
}


struct Obj {
  bool temp = false;
  bool is_int = false;
  int64_t elems = 0;  // doubles (or ints)
  int rows = 0;       // row space used for dependency regions
  void* ptr = nullptr;  // persistent objects
  int64_t off = -1;     // temps: byte offset in the arena
  int first_wave = -1, last_wave = -1;
};

// A dimension: static capacity plus an optional rank object holding the value.
struct Dim {
  int stat = 0;
  int rank_obj = -1;
};

// A matrix operand: element (i, j) at base[off + i + j*ld] (or base[off + j + i*ld]
// when trans).  rows x cols (cols possibly dynamic).  Region rows are
// [rlo, rlo + rows) of the object when not transposed, the whole object otherwise.
struct View {
  int obj = -1;
  int64_t off = 0;
  int ld = 0;
  int trans = 0;
  int rows = 0;
  Dim cols;
  int rlo = 0;
  View rows_sub(int r0, int nr) const {
    View v = *this;
    if (!trans) {
      v.off += r0;
      v.rlo += r0;
    } else {
      v.off += (int64_t)r0 * ld;
    }
    v.rows = nr;
    return v;
  }
};

// Host-side work items (objects instead of pointers).
struct HTerm {
  View A, B;  // op(A) = A^T when ta etc. (views are taken as stored)
  int ta = 0, tb = 0;
  double alpha = 1.0;
  Dim k;
};
struct HGemm {
  View C;  // output, m = C.rows (static), n = C.cols
  Dim m;
  int beta = 0;
  int term0 = 0, nterms = 0;
  int row0 = 0, col0 = 0;
};
struct HPart {
  View A, B;
  double alpha = 1.0;
  int row_off = 0, rows = 0, col_off = 0, cols = 0;
  Dim k;
};
struct HTrunc {
  int objA, objB, objR;  // output rk object (A: m x cap, B: n x cap)
  int m, n, cap;
  int part0, nparts;
  int lmax;
  int flags;
  int level = 0;  // level of the row cluster of the target block
};
inline bool trunc_is_small(const HTrunc& t) { return t.m <= TRUNC_SMALL_MAX && t.n <= TRUNC_SMALL_MAX; }
struct HLu {
  int obj;
  int n;
  int kind = LEAF_LU;
};
struct HTrsm {
  View T;  // n x n leaf factor
  View X;  // n x c operand
  int n;
  int kind;
  int col0;
};
struct HCopy {
  View src, dst;  // dst rows x cols
  Dim m, n;
  int mode = COPY_COPY;
  double alpha = 1.0;
  int rank_src = -1, rank_dst = -1;  // rank objects (-1 none); rank_src -1 with rank_dst sets 0
};

struct Region {
  int obj, lo, hi;
};

struct Item {
  int op;
  int idx;
  int wave;
  int rec;  // the record whose regions and dependencies the item has
};

struct ProgramStats {
  int64_t items[OP_COUNT] = {0, 0, 0, 0, 0};
  int64_t waves = 0;
  int64_t launches = 0;
  int64_t temp_bytes = 0;
  int64_t ws_bytes = 0;
  int64_t desc_bytes = 0;
  int64_t trunc_bytes = 0;  // algorithmic bytes of truncations at capacity (upper bound)
  int64_t temp_live_peak = 0;  // largest sum of the sizes of the temporaries alive in one wave
  bool late_schedule = false;  // the late schedule of temporary-only operations was used
  bool dataflow = false;       // the dataflow schedule was used
  int64_t epochs = 0;          // dataflow schedule: epochs (all streams join between two)
};

// Largest number of launches of a plan that is captured into a hipGraph; a
// larger plan runs launch by launch (the 64-instance batch of 2D Laplacians,
// about 20,000 launches, is the largest capture known to complete).
constexpr size_t kGraphMaxLaunches = 24000;

// Runs fn(0 .. n-1) on up to `threads` host threads.
void parallel_for(int n, int threads, const std::function<void(size_t)>& fn);
int host_threads();


class Program {
 public:
  // objects
  int add_persistent(void* ptr, int64_t elems, int rows, bool is_int = false);
  int add_temp(int64_t elems, int rows, bool is_int = false);

  // recording (regions: reads, writes)
  int record(int op, int idx, const std::vector<Region>& reads, const std::vector<Region>& writes);
  // Reserve room for f times the objects, items and records held now (a
  // batch of similar instances: called after the first one is recorded).
  void reserve_scaled(double f);
  // Append programs recorded separately, in order, on up to `threads` host
  // threads.  Their objects are disjoint from each other's and from this
  // program's, so every item keeps the wave it had in its own program: the
  // result equals recording them one after another into this program.
  // Nothing is recorded into this program afterwards.
  void absorb(std::vector<std::unique_ptr<Program>>& parts, int threads);
  // another item of the last record (a column chunk of the same operation)
  void push_sibling(int op, int idx) { items.push_back({op, idx, items.back().wave, items.back().rec}); }

  std::vector<Obj> objs;
  std::vector<HGemm> gemms;
  std::vector<HTerm> terms;
  std::vector<HTrunc> truncs;
  std::vector<HPart> parts;
  std::vector<HLu> lus;
  std::vector<HTrsm> trsms;
  std::vector<HCopy> copies;
  std::vector<Item> items;
  int nwaves = 0;
  int lu_nmax = 0, trsm_nmax = 0;

  // finalisation and execution
  void finalize(int kmax_lds);
  hipError_t upload(hipStream_t s);
  hipError_t run(hipStream_t s, int* status, double eps);
  // the same launches replayed from a hipGraph captured on the first call (and
  // again when eps or the status block change)
  hipError_t run_graph(hipStream_t s, int* status, double eps);
  // Autotuner: runs the plan once per variant of the small-block truncation
  // kernel (4 or 8 threads per column), timing every launch, with restore()
  // bringing the written matrix back to its state before each trial; every
  // small-block launch then keeps its faster variant.  chosen[v] counts the
  // launches that chose 4 (v = 0) or 8 (v = 1) threads per column.
  hipError_t autotune(hipStream_t s, int* status, double eps, hipError_t (*restore)(void*), void* ctx,
                      int64_t* chosen);
  std::vector<float> launch_ms;  // with profile_ops: device time of every launch of the last run
  size_t trunc_items() const { return truncs.size(); }
  void invalidate_graph() {
    if (gexec_) (void)hipGraphExecDestroy(gexec_);
    gexec_ = nullptr;
  }
  int64_t launch_count() const { return (int64_t)launches_.size(); }
  // wave, kind, variant, items, milliseconds (0 unless profile_ops) of launch i
  void launch_entry(int64_t i, double* e) const {
    const Launch& L = launches_[i];
    e[0] = L.wave;
    e[1] = L.op;
    e[2] = L.variant;
    e[3] = L.count;
    e[4] = (size_t)i < launch_ms.size() ? launch_ms[i] : 0.0;
  }
  bool use_graph = false;
  bool replayed = false;  // the last run was replayed from the hipGraph
  // Debug run: synchronise after every launch and scan all memory for NaN/Inf;
  // stops at the first launch that produced one and describes it in `error`.
  hipError_t run_checked(hipStream_t s, int* status, double eps);
  bool debug = false;
  bool profile_ops = false;           // time every launch with events (per kind)
  int small_tpc = 4;                  // initial threads per column of the small-block kernel (4 or 8)
  int prec = 0;                       // arithmetic of the dense products and small-block contractions (Precision)
  const DPredictor* pred = nullptr;   // rank predictor (device) for the small-block truncations, or NULL
  float* feat_log = nullptr;          // per truncation item: features, k^, outcome (device), or NULL
  bool feature_logging = false;       // allocate feat_log when a predictor is attached
  double small_seconds = 0;           // with profile_ops: device time of the small-block truncation launches
  int64_t small_launches = 0, general_launches = 0;  // truncation launches per run by kernel
  bool size_logging = false;          // record (m, n, l, k) of every executed truncation
  // Streams of a wave plan: 2 runs the small-block truncations on a second
  // stream and everything else on the caller's; 4 gives the larger
  // truncations and the leaf factorisations and solves a stream each, so that
  // the independent launches of one wave run side by side (plans on more than
  // two streams are not captured into a hipGraph)
  int lanes = 4;
  int schedule = 1;                   // 0 waves, 1 dataflow (HM_SCHEDULE=waves|late|dataflow overrides)
  std::vector<int> read_size_log() const;
  // Host check of the finished schedule (no device needed): out[0] launches,
  // out[1] pairs of conflicting operations, out[2] of them not ordered by the
  // schedule, out[3] pairs of temporaries sharing memory, out[4] of them not
  // ordered, out[5] waits for a launch that records no event, out[6] items
  // placed in no launch or in more than one, out[7] 1 for the dataflow
  // schedule.
  void verify_schedule(int64_t* out) const;
  double op_seconds[OP_COUNT] = {0, 0, 0, 0, 0};
  AllocRef alloc = default_alloc();  // device memory of the plan
  // Rank override (test hook): ranks[i] >= 0 replaces the rank rule's choice
  // of truncation item i (recording order), -1 keeps the rule; NULL removes
  // the override.  Rewrites the uploaded truncation descriptors.
  hipError_t set_rank_override(const int* ranks, hipStream_t s);
  void release();
  ProgramStats stats;
  std::string error;

 private:
  struct Access {
    int wave, lo, hi;
    bool w;
  };
  // accesses of one object: two in place (most temporaries are written once
  // and read once or twice), more on the heap
  struct AccessList {
    Access in[2];
    std::vector<Access> more;
    int n = 0;
    Access& at(int i) { return i < 2 ? in[i] : more[i - 2]; }
    const Access& at(int i) const { return i < 2 ? in[i] : more[i - 2]; }
    void push(const Access& a) {
      if (n < 2)
        in[n] = a;
      else
        more.push_back(a);
      ++n;
    }
    // drop the accesses with lo <= a.lo, a.hi <= hi (order kept)
    void drop_inside(int lo, int hi) {
      int k = 0;
      for (int i = 0; i < n; ++i) {
        const Access a = at(i);
        if (a.lo >= lo && a.hi <= hi) continue;
        at(k++) = a;
      }
      n = k;
      if ((int)more.size() > std::max(n - 2, 0)) more.resize(std::max(n - 2, 0));
    }
  };
  std::vector<AccessList> track_;
  bool closed_ = false;  // absorb() ran: no more recording
  // device buffers
  char* arena_ = nullptr;
  double* ws_ = nullptr;
  char* desc_ = nullptr;
  int* counters_ = nullptr;
  int* size_log_ = nullptr;
  size_t arena_bytes_ = 0, ws_doubles_ = 0, desc_bytes_ = 0;
  int64_t arena_top_peak_ = 0;  // highest end of the temporaries' ranges
  // recorded operations: earliest wave, regions (reads then writes) in
  // rec_regions_, and whether a persistent object is written
  struct Record {
    int wave;
    int r0, nr, nw;
    bool persistent_write;
  };
  std::vector<Record> recs_;
  std::vector<Region> rec_regions_;
  void schedule_late();
  void order_tiny_first();
  int64_t live_peak(int nslots) const;
  int64_t layout_temps(int nslots);
  int64_t layout_objs(int lo, int hi, int nslots);  // one part's temporaries, offsets from 0
  std::vector<int> part_obj_;   // after absorb: object range of every appended part
  std::vector<size_t> part_item_;  // after absorb: item range of every appended part
  bool finalize_dataflow(double budget);
  hipError_t run_dataflow(hipStream_t s, int* status, double eps);
  hipError_t launch_one(size_t li, hipStream_t st, int* status, double eps, int* tl);
  int n_trunc_launches_ = 0;
  struct Launch {
    int op, first, count;
    int variant;  // truncations: 0 = general kernels; small-block kernel with 4 (1) or 8 (2) threads per column
    int wave;     // wave (wave schedules) or epoch (dataflow schedule)
    // small-block truncations: the first `tiny` items have m, n <= 32 (one
    // per wavefront)
    int tiny = 0;
    // dataflow schedule: the launch's stream (0 the caller's, 1 the side
    // stream, 2 and 3 the large truncations), whether all streams join before
    // it, the launches of other streams it waits for (waits_[w0, w0 + nw)),
    // whether an event is recorded after it, and its part of the workspace
    int stream = 0;
    bool epoch_start = false;
    int w0 = 0, nw = 0;
    bool signal = false;
    int64_t ws_off = 0, ws_len = 0;
  };
  bool dataflow_ = false;
  hipStream_t long_[2] = {nullptr, nullptr};
  hipEvent_t ev_tail_[3] = {nullptr, nullptr, nullptr};  // end of streams 1..3 of a run
  std::vector<hipEvent_t> lev_;  // per launch with signal set
  std::vector<int> waits_;
  // small-block truncations run on a second stream, concurrently with the
  // other launches of the same wave; events order the two streams at wave
  // boundaries
  hipStream_t side_ = nullptr;
  hipStream_t lane_[2] = {nullptr, nullptr};  // wave plans on four streams: the larger truncations, LU and TRSM
  hipEvent_t ev_lane_[2] = {nullptr, nullptr};
  int lane_of(const Launch& L) const;
  // per truncation item: 1 when the register-resident kernel took it in the
  // current run (cleared at the start of every run)
  int* done_ = nullptr;
  hipError_t reset_counters(hipStream_t s);
  // graph mode: the launch sequence captured once per (eps, status block)
  hipGraphExec_t gexec_ = nullptr;
  hipStream_t cap_ = nullptr;  // capture and replay stream
  hipEvent_t ev_cap_ = nullptr;
  double graph_eps_ = -1.0;
  int* graph_status_ = nullptr;
  hipEvent_t ev_main_ = nullptr, ev_side_ = nullptr;
  std::vector<Launch> launches_;
  std::vector<std::vector<int>> emit_order_;  // per kind: device position -> item index
  size_t off_[OP_COUNT] = {0, 0, 0, 0, 0};
  size_t off_term_ = 0, off_part_ = 0;
  std::vector<DTrunc> dt_host_;  // the uploaded truncation descriptors (emit order)
  void* ptr_of(int obj) const;
  DDim ddim(const Dim& d) const;
};

}  // namespace hm
