// Host-only rehearsal of an H-LU plan of a Laplacian grid: recording,
// scheduling, upload (the lowering of every descriptor) and the launch
// sequence, against stubs of the HIP runtime calls of the host code.  "Device"
// memory is host memory (mapped, untouched until written); every copy and
// fill is checked to lie inside one allocation, every event to be recorded
// before it is waited for and not used after it is destroyed.  The test
// builds it with UBSan and the libstdc++ assertions (host_shim.h included
// ahead of every source).
//
//   driver <side> <dims 2|3> <mode 0 standard | 1 accumulated | 2 fused> <leaf> <kmax> [count]
//   (count > 1: a batch of grids of sides side, side - 1, ..., recorded on
//   parallel threads and appended, as the batch entry point plans them)
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <sys/mman.h>
#include <vector>
#include "../../paper_1703_09085_amd/csrc/planner.h"
#include "../../paper_1703_09085_amd/csrc/structure.h"
using namespace hm;
static size_t n_launch = 0, n_items_launched = 0, n_wait = 0, n_record = 0;
static std::vector<std::pair<char*, size_t>> allocs;  // (base, bytes) of the stub's "device" memory
static void check_range(const void* p, size_t n, const char* what) {
  const char* c = (const char*)p;
  for (auto& a : allocs)
    if (a.first && c >= a.first && c + n <= a.first + a.second) return;
  fprintf(stderr, "%s outside every allocation: %p + %zu\n", what, p, n);
  abort();
}
// a launch: its grid fits (at most 512 threads a workgroup, fewer than 2^32
// threads) and its descriptors lie inside one allocation
template <class T>
static void launched(const T* d, int count, const char* what) {
  if (count <= 0) return;
  if ((unsigned long long)count * 512ULL >= (1ULL << 32)) {
    fprintf(stderr, "%s: a grid of %d workgroups\n", what, count);
    abort();
  }
  check_range(d, sizeof(T) * (size_t)count, what);
  n_launch++;
  n_items_launched += (size_t)count;
}
// the parts of every truncation item lie inside the parts array
static void check_parts(const DTrunc* d, const DTruncPart* parts, int count, const char* what) {
  for (int i = 0; i < count; ++i) {
    if (d[i].part0 < 0 || d[i].nparts < 1 || d[i].nparts > 4) {
      fprintf(stderr, "%s: item %d has parts [%d, +%d)\n", what, i, d[i].part0, d[i].nparts);
      abort();
    }
    check_range(parts + d[i].part0, sizeof(DTruncPart) * (size_t)d[i].nparts, what);
  }
}
namespace hm {
hipError_t launch_gemm(const DGemm* d, const DGemmTerm* terms, int count, int, hipStream_t) {
  launched(d, count, "gemm");
  for (int i = 0; i < count; ++i) {
    if (d[i].term0 < 0 || d[i].nterms < 0) {
      fprintf(stderr, "gemm: item %d has terms [%d, +%d)\n", i, d[i].term0, d[i].nterms);
      abort();
    }
    if (d[i].nterms > 0) check_range(terms + d[i].term0, sizeof(DGemmTerm) * (size_t)d[i].nterms, "gemm terms");
  }
  return hipSuccess;
}
hipError_t launch_lu(const DLu* d, int count, int, int*, hipStream_t) { launched(d, count, "lu"); return hipSuccess; }
hipError_t launch_trsm(const DTrsm* d, int count, int, hipStream_t) { launched(d, count, "trsm"); return hipSuccess; }
hipError_t launch_copy(const DCopy* d, int count, hipStream_t) { launched(d, count, "copy"); return hipSuccess; }
hipError_t launch_nan_scan(const double*, int64_t, int*, hipStream_t) { return hipSuccess; }
hipError_t launch_fill_u32(unsigned int* p, int64_t n, unsigned int v, hipStream_t) {
  check_range(p, sizeof(unsigned) * (size_t)n, "fill");
  for (int64_t i = 0; i < n; ++i) p[i] = v;
  return hipSuccess;
}
// the register-resident kernel and then the general kernel on the same items:
// counted once, at the second
hipError_t launch_trunc_tall(const DTrunc* d, const DTruncPart* parts, int count, double*, int64_t, int*, int*, double,
                             int*, int* done, int, hipStream_t, bool) {
  check_range(d, sizeof(DTrunc) * (size_t)count, "tall");
  check_parts(d, parts, count, "tall");
  check_range(done, sizeof(int) * (size_t)count, "tall done");
  return hipSuccess;
}
hipError_t launch_trunc(const DTrunc* d, const DTruncPart*, int count, double*, int64_t, int*, int*, double, int*,
                        const int* done, int, hipStream_t) {
  check_range(done, sizeof(int) * (size_t)count, "trunc done");
  launched(d, count, "trunc");
  return hipSuccess;
}
hipError_t launch_trunc_small(const DTrunc* d, const DTruncPart* parts, int count, int*, double, int*, int,
                              const DPredictor*, float*, int, hipStream_t, int) {
  launched(d, count, "small");
  check_parts(d, parts, count, "small");
  return hipSuccess;
}
}  // namespace hm
// the HIP runtime calls of the host code
extern "C" {
hipError_t hipMalloc(void** p, size_t bytes) {
  void* q = mmap(nullptr, bytes, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
  if (q == MAP_FAILED) return hipErrorOutOfMemory;
  *p = q; allocs.push_back({(char*)q, bytes}); return hipSuccess;
}
hipError_t hipFree(void* p) {
  for (auto& a : allocs) if (a.first == p) { munmap(a.first, a.second); a.first = nullptr; return hipSuccess; }
  if (p) { fprintf(stderr, "hipFree of an unknown pointer %p\n", p); abort(); }
  return hipSuccess;
}
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind k) {
  if (k == hipMemcpyHostToDevice) check_range(d, n, "hipMemcpy H2D");
  if (k == hipMemcpyDeviceToHost) check_range(s, n, "hipMemcpy D2H");
  memcpy(d, s, n); return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t) { return hipMemcpy(d, s, n, k); }
hipError_t hipMemset(void* d, int v, size_t n) { check_range(d, n, "hipMemset"); memset(d, v, n); return hipSuccess; }
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) { return hipMemset(d, v, n); }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { static long k = 1; *s = (hipStream_t)(k++ << 4); return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t) { return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
static std::vector<int> ev_state;  // 0 created, 1 recorded, 2 destroyed
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { ev_state.push_back(0); *e = (hipEvent_t)(uintptr_t)ev_state.size(); return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) { return hipEventCreateWithFlags(e, 0); }
static int& ev(hipEvent_t e, const char* what) {
  size_t i = (size_t)(uintptr_t)e;
  if (i == 0 || i > ev_state.size()) { fprintf(stderr, "%s: unknown event %zu\n", what, i); abort(); }
  if (ev_state[i - 1] == 2) { fprintf(stderr, "%s: destroyed event %zu\n", what, i); abort(); }
  return ev_state[i - 1];
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) { ev(e, "record") = 1; n_record++; return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t e, unsigned) { if (ev(e, "wait") != 1) { fprintf(stderr, "wait on an event never recorded\n"); abort(); } n_wait++; return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t e) { ev(e, "sync"); return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 0.f; return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { ev(e, "destroy") = 2; return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipPeekAtLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "stub"; }
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { abort(); }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t*) { abort(); }
hipError_t hipGraphInstantiate(hipGraphExec_t*, hipGraph_t, hipGraphNode_t*, char*, size_t) { abort(); }
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { abort(); }
}
double now() { return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count(); }
// the H-matrix structure of a Laplacian grid, with "device" storage for its blocks
static void make_matrix(DevHMatrix& M, int side, int dims, int leaf, int kmax) {
  const int n = dims == 3 ? side * side * side : side * side;
  std::vector<double> x((size_t)n * dims);
  for (int i = 0; i < n; ++i) {
    x[(size_t)dims * i] = 1 + i % side;
    x[(size_t)dims * i + 1] = 1 + (i / side) % side;
    if (dims == 3) x[(size_t)dims * i + 2] = 1 + i / (side * side);
  }
  M.ct = build_cluster_tree(dims, n, x.data(), leaf); M.bt = build_block_tree(*M.ct, 2.0); M.kmax = kmax;
  size_t nb = M.bt.b.size();
  M.N.assign(nb, nullptr); M.A.assign(nb, nullptr); M.B.assign(nb, nullptr); M.R.assign(nb, nullptr); M.cap.assign(nb, 0);
  M.leafmax = 1; for (auto& c : M.ct->c) if (c.nsons == 0) M.leafmax = std::max(M.leafmax, c.size);
  // the matrix's storage: one pool, as the library lays it out
  size_t total = 0;
  for (size_t i = 0; i < nb; ++i) { const Block& b = M.bt.b[i]; int r = M.ct->c[b.t].size, c = M.ct->c[b.s].size;
    if (b.kind == BLK_DENSE) total += (size_t)r * c;
    if (b.kind == BLK_RK) { int cap = std::min(std::min(r, c), kmax); total += (size_t)(r + c) * cap; } }
  double* pool; hipMalloc((void**)&pool, (total + 1) * 8);
  int* ranks; hipMalloc((void**)&ranks, (nb + 1) * 4);
  size_t off = 0;
  for (size_t i = 0; i < nb; ++i) { const Block& b = M.bt.b[i]; int r = M.ct->c[b.t].size, c = M.ct->c[b.s].size;
    if (b.kind == BLK_DENSE) { M.N[i] = pool + off; off += (size_t)r * c; }
    if (b.kind == BLK_RK) { M.cap[i] = std::min(std::min(r, c), kmax); M.A[i] = pool + off; off += (size_t)r * M.cap[i]; M.B[i] = pool + off; off += (size_t)c * M.cap[i]; M.R[i] = ranks + i; } }
  double* ident; hipMalloc((void**)&ident, 64 * 64 * 8); M.ident = ident;
}
int main(int argc, char** argv) {
  const int side = argc > 1 ? atoi(argv[1]) : 16;
  const int dims = argc > 2 ? atoi(argv[2]) : 3;
  const int mode = argc > 3 ? atoi(argv[3]) : 1;
  const int leaf = argc > 4 ? atoi(argv[4]) : 32;
  const int kmax = argc > 5 ? atoi(argv[5]) : 96;
  const int count = argc > 6 ? atoi(argv[6]) : 1;  // > 1: a batch of grids of sides side, side - 1, ...
  const int n = dims == 3 ? side * side * side : side * side;
  double t = now();
  std::vector<DevHMatrix> Ms(count);
  for (int i = 0; i < count; ++i) make_matrix(Ms[i], std::max(4, side - i), dims, leaf, kmax);
  DevHMatrix& M = Ms[0];
  size_t nb = M.bt.b.size();
  printf("structure: n %d, %zu blocks, %.1f s\n", n, nb, now() - t); fflush(stdout);
  t = now();
  Program P; P.schedule = 1;
  std::vector<std::unique_ptr<PNode>> roots;
  if (count == 1) {
    Planner pl(P, *M.ct, M.kmax, M.ident, M.leafmax); roots.push_back(pl.attach(M)); pl.lu(roots[0].get(), mode);
  } else {  // as the batch entry point does: one program per instance on parallel threads, then appended
    std::vector<std::unique_ptr<Program>> parts(count);
    roots.resize(count);
    parallel_for(count, host_threads(), [&](size_t i) {
      parts[i] = std::make_unique<Program>();
      Planner pl(*parts[i], *Ms[i].ct, Ms[i].kmax, Ms[i].ident, Ms[i].leafmax);
      roots[i] = pl.attach(Ms[i]); pl.lu(roots[i].get(), mode);
    });
    P.absorb(parts, host_threads());
  }
  printf("recorded: %zu items, %d waves, %.1f s\n", P.items.size(), P.nwaves, now() - t); fflush(stdout);
  t = now();
  P.finalize(0);
  printf("scheduled: temporaries %.2f GB, late %d, dataflow %d, %lld launches, %.1f s\n", P.stats.temp_bytes / 1e9,
         (int)P.stats.late_schedule, (int)P.stats.dataflow, (long long)P.stats.launches, now() - t);
  unsigned long long h = 1469598103934665603ULL;  // FNV-1a over the temporaries' offsets
  for (size_t i = 0; i < P.objs.size(); ++i)
    if (P.objs[i].temp) {
      h ^= (unsigned long long)P.objs[i].off + 0x9e3779b97f4a7c15ULL * i;
      h *= 1099511628211ULL;
    }
  printf("layout %016llx\n", h);
  fflush(stdout);
  t = now();
  hipError_t e = P.upload(nullptr);
  printf("upload: %d, descriptors %.2f GB, %.1f s\n", (int)e, P.stats.desc_bytes / 1e9, now() - t); fflush(stdout);
  int* status; hipMalloc((void**)&status, 64);
  t = now();
  e = P.run(nullptr, status, 1e-6);
  printf("run: %d, %zu launches, %zu items, %zu event records, %zu waits, %.1f s\n", (int)e, n_launch,
         n_items_launched, n_record, n_wait, now() - t);
  if (e != hipSuccess || n_items_launched != P.items.size()) {
    fprintf(stderr, "launched %zu of %zu items\n", n_items_launched, P.items.size());
    return 1;
  }
  printf("ok\n");
  return 0;
}
