// hm_trunc_batch_device_noalloc: the device-descriptor truncation batch with
// all of its scratch memory (lowered descriptors, work-group claim counter,
// per-item marks and the truncation workspace) in one file-scope device
// array, for callers that cannot allocate (graph capture, serving loops).
//
// Each device that runs the library holds its own copy of the array until the
// process ends.  Host code reaches it only through the address that
// hipGetSymbolAddress returns on that device (kept per device); the array's
// name is not a device address on the host.  Every call on one device shares
// that device's array and leaves its contents behind: whatever must start at
// zero is cleared by a fill kernel at the start of each call, and calls that
// overlap on one device (different streams, threads) race on it.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/hm.h"
#include "api_internal.h"
#include "build_kernels.h"

namespace hm {
hipError_t launch_fill_u32(unsigned int* p, int64_t n, unsigned int v, hipStream_t s);
}

using namespace hm;

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // 64 MiB per device
constexpr int kMaxItems = 4096;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
std::vector<char*> g_scratch;  // per device: the array's device address (NULL until resolved)

// The device address of this device's scratch array (resolved once per device,
// with the device current).
char* scratch_address() {
  int dev = 0;
  check(hipGetDevice(&dev), "hipGetDevice");
  std::lock_guard<std::mutex> g(g_mu);
  if ((int)g_scratch.size() <= dev) g_scratch.resize(dev + 1, nullptr);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) throw HipError("hipGetSymbolAddress(scratch): NULL address");
    g_scratch[dev] = (char*)p;
  }
  return g_scratch[dev];
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

hm_status hm_trunc_batch_device_noalloc(hm_ctx* ctx, int32_t count, const hm_trunc_desc* descs, int32_t max_rows,
                                        int32_t max_stack, double eps, int32_t precision, int64_t* executed) {
  return guard([&] {
    if (!ctx || count < 0 || (count > 0 && !descs) || max_rows < 1 || max_stack < 0 || !(eps >= 0) ||
        precision < HM_FP64 || precision > HM_BF16X3)
      return fail(HM_ERR_ARG, "hm_trunc_batch_device_noalloc: invalid argument");
    if (executed) *executed = 0;
    if (count == 0) return HM_OK;
    if (count > kMaxItems)
      return fail(HM_ERR_ARG, "hm_trunc_batch_device_noalloc: more than " + std::to_string(kMaxItems) + " items");
    // layout: descriptors | parts | claim counter | marks | workspace
    const size_t o_dt = 0;
    const size_t o_dp = align256(o_dt + (size_t)count * sizeof(DTrunc));
    const size_t o_ctr = align256(o_dp + 2 * (size_t)count * sizeof(DTruncPart));
    const size_t o_done = align256(o_ctr + sizeof(unsigned long long));
    const size_t o_pool = align256(o_done + (size_t)count * sizeof(int));
    const int64_t per = trunc_ws_doubles(max_rows, max_rows, max_stack);
    const int64_t pool_doubles = (int64_t)((kScratchBytes - o_pool) / sizeof(double));
    if (per > 0 && per * (int64_t)count > pool_doubles)
      return fail(HM_ERR_ARG, "hm_trunc_batch_device_noalloc: the workspace that the bounds need (" +
                                  std::to_string(per * (int64_t)count * 8) + " bytes) exceeds the " +
                                  std::to_string((kScratchBytes - o_pool)) + " bytes of scratch");
    char* base = scratch_address();
    DTrunc* dt = (DTrunc*)(base + o_dt);
    DTruncPart* dp = (DTruncPart*)(base + o_dp);
    int* counter = (int*)(base + o_ctr);
    int* done = (int*)(base + o_done);
    double* pool = (double*)(base + o_pool);
    hipStream_t s = ctx->stream;
    check(launch_fill_u32((unsigned int*)ctx->status, STATUS_INTS, 0u, s), "status reset");
    check(launch_fill_u32((unsigned int*)counter, 2, 0u, s), "counter reset");
    check(launch_fill_u32((unsigned int*)done, count, 0u, s), "marks reset");
    check(launch_lower_trunc_descs(descs, count, max_rows, max_stack, dt, dp, ctx->status, s), "lower descriptors");
    check(launch_trunc_small(dt, dp, count, ctx->status, eps, nullptr, 4, nullptr, nullptr, precision, s,
                             tiny_path_enabled() ? -1 : 0),
          "small truncations");
    check(launch_trunc_tall(dt, dp, count, pool, pool_doubles, counter, ctx->status, eps, nullptr, done, 1, s,
                            thin_path_enabled()),
          "tall truncations");
    check(launch_trunc(dt, dp, count, pool, pool_doubles, counter, ctx->status, eps, nullptr, done, 1, s),
          "truncations");
    if (!executed) return HM_OK;  // asynchronous: nothing is read back
    int st[STATUS_INTS] = {0};
    check(hipMemcpyAsync(st, ctx->status, sizeof(st), hipMemcpyDeviceToHost, s), "status read");
    check(hipStreamSynchronize(s), "hm_trunc_batch_device_noalloc");
    std::memcpy(executed, st + 2, sizeof(int64_t));
    if (st[0] & ST_BAD_DESC)
      return fail(HM_ERR_ARG, "hm_trunc_batch_device_noalloc: invalid descriptor or beyond the bounds");
    return status_to_error(st[0]);
  });
}

}  // extern "C"
