// Shared pieces of the C ABI implementation: the context, error reporting
// and the exception guard of every entry point.
#pragma once
#include <hip/hip_runtime.h>

#include <mutex>
#include <new>
#include <stdexcept>
#include <string>

#include "../../include/hm.h"
#include "devmem.h"

struct hm_ctx {
  hipStream_t stream = nullptr;
  int* status = nullptr;  // device status block (16 ints)
  int schedule = 1;       // hm_schedule of the plans made on this context
  hm::AllocRef alloc;     // device memory of everything made for this context
  // totals for hm_get_stats
  mutable std::mutex mu;
  int64_t plans = 0, runs = 0, truncations = 0, trunc_bytes = 0, builds = 0;
  double plan_seconds = 0, run_seconds = 0, build_seconds = 0;
};

namespace hm {

inline thread_local std::string g_err;

struct HipError : std::runtime_error {
  explicit HipError(const std::string& s) : std::runtime_error(s) {}
};

inline void check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw HipError(std::string(what) + ": " + hipGetErrorString(e));
}

inline hm_status fail(hm_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

// Runs f(), turning exceptions into status codes (nothing throws across the ABI).
template <class F>
hm_status guard(F&& f) {
  try {
    return f();
  } catch (const HipError& e) {
    return fail(HM_ERR_HIP, e.what());
  } catch (const std::bad_alloc&) {
    return fail(HM_ERR_ALLOC, "host allocation failed");
  } catch (const std::invalid_argument& e) {
    return fail(HM_ERR_ARG, e.what());
  } catch (const std::exception& e) {
    return fail(HM_ERR_STATE, e.what());
  }
}

}  // namespace hm
