// Shared pieces of the C ABI implementation: the context, error reporting
// and the exception guard of every entry point.
#pragma once
#include <hip/hip_runtime.h>

#include <new>
#include <stdexcept>
#include <string>

#include "../../include/hm.h"

struct hm_ctx {
  hipStream_t stream = nullptr;
  int* status = nullptr;  // device status block (8 ints)
  int schedule = 1;       // hm_schedule of the plans made on this context
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
