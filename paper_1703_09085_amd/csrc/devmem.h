// Device memory of a context: the caller's allocator (for example a framework's
// caching allocator) or hipMalloc / hipFree, with the bytes in use tracked for
// the context's statistics.  Every object that holds device memory (matrices,
// plans, networks) keeps a reference, so it frees through the allocator that
// gave it the memory even after its context is gone.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <mutex>
#include <unordered_map>

#include "../../include/hm.h"

namespace hm {

class DevAlloc {
 public:
  DevAlloc() = default;
  DevAlloc(hm_alloc_fn a, hm_free_fn f, void* user) : fa_(a), ff_(f), user_(user) {}

  hipError_t get(void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 1;
    if (fa_) {
      *p = fa_(bytes, user_);
      if (!*p) return hipErrorOutOfMemory;
    } else {
      hipError_t e = hipMalloc(p, bytes);
      if (e != hipSuccess) {
        *p = nullptr;
        return e;
      }
    }
    std::lock_guard<std::mutex> g(mu_);
    live_[*p] = bytes;
    in_use_ += (int64_t)bytes;
    if (in_use_ > peak_) peak_ = in_use_;
    ++count_;
    return hipSuccess;
  }
  template <class T>
  hipError_t get(T** p, size_t bytes) {
    void* v = nullptr;
    hipError_t e = get(&v, bytes);
    *p = (T*)v;
    return e;
  }
  void put(void* p) {
    if (!p) return;
    {
      std::lock_guard<std::mutex> g(mu_);
      auto it = live_.find(p);
      if (it != live_.end()) {
        in_use_ -= (int64_t)it->second;
        live_.erase(it);
      }
    }
    if (ff_)
      ff_(p, user_);
    else
      (void)hipFree(p);
  }
  int64_t in_use() const {
    std::lock_guard<std::mutex> g(mu_);
    return in_use_;
  }
  int64_t peak() const {
    std::lock_guard<std::mutex> g(mu_);
    return peak_;
  }
  int64_t allocations() const {
    std::lock_guard<std::mutex> g(mu_);
    return count_;
  }
  bool external() const { return fa_ != nullptr; }

 private:
  hm_alloc_fn fa_ = nullptr;
  hm_free_fn ff_ = nullptr;
  void* user_ = nullptr;
  mutable std::mutex mu_;
  std::unordered_map<void*, size_t> live_;
  int64_t in_use_ = 0, peak_ = 0, count_ = 0;
};

using AllocRef = std::shared_ptr<DevAlloc>;

// The allocator of objects made without a context (host-only checks).
inline AllocRef default_alloc() {
  static AllocRef a = std::make_shared<DevAlloc>();
  return a;
}

}  // namespace hm
