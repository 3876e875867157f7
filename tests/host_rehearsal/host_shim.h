// Host definitions of two device helpers that the library's headers use, for
// building its host code with g++ (included ahead of every source).
#pragma once
#include <cstring>
#include <hip/hip_runtime.h>
static inline float __uint_as_float(unsigned u) {
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
static inline unsigned __float_as_uint(float f) {
  unsigned u;
  std::memcpy(&u, &f, 4);
  return u;
}
