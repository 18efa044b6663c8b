// Private accumulators of the intensity epilogue (see accum.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace toprop {

template <typename T>
struct Accum {
  static hipError_t zero(T* p, int64_t n, hipStream_t s);             // p[0..n) = 0 (a kernel, no memset)
  static hipError_t add(T* dst, const T* src, int64_t n, hipStream_t s);  // dst += src
};

}  // namespace toprop
