// Private accumulators of the intensity epilogue.  Jobs of one call that add
// their intensities into the same image may run on different lanes: each
// lane after the first accumulates into a private zeroed copy, and the
// copies are added into the image in lane order after the lanes join
// (deterministic for a given call).  Zeroing is a kernel rather than a
// memset so that the call stays safe to capture in a graph.
#include <hip/hip_runtime.h>

#include "accum.hpp"

namespace toprop {

template <typename T>
__global__ void __launch_bounds__(256) accum_zero_kernel(T* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = T(0);
}

template <typename T>
__global__ void __launch_bounds__(256) accum_add_kernel(T* dst, const T* src, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] += src[i];
}

namespace {
int accum_grid(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (int)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}
}  // namespace

template <typename T>
hipError_t Accum<T>::zero(T* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((accum_zero_kernel<T>), dim3(accum_grid(n)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

template <typename T>
hipError_t Accum<T>::add(T* dst, const T* src, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((accum_add_kernel<T>), dim3(accum_grid(n)), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}

template struct Accum<float>;
template struct Accum<double>;

}  // namespace toprop
