// Entry point that allocates nothing, for callers that cannot call
// hipMalloc: code under HIP graph capture, tight serving loops, harnesses
// that forbid allocation.  Every workspace of the forward propagation (the
// chunk's padded intermediate, loss partial sums, transfer-function tables,
// twiddle tables) lives in one static device array, `scratch`, of
// TO_NOALLOC_SCRATCH_BYTES per GPU.  Each GPU's copy sits at its own device
// address, looked up once per device with hipGetSymbolAddress; host code
// passes only that looked-up address to kernels.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "../../include/toprop.h"
#include "fft.hpp"
#include "noalloc.hpp"

static __device__ __align__(256) unsigned char scratch[TO_NOALLOC_SCRATCH_BYTES];

namespace {

using toprop::cx;

constexpr size_t kTwBytes = (size_t)toprop::kTwPacked * (sizeof(cx<float>) + sizeof(cx<double>));
constexpr size_t kTwRegion = (kTwBytes + 255) / 256 * 256;

std::mutex g_mu;
std::vector<void*> g_scratch;  // per device: the device address of `scratch`

// Device address of this device's `scratch` (looked up once per device,
// with that device current).
to_status scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return toprop::hip_error(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_mu);
  if ((int)g_scratch.size() <= dev) g_scratch.resize(dev + 1, nullptr);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return toprop::hip_error(e, "hipGetSymbolAddress(scratch)");
    if (!p) return toprop::set_error(TO_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return TO_OK;
}

// Entry i of the packed tables: exp(-2 pi i m / L) for the length L with
// L - 8 <= i < 2 L - 8, m = i + 8 - L, from sincospi of the exact ratio
// 2 m / L in FP64; the complex64 table holds the same values rounded.
__global__ void __launch_bounds__(256) twiddle_build_kernel(cx<float>* t32, cx<double>* t64) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= toprop::kTwPacked) return;
  const int L = 1 << (31 - __clz(i + 8));
  const int m = i + 8 - L;
  double s, c;
  sincospi(2.0 * (double)m / (double)L, &s, &c);
  t64[i] = {c, -s};
  t32[i] = {(float)c, (float)-s};
}

}  // namespace

extern "C" to_status to_propagate_noalloc(const to_job* jobs, int32_t njobs, to_dtype dtype, void* stream) {
  if (njobs < 0) return toprop::set_error(TO_E_INVAL, "njobs < 0");
  if (njobs > 0 && !jobs) return toprop::set_error(TO_E_INVAL, "jobs is NULL");
  if (dtype != TO_C64 && dtype != TO_C128) return toprop::set_error(TO_E_INVAL, "dtype is not TO_C64/TO_C128");
  if (njobs == 0) return TO_OK;
  constexpr size_t kArea = (size_t)TO_NOALLOC_SCRATCH_BYTES - kTwRegion;
  to_status st = toprop::validate_forward(jobs, njobs, dtype, kArea);  // before anything is enqueued
  if (st != TO_OK) return st;
  void* base = nullptr;
  st = scratch_address(&base);
  if (st != TO_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  cx<float>* t32 = (cx<float>*)base;
  cx<double>* t64 = (cx<double>*)((char*)base + sizeof(cx<float>) * toprop::kTwPacked);
  hipLaunchKernelGGL(twiddle_build_kernel, dim3((toprop::kTwPacked + 255) / 256), dim3(256), 0, s, t32, t64);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return toprop::hip_error(e, "twiddle table launch");
  return toprop::propagate_fixed(jobs, njobs, dtype, s, base, (char*)base + kTwRegion, kArea);
}
