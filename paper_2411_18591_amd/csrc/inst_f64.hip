// Propagation kernels instantiated for complex128 fields.
#include "launch_impl.hpp"

namespace toprop {
template struct Launch<double>;
}  // namespace toprop

namespace toprop {
template <>
hipError_t launch_sum_parts<double>(const double* part, int groups, int64_t n, double* dst, hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL((sum_parts_kernel<double>), dim3((unsigned)blocks), dim3(256), 0, s, part, groups, n, dst);
  return hipGetLastError();
}
}  // namespace toprop
