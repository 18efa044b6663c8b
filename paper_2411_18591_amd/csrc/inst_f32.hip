// Propagation kernels instantiated for complex64 fields.
#include "launch_impl.hpp"

namespace toprop {
template struct Launch<float>;

hipError_t launch_reduce_add(const double* src, int64_t n, double scale, double* dst,
                             hipStream_t s) {
  hipLaunchKernelGGL((reduce_add_kernel<256>), dim3(1), dim3(256), 0, s, src, n, scale, dst);
  return hipGetLastError();
}

int col_tile_width(int ly, bool is_double) {
  int tc = 0;
  auto q = [&](auto Lc) -> hipError_t {
    constexpr int L = decltype(Lc)::value;
    tc = is_double ? ColCfg<double, L>::TC : ColCfg<float, L>::TC;
    return hipSuccess;
  };
  if (dispatch_len(ly, q) != hipSuccess) return 0;
  return tc;
}
}  // namespace toprop
