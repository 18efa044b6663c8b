// Propagation kernels instantiated for complex64 fields.
#include <algorithm>

#include "launch_impl.hpp"

namespace toprop {
template struct Launch<float>;

hipError_t launch_reduce_add(const double* src, int64_t n, double scale, double* dst,
                             hipStream_t s) {
  hipLaunchKernelGGL((reduce_add_kernel<256>), dim3(1), dim3(256), 0, s, src, n, scale, dst);
  return hipGetLastError();
}

int col_tile_width(int ly, bool is_double, int variant) {
  int tc = 0;
  auto q = [&](auto Lc) -> hipError_t {
    constexpr int L = decltype(Lc)::value;
    auto w = [&](auto vc) {
      constexpr int V = decltype(vc)::value;
      tc = is_double ? ColCfg<double, L, V>::TC : ColCfg<float, L, V>::TC;
    };
    switch (variant) {
      case 1: w(std::integral_constant<int, 1>()); break;
      case 2: w(std::integral_constant<int, 2>()); break;
      case 3: w(std::integral_constant<int, 3>()); break;
      case 4: w(std::integral_constant<int, 4>()); break;
      default: w(std::integral_constant<int, 0>()); break;
    }
    return hipSuccess;
  };
  if (dispatch_len(ly, q) != hipSuccess) return 0;
  return tc;
}
}  // namespace toprop

namespace toprop {
hipError_t launch_tf_tables(cx<float>* ex, float* sx, int lx, double inv_lxdx, cx<float>* ey,
                            float* sy, int ly, double inv_lydy, double fres_a, double q_frac,
                            double lam2, hipStream_t s) {
  const int n = lx + ly;
  hipLaunchKernelGGL((tf_tables_kernel<float>), dim3((n + 255) / 256), dim3(256), 0, s, ex, sx, lx,
                     inv_lxdx, ey, sy, ly, inv_lydy, fres_a, q_frac, lam2);
  return hipGetLastError();
}
}  // namespace toprop

namespace toprop {
int row_rows_per_block(int lx, bool is_double, bool heavy) {
  int g = 0;
  auto q = [&](auto Lc) -> hipError_t {
    constexpr int L = decltype(Lc)::value;
    if (is_double)
      g = heavy ? RowCfg<double, L, true>::G : RowCfg<double, L>::G;
    else
      g = heavy ? RowCfg<float, L, true>::G : RowCfg<float, L>::G;
    return hipSuccess;
  };
  if (dispatch_len(lx, q) != hipSuccess) return 1;
  return g;
}

int row_blocks_per_cu(int lx, bool is_double, bool heavy) {
  int n = 1;
  auto q = [&](auto Lc) -> hipError_t {
    auto per = [&](auto cfg) {
      using C = decltype(cfg);
      using T = typename C::Real;
      const int by_lds = 163840 / row_lds_bytes<T, C::Len, C::R, C::G, true>();
      const int by_threads = 2048 / C::threads;
      n = std::max(1, std::min(by_lds, by_threads));
    };
    constexpr int L = decltype(Lc)::value;
    if (is_double)
      heavy ? per(RowCfg<double, L, true>()) : per(RowCfg<double, L>());
    else
      heavy ? per(RowCfg<float, L, true>()) : per(RowCfg<float, L>());
    return hipSuccess;
  };
  if (dispatch_len(lx, q) != hipSuccess) return 1;
  return n;
}
}  // namespace toprop

namespace toprop {
template <>
hipError_t launch_sum_parts<float>(const float* part, int groups, int64_t n, float* dst, hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL((sum_parts_kernel<float>), dim3((unsigned)blocks), dim3(256), 0, s, part, groups, n, dst);
  return hipGetLastError();
}
}  // namespace toprop
