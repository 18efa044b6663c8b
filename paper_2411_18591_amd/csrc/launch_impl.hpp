// Definitions of the launchers declared in launch.hpp (included once per
// real type).
#pragma once
#include "launch.hpp"

namespace toprop {

// Calls f(std::integral_constant<int, L>) for the runtime power of two L.
template <typename F>
static hipError_t dispatch_len(int L, F&& f) {
  switch (L) {
    case 8: return f(std::integral_constant<int, 8>());
    case 16: return f(std::integral_constant<int, 16>());
    case 32: return f(std::integral_constant<int, 32>());
    case 64: return f(std::integral_constant<int, 64>());
    case 128: return f(std::integral_constant<int, 128>());
    case 256: return f(std::integral_constant<int, 256>());
    case 512: return f(std::integral_constant<int, 512>());
    case 1024: return f(std::integral_constant<int, 1024>());
    case 2048: return f(std::integral_constant<int, 2048>());
    case 4096: return f(std::integral_constant<int, 4096>());
    case 8192: return f(std::integral_constant<int, 8192>());
    default: return hipErrorInvalidValue;
  }
}

// Calls f(std::bool_constant<EX>) with EX = `exact` where exact-width
// kernels are instantiated (transforms of 256 points and more), else false.
template <int L, typename F>
static void dispatch_exact(bool exact, F&& f) {
  if constexpr (L >= 256) {
    if (exact) {
      f(std::true_type());
      return;
    }
  }
  f(std::false_type());
}

template <typename T>
hipError_t Launch<T>::row_fwd(int lx, bool half, int nc, int ny, int nfields, const RowFwdArgs<T>& a,
                              hipStream_t s) {
  return dispatch_len(lx, [&](auto Lc) -> hipError_t {
    constexpr int L = decltype(Lc)::value;
    const int fpb = a.fpb > 0 ? a.fpb : 1;
    const bool exact = a.nx == (half ? L / 2 : L);
    dispatch_exact<L>(exact, [&](auto ex) {
      constexpr bool EX = decltype(ex)::value;
      if (nc == 3) {
        using C = RowCfg<T, L, true>;
        dim3 grid((ny + C::G - 1) / C::G, (nfields + fpb - 1) / fpb);
        if (half)
          hipLaunchKernelGGL((row_fwd_kernel<T, L, C::R, C::G, true, 3, EX>), grid, dim3(C::threads), 0, s, a);
        else
          hipLaunchKernelGGL((row_fwd_kernel<T, L, C::R, C::G, false, 3, EX>), grid, dim3(C::threads), 0, s, a);
      } else {
        using C = RowCfg<T, L>;
        dim3 grid((ny + C::G - 1) / C::G, (nfields + fpb - 1) / fpb);
        if (half)
          hipLaunchKernelGGL((row_fwd_kernel<T, L, C::R, C::G, true, 1, EX>), grid, dim3(C::threads), 0, s, a);
        else
          hipLaunchKernelGGL((row_fwd_kernel<T, L, C::R, C::G, false, 1, EX>), grid, dim3(C::threads), 0, s, a);
      }
    });
    return hipGetLastError();
  });
}

template <typename T>
hipError_t Launch<T>::col(int ly, bool half, int ntiles, int nfields, int variant,
                          const ColArgs<T>& a, hipStream_t s) {
  return dispatch_len(ly, [&](auto Lc) -> hipError_t {
    constexpr int L = decltype(Lc)::value;
    const bool exact = a.ny == (half ? L / 2 : L);
    auto go = [&](auto vc) {
      using C = ColCfg<T, L, decltype(vc)::value>;
      dim3 grid(ntiles, (nfields + a.fpc - 1) / a.fpc);
      dim3 block(C::threads);
      dispatch_exact<L>(exact, [&](auto ex) {
        constexpr bool EX = decltype(ex)::value;
        if (half)
          hipLaunchKernelGGL((col_kernel<T, L, C::R, C::TC, true, EX, C::PF>), grid, block, 0, s, a);
        else
          hipLaunchKernelGGL((col_kernel<T, L, C::R, C::TC, false, EX, C::PF>), grid, block, 0, s, a);
      });
    };
    switch (variant) {
      case 1: go(std::integral_constant<int, 1>()); break;
      case 2: go(std::integral_constant<int, 2>()); break;
      case 3: go(std::integral_constant<int, 3>()); break;
      case 4: go(std::integral_constant<int, 4>()); break;
      default: go(std::integral_constant<int, 0>()); break;
    }
    return hipGetLastError();
  });
}

template <typename T>
hipError_t Launch<T>::row_mid(int lx, bool half, int ny, int nblocks_y, const RowMidArgs<T>& a,
                              hipStream_t s) {
  return dispatch_len(lx, [&](auto Lc) -> hipError_t {
    constexpr int L = decltype(Lc)::value;
    using C = RowCfg<T, L, false, true>;
    dim3 grid((ny + C::G - 1) / C::G, nblocks_y);
    dim3 block(C::threads);
    dispatch_exact<L>(a.nx == (half ? L / 2 : L), [&](auto ex) {
      constexpr bool EX = decltype(ex)::value;
      if (half)
        hipLaunchKernelGGL((row_mid_kernel<T, L, C::R, C::G, true, EX>), grid, block, 0, s, a);
      else
        hipLaunchKernelGGL((row_mid_kernel<T, L, C::R, C::G, false, EX>), grid, block, 0, s, a);
    });
    return hipGetLastError();
  });
}

template <typename T>
hipError_t Launch<T>::row_mid_bwd(int lx, bool half, int ny, int nblocks_y, const RowMidBwdArgs<T>& a,
                                  hipStream_t s) {
  return dispatch_len(lx, [&](auto Lc) -> hipError_t {
    constexpr int L = decltype(Lc)::value;
    using C = RowCfg<T, L>;
    dim3 grid((ny + C::G - 1) / C::G, nblocks_y);
    dim3 block(C::threads);
    dispatch_exact<L>(a.nx == (half ? L / 2 : L), [&](auto ex) {
      constexpr bool EX = decltype(ex)::value;
      if (half)
        hipLaunchKernelGGL((row_mid_bwd_kernel<T, L, C::R, C::G, true, EX>), grid, block, 0, s, a);
      else
        hipLaunchKernelGGL((row_mid_bwd_kernel<T, L, C::R, C::G, false, EX>), grid, block, 0, s, a);
    });
    return hipGetLastError();
  });
}

template <typename T>
hipError_t Launch<T>::row_inv(int lx, bool half, int nc, int ny, int nblocks_y,
                              const RowInvArgs<T>& a, hipStream_t s) {
  return dispatch_len(lx, [&](auto Lc) -> hipError_t {
    constexpr int L = decltype(Lc)::value;
    const bool exact = a.nx == (half ? L / 2 : L);
    auto go = [&](auto bwd) {
      constexpr bool B = decltype(bwd)::value;
      dispatch_exact<L>(exact, [&](auto ex) {
        constexpr bool EX = decltype(ex)::value;
        if (nc == 3) {
          using C = RowCfg<T, L, true>;
          dim3 grid((ny + C::G - 1) / C::G, nblocks_y);
          if (half)
            hipLaunchKernelGGL((row_inv_kernel<T, L, C::R, C::G, true, 3, B, EX>), grid, dim3(C::threads), 0, s, a);
          else
            hipLaunchKernelGGL((row_inv_kernel<T, L, C::R, C::G, false, 3, B, EX>), grid, dim3(C::threads), 0, s, a);
        } else {
          using C = RowCfg<T, L, B, !B>;
          dim3 grid((ny + C::G - 1) / C::G, nblocks_y);
          if (half)
            hipLaunchKernelGGL((row_inv_kernel<T, L, C::R, C::G, true, 1, B, EX>), grid, dim3(C::threads), 0, s, a);
          else
            hipLaunchKernelGGL((row_inv_kernel<T, L, C::R, C::G, false, 1, B, EX>), grid, dim3(C::threads), 0, s, a);
        }
      });
    };
    if (a.backward)
      go(std::true_type());
    else
      go(std::false_type());
    return hipGetLastError();
  });
}

template <typename T>
hipError_t Launch<T>::modulate(int nc, const cx<T>* in, cx<T>* out, int64_t fstride, int64_t cstride,
                               int ny, int nx, int nfields, int adjoint, const ElementParams<T>& el,
                               hipStream_t s) {
  const int64_t total = (int64_t)ny * nx * nfields;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  if (nc == 3)
    hipLaunchKernelGGL((modulate_kernel<T, 3>), dim3((unsigned)blocks), dim3(256), 0, s, in, out,
                       fstride, cstride, ny, nx, nfields, adjoint, el);
  else
    hipLaunchKernelGGL((modulate_kernel<T, 1>), dim3((unsigned)blocks), dim3(256), 0, s, in, out,
                       fstride, cstride, ny, nx, nfields, adjoint, el);
  return hipGetLastError();
}

}  // namespace toprop
