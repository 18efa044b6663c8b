// Definitions of the job-queue launchers declared in queue.hpp (included
// once per real type).
#pragma once
#include <algorithm>
#include <map>
#include <mutex>

#include "launch_impl.hpp"
#include "queue.hpp"

namespace toprop {

// Row configuration of the job-queue row passes (which also serve the
// per-job row passes of jobs without element or epilogue): complex64 rows
// of 1024 points and more take 32 points per thread, one LDS exchange fewer
// per transform than the per-job kernels' 8 or 16 (the element and
// epilogue branches those carry leave no registers for it).  Measured
// against the per-job configuration, forward + adjoint per step: 28 jobs of
// 512^2 0.51 -> 0.46 ms, 28 of 1024^2 1.87 -> 1.82 ms, 24 of 2048^2
// 6.93 -> 6.52 ms, 23 of 4096^2 36.9 -> 34.2 ms; rows of 512 points
// unchanged (kept at 8); complex128 keeps the per-job configuration.
template <typename T, int L, bool Heavy = false>
struct QRowCfg {
  using B = RowCfg<T, L, Heavy>;
  static constexpr int R = (L >= 1024 && sizeof(T) == 4) ? 32 : B::R;
  static constexpr int TT = L / R;
  static constexpr int G = TT >= 256 ? 1 : 256 / TT;
  static constexpr int threads = G * TT;
};

// Items of the jobs laid out one after the other from the grids already in
// q.job[k].gx / gy.
template <typename T>
static void queue_lay_out(QueueArgs<T>& q) {
  int next = 0;
  q.items = 0;
  for (int k = 0; k < q.njobs; ++k) {
    q.job[k].first = next;
    q.items = next + q.job[k].gx * q.job[k].gy;
    next = (q.items + 7) & ~7;
  }
}

// Workgroups of `kernel` resident on one CU (cached per kernel).
static int queue_blocks_per_cu(const void* kernel, int threads) {
  static std::mutex mu;
  static std::map<const void*, int> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(kernel);
  if (it != cache.end()) return it->second;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, threads, 0) != hipSuccess || n < 1) n = 1;
  cache[kernel] = n;
  return n;
}

template <typename A>
static hipError_t queue_go(const void* kernel, A& args, int threads, int items, int cus, hipStream_t s) {
  if (items <= 0) return hipSuccess;
  int grid = items;
  if (cus > 0) {
    grid = std::min(items, queue_blocks_per_cu(kernel, threads) * cus);
    if (grid > 8) grid &= ~7;
  }
  void* kargs[] = {&args};
  return hipLaunchKernel(kernel, dim3(grid), dim3(threads), kargs, 0, s);
}

template <typename T>
hipError_t QueueLaunch<T>::row_fwd(int lx, bool half, bool exact, QueueArgs<T>& q, int cus, hipStream_t s) {
  if (!queue_row_len_ok(lx)) return hipErrorInvalidValue;
  return dispatch_len(lx, [&](auto Lc) -> hipError_t {
    constexpr int L = decltype(Lc)::value;
    if constexpr (L < kQueueMinLen || L > kQueueRowMaxLen) {
      return hipErrorInvalidValue;
    } else {
      using C = QRowCfg<T, L>;
      for (int k = 0; k < q.njobs; ++k) {
        q.job[k].gx = (q.job[k].ny + C::G - 1) / C::G;
        q.job[k].gy = (q.job[k].nfields + q.job[k].fpb - 1) / q.job[k].fpb;
      }
      queue_lay_out(q);
      hipError_t e = hipSuccess;
      dispatch_exact<L>(exact, [&](auto ex) {
        constexpr bool EX = decltype(ex)::value;
        const void* kern = half ? reinterpret_cast<const void*>(&row_fwd_queue_kernel<T, L, C::R, C::G, true, EX>)
                                : reinterpret_cast<const void*>(&row_fwd_queue_kernel<T, L, C::R, C::G, false, EX>);
        e = queue_go(kern, q, C::threads, q.items, cus, s);
      });
      return e;
    }
  });
}

template <typename T>
hipError_t QueueLaunch<T>::col(int ly, bool half, bool exact, int variant, ColQueueArgs<T>& cq, int cus,
                               hipStream_t s) {
  if (!queue_len_ok(ly)) return hipErrorInvalidValue;
  QueueArgs<T>& q = cq.q;
  return dispatch_len(ly, [&](auto Lc) -> hipError_t {
    constexpr int L = decltype(Lc)::value;
    if constexpr (L < kQueueMinLen || L > kQueueMaxLen) {
      return hipErrorInvalidValue;
    } else {
      if (q.cpb < 1) return hipErrorInvalidValue;
      for (int k = 0; k < q.njobs; ++k) {
        q.job[k].gx = q.lx / q.cpb;
        q.job[k].gy = (q.job[k].nfields + q.job[k].fpb - 1) / q.job[k].fpb;
      }
      queue_lay_out(q);
      hipError_t e = hipSuccess;
      auto go = [&](auto vc) {
        using C = ColCfg<T, L, decltype(vc)::value>;
        dispatch_exact<L>(exact, [&](auto ex) {
          constexpr bool EX = decltype(ex)::value;
          const void* kern =
              half ? reinterpret_cast<const void*>(&col_queue_kernel<T, L, C::R, C::TC, true, EX, C::PF>)
                   : reinterpret_cast<const void*>(&col_queue_kernel<T, L, C::R, C::TC, false, EX, C::PF>);
          e = queue_go(kern, cq, C::threads, q.items, cus, s);
        });
      };
      switch (variant) {
        case 1: go(std::integral_constant<int, 1>()); break;
        case 2: go(std::integral_constant<int, 2>()); break;
        case 3: go(std::integral_constant<int, 3>()); break;
        case 4: go(std::integral_constant<int, 4>()); break;
        default: go(std::integral_constant<int, 0>()); break;
      }
      return e;
    }
  });
}

template <typename T>
hipError_t QueueLaunch<T>::row_inv(int lx, bool half, bool exact, bool bwd, QueueArgs<T>& q, int cus,
                                   hipStream_t s) {
  if (!queue_row_len_ok(lx)) return hipErrorInvalidValue;
  return dispatch_len(lx, [&](auto Lc) -> hipError_t {
    constexpr int L = decltype(Lc)::value;
    if constexpr (L < kQueueMinLen || L > kQueueRowMaxLen) {
      return hipErrorInvalidValue;
    } else {
      hipError_t e = hipSuccess;
      auto go = [&](auto bc) {
        constexpr bool B = decltype(bc)::value;
        using C = QRowCfg<T, L, B>;
        for (int k = 0; k < q.njobs; ++k) {
          q.job[k].gx = (q.job[k].ny + C::G - 1) / C::G;
          q.job[k].gy = B ? 1 : (q.job[k].nfields + q.job[k].fpb - 1) / q.job[k].fpb;
        }
        queue_lay_out(q);
        dispatch_exact<L>(exact, [&](auto ex) {
          constexpr bool EX = decltype(ex)::value;
          const void* kern =
              half ? reinterpret_cast<const void*>(&row_inv_queue_kernel<T, L, C::R, C::G, true, B, EX>)
                   : reinterpret_cast<const void*>(&row_inv_queue_kernel<T, L, C::R, C::G, false, B, EX>);
          e = queue_go(kern, q, C::threads, q.items, cus, s);
        });
      };
      if (bwd)
        go(std::true_type());
      else
        go(std::false_type());
      return e;
    }
  });
}

}  // namespace toprop
