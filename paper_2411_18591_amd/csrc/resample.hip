// Resampling of sampled fields onto another grid (TorchOptics paper, section
// "Computational Fourier optics": when the output grid's spacing differs
// from the input's, the field is propagated on the input spacing and then
// interpolated onto the output grid, bilinearly or to the nearest sample).
//
// Along each axis, output sample j sits at the fractional input index
//   t(j) = ((j - n_out/2) d_out/d_in + (o_out - o_in)/d_in) + n_in/2,
// evaluated in FP64 without contraction (the products and sums round
// exactly as written, so the integer decisions are reproducible and the
// map is exact on identical grids).  Bilinear: i0 = floor(t), a = t - i0,
// weights (1 - a, a) on samples i0 and i0 + 1; nearest: sample
// floor(t + 1/2).  Samples outside the input window read zero.  The 2-D
// weights are the products of the axis weights; the taps are summed in the
// order (y0, x0), (y0, x1), (y1, x0), (y1, x1).
//
// The adjoint (the weights are real: the transpose) is a gather, one thread
// per input sample: it visits the output samples whose stencil can contain
// it (a range of each axis found by inverting t, widened by one sample on
// each side) and takes their weights from the same tap tables the forward
// map uses, so forward and adjoint agree on every weight; no atomics, fixed
// order.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "resample.hpp"

namespace toprop {

namespace {

__device__ __forceinline__ double frac_index(int j, const AxisMap& m) {
  return __dadd_rn(__dadd_rn(__dmul_rn((double)(j - m.half_out), m.ratio), m.shift), (double)m.half_in);
}

// Fractional index clamped to [-4, n_in + 4]: far outside the input window
// every tap is out of range, and the clamp keeps the integer conversion
// defined without changing which taps are inside.
__device__ __forceinline__ double clamped_index(int j, const AxisMap& m) {
  return fmin(fmax(frac_index(j, m), -4.0), (double)m.n_in + 4.0);
}

// First tap index of output sample j (nondecreasing in j).
__device__ __forceinline__ int first_tap(int j, const AxisMap& m, int mode) {
  const double t = clamped_index(j, m);
  return (int)floor(mode == 0 ? __dadd_rn(t, 0.5) : t);
}

// Smallest j in [0, n_out] with first_tap(j) >= v (n_out if none).
__device__ __forceinline__ int lower_bound_tap(int v, const AxisMap& m, int mode) {
  int lo = 0, hi = m.n_out;
  while (lo < hi) {
    const int mid = lo + (hi - lo) / 2;
    if (first_tap(mid, m, mode) >= v)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
}

}  // namespace

// Per-axis tables, built once per call: the taps of every output sample
// (index i0 and weights w0, w1 of samples i0 and i0 + 1; nearest: w1 = 0),
// and for every input sample i the range of output samples whose taps
// include it: those with i0 in [i - 1, i] (bilinear) or i0 = i (nearest),
// found by binary search since i0 does not decrease with the output index.
template <typename W>
__global__ void __launch_bounds__(256) resample_tables_kernel(AxisMap ay, AxisMap ax, int mode, AxisTap<W>* tap_y,
                                                              AxisTap<W>* tap_x, AxisRange* rng_y, AxisRange* rng_x) {
  const AxisMap& m = blockIdx.y == 0 ? ay : ax;
  AxisTap<W>* tap = blockIdx.y == 0 ? tap_y : tap_x;
  AxisRange* rng = blockIdx.y == 0 ? rng_y : rng_x;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < m.n_out) {
    const double t = clamped_index(e, m);
    AxisTap<W> a;
    if (mode == 0) {
      a.i0 = (int)floor(__dadd_rn(t, 0.5));
      a.w0 = W(1);
      a.w1 = W(0);
    } else {
      const double f = floor(t);
      const double fr = __dadd_rn(t, -f);
      a.i0 = (int)f;
      a.w0 = (W)__dadd_rn(1.0, -fr);
      a.w1 = (W)fr;
    }
    tap[e] = a;
  } else if (e < m.n_out + m.n_in) {
    const int i = e - m.n_out;
    AxisRange r;
    r.lo = lower_bound_tap(mode == 0 ? i : i - 1, m, mode);
    r.hi = lower_bound_tap(i + 1, m, mode) - 1;
    rng[i] = r;
  }
}

// Forward: a workgroup per output row q (and a share of the fields); the
// row's taps are uniform over the workgroup, the columns' taps are coalesced
// table reads.
template <typename T>
__global__ void __launch_bounds__(256) resample_kernel(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst,
                                                       int64_t batch, int ny, int nx, int my, int mx,
                                                       const AxisTap<double>* __restrict__ tap_y,
                                                       const AxisTap<double>* __restrict__ tap_x) {
  const int q = blockIdx.x;
  const AxisTap<double> ty = tap_y[q];
  const int iy[2] = {ty.i0, ty.i0 + 1};
  const double wy[2] = {ty.w0, ty.w1};
  // FB fields at a time: their 4 FB gathers are in flight together
  constexpr int FB = 4;
  for (int r = threadIdx.x; r < mx; r += blockDim.x) {
    const AxisTap<double> tx = tap_x[r];
    const int ix[2] = {tx.i0, tx.i0 + 1};
    const double wx[2] = {tx.w0, tx.w1};
    int64_t off[2][2];
    T w[2][2];
    bool in[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        in[u][v] = iy[u] >= 0 && iy[u] < ny && ix[v] >= 0 && ix[v] < nx;
        off[u][v] = in[u][v] ? (int64_t)iy[u] * nx + ix[v] : 0;
        w[u][v] = (T)(wy[u] * wx[v]);
      }
    for (int64_t b0 = blockIdx.y; b0 < batch; b0 += (int64_t)FB * gridDim.y) {
      cx<T> val[FB][2][2];
#pragma unroll
      for (int k = 0; k < FB; ++k) {
        const int64_t b = b0 + (int64_t)k * gridDim.y;
        const cx<T>* s = src + (b < batch ? b : 0) * ((int64_t)ny * nx);
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
          for (int v = 0; v < 2; ++v)
            val[k][u][v] = (b < batch && in[u][v]) ? s[off[u][v]] : cx<T>{T(0), T(0)};
      }
#pragma unroll
      for (int k = 0; k < FB; ++k) {
        const int64_t b = b0 + (int64_t)k * gridDim.y;
        if (b >= batch) break;
        cx<T> acc = {T(0), T(0)};
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
          for (int v = 0; v < 2; ++v) {
            if (!in[u][v]) continue;
            acc.x += w[u][v] * val[k][u][v].x;
            acc.y += w[u][v] * val[k][u][v].y;
          }
        dst[b * ((int64_t)my * mx) + (int64_t)q * mx + r] = acc;
      }
    }
  }
}

__device__ __forceinline__ double tap_weight(const AxisTap<double>& t, int i) {
  return t.i0 == i ? t.w0 : (t.i0 + 1 == i ? t.w1 : 0.0);
}

// Adjoint: a workgroup per input row i (and a share of the fields); a
// gather over the output samples whose taps include (i, k), in a fixed
// order.
template <typename T>
__global__ void __launch_bounds__(256) resample_adjoint_kernel(const cx<T>* __restrict__ src,
                                                               cx<T>* __restrict__ dst, int64_t batch, int ny,
                                                               int nx, int my, int mx,
                                                               const AxisTap<double>* __restrict__ tap_y,
                                                               const AxisTap<double>* __restrict__ tap_x,
                                                               const AxisRange* __restrict__ rng_y,
                                                               const AxisRange* __restrict__ rng_x) {
  const int i = blockIdx.x;
  const AxisRange ry = rng_y[i];
  constexpr int FB = 4;  // fields whose gathers are in flight together
  for (int k = threadIdx.x; k < nx; k += blockDim.x) {
    const AxisRange rx = rng_x[k];
    for (int64_t b0 = blockIdx.y; b0 < batch; b0 += (int64_t)FB * gridDim.y) {
      const cx<T>* g[FB];
      bool ok[FB];
#pragma unroll
      for (int f = 0; f < FB; ++f) {
        const int64_t b = b0 + (int64_t)f * gridDim.y;
        ok[f] = b < batch;
        g[f] = src + (ok[f] ? b : 0) * ((int64_t)my * mx);
      }
      cx<T> acc[FB];
#pragma unroll
      for (int f = 0; f < FB; ++f) acc[f] = {T(0), T(0)};
      for (int q = ry.lo; q <= ry.hi; ++q) {
        const double wy = tap_weight(tap_y[q], i);
        if (wy == 0.0) continue;
        for (int r = rx.lo; r <= rx.hi; ++r) {
          const double wx = tap_weight(tap_x[r], k);
          if (wx == 0.0) continue;
          const T w = (T)(wy * wx);
          const int64_t o = (int64_t)q * mx + r;
          cx<T> val[FB];
#pragma unroll
          for (int f = 0; f < FB; ++f) val[f] = ok[f] ? g[f][o] : cx<T>{T(0), T(0)};
#pragma unroll
          for (int f = 0; f < FB; ++f) {
            acc[f].x += w * val[f].x;
            acc[f].y += w * val[f].y;
          }
        }
      }
#pragma unroll
      for (int f = 0; f < FB; ++f)
        if (ok[f]) dst[(b0 + (int64_t)f * gridDim.y) * ((int64_t)ny * nx) + (int64_t)i * nx + k] = acc[f];
    }
  }
}

size_t resample_table_bytes(const AxisMap& ay, const AxisMap& ax) {
  return (size_t)(ay.n_out + ax.n_out) * sizeof(AxisTap<double>) + (size_t)(ay.n_in + ax.n_in) * sizeof(AxisRange);
}

template <typename T>
hipError_t Resample<T>::run(const cx<T>* src, cx<T>* dst, int64_t batch, const AxisMap& ay, const AxisMap& ax,
                            int mode, bool adjoint, void* tables, hipStream_t s) {
  AxisTap<double>* tap_y = static_cast<AxisTap<double>*>(tables);
  AxisTap<double>* tap_x = tap_y + ay.n_out;
  AxisRange* rng_y = reinterpret_cast<AxisRange*>(tap_x + ax.n_out);
  AxisRange* rng_x = rng_y + ay.n_in;
  const int tn = std::max(ay.n_out + ay.n_in, ax.n_out + ax.n_in);
  hipLaunchKernelGGL((resample_tables_kernel<double>), dim3((tn + 255) / 256, 2), dim3(256), 0, s, ay, ax, mode,
                     tap_y, tap_x, rng_y, rng_x);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // rows x field shares: enough workgroups to fill the GPU several times
  const int rows = adjoint ? ay.n_in : ay.n_out;
  const int zb = (int)std::max<int64_t>(1, std::min<int64_t>(batch, (16384 + rows - 1) / rows));
  if (adjoint) {
    hipLaunchKernelGGL((resample_adjoint_kernel<T>), dim3(ay.n_in, zb), dim3(256), 0, s, src, dst, batch, ay.n_in,
                       ax.n_in, ay.n_out, ax.n_out, tap_y, tap_x, rng_y, rng_x);
  } else {
    hipLaunchKernelGGL((resample_kernel<T>), dim3(ay.n_out, zb), dim3(256), 0, s, src, dst, batch, ay.n_in,
                       ax.n_in, ay.n_out, ax.n_out, tap_y, tap_x);
  }
  return hipGetLastError();
}

template struct Resample<float>;
template struct Resample<double>;

}  // namespace toprop
