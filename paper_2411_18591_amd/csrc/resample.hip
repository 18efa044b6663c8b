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
// each side) and recomputes their t exactly as the forward map does, so
// forward and adjoint agree on every weight; no atomics, fixed order.
#include <hip/hip_runtime.h>

#include "resample.hpp"

namespace toprop {

namespace {

__device__ __forceinline__ double frac_index(int j, const AxisMap& m) {
  return __dadd_rn(__dadd_rn(__dmul_rn((double)(j - m.half_out), m.ratio), m.shift), (double)m.half_in);
}

// Taps of output sample j along one axis: up to two (index, weight) pairs.
__device__ __forceinline__ int axis_taps(int j, const AxisMap& m, int mode, int* idx, double* w) {
  // far outside the input window every tap is out of range: clamping keeps
  // the integer conversion defined without changing which taps are inside
  const double t = fmin(fmax(frac_index(j, m), -4.0), (double)m.n_in + 4.0);
  if (mode == 0) {
    idx[0] = (int)floor(__dadd_rn(t, 0.5));
    w[0] = 1.0;
    return 1;
  }
  const double f = floor(t);
  const double a = __dadd_rn(t, -f);
  idx[0] = (int)f;
  w[0] = __dadd_rn(1.0, -a);
  idx[1] = (int)f + 1;
  w[1] = a;
  return 2;
}

// Weight of input index i in output sample j's stencil (0 if absent).
__device__ __forceinline__ double axis_weight(int j, int i, const AxisMap& m, int mode) {
  int idx[2];
  double w[2];
  const int k = axis_taps(j, m, mode, idx, w);
  double r = 0.0;
  for (int q = 0; q < k; ++q)
    if (idx[q] == i) r = w[q];
  return r;
}

// Output samples whose stencil may contain input index i: [lo, hi].
__device__ __forceinline__ void axis_range(int i, const AxisMap& m, int* lo, int* hi) {
  const double a = (double)(i - 1 - m.half_in) - m.shift;
  const double b = (double)(i + 1 - m.half_in) - m.shift;
  double jl = floor(a / m.ratio) + m.half_out - 1;
  double jh = ceil(b / m.ratio) + m.half_out + 1;
  jl = jl < 0 ? 0 : jl;
  jh = jh > m.n_out - 1 ? m.n_out - 1 : jh;
  *lo = (int)jl;
  *hi = (int)jh;
}

}  // namespace

template <typename T>
__global__ void __launch_bounds__(256) resample_kernel(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst,
                                                       int64_t batch, AxisMap ay, AxisMap ax, int mode) {
  const int64_t plane_out = (int64_t)ay.n_out * ax.n_out;
  const int64_t plane_in = (int64_t)ay.n_in * ax.n_in;
  const int64_t total = batch * plane_out;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / plane_out;
    const int64_t p = e - b * plane_out;
    const int q = (int)(p / ax.n_out), r = (int)(p - (int64_t)q * ax.n_out);
    int iy[2], ix[2];
    double wy[2], wx[2];
    const int ky = axis_taps(q, ay, mode, iy, wy);
    const int kx = axis_taps(r, ax, mode, ix, wx);
    const cx<T>* s = src + b * plane_in;
    cx<T> acc = {T(0), T(0)};
    for (int u = 0; u < ky; ++u) {
      if (iy[u] < 0 || iy[u] >= ay.n_in) continue;
      for (int v = 0; v < kx; ++v) {
        if (ix[v] < 0 || ix[v] >= ax.n_in) continue;
        const T w = (T)(wy[u] * wx[v]);
        const cx<T> val = s[(int64_t)iy[u] * ax.n_in + ix[v]];
        acc.x += w * val.x;
        acc.y += w * val.y;
      }
    }
    dst[e] = acc;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) resample_adjoint_kernel(const cx<T>* __restrict__ src,
                                                               cx<T>* __restrict__ dst, int64_t batch,
                                                               AxisMap ay, AxisMap ax, int mode) {
  const int64_t plane_out = (int64_t)ay.n_out * ax.n_out;
  const int64_t plane_in = (int64_t)ay.n_in * ax.n_in;
  const int64_t total = batch * plane_in;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / plane_in;
    const int64_t p = e - b * plane_in;
    const int i = (int)(p / ax.n_in), k = (int)(p - (int64_t)i * ax.n_in);
    int qlo, qhi, rlo, rhi;
    axis_range(i, ay, &qlo, &qhi);
    axis_range(k, ax, &rlo, &rhi);
    const cx<T>* g = src + b * plane_out;
    cx<T> acc = {T(0), T(0)};
    for (int q = qlo; q <= qhi; ++q) {
      const double wy = axis_weight(q, i, ay, mode);
      if (wy == 0.0) continue;
      for (int r = rlo; r <= rhi; ++r) {
        const double wx = axis_weight(r, k, ax, mode);
        if (wx == 0.0) continue;
        const T w = (T)(wy * wx);
        const cx<T> val = g[(int64_t)q * ax.n_out + r];
        acc.x += w * val.x;
        acc.y += w * val.y;
      }
    }
    dst[e] = acc;
  }
}

namespace {
int resample_grid(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (int)(b > 65536 ? 65536 : (b < 1 ? 1 : b));
}
}  // namespace

template <typename T>
hipError_t Resample<T>::run(const cx<T>* src, cx<T>* dst, int64_t batch, const AxisMap& ay, const AxisMap& ax,
                            int mode, bool adjoint, hipStream_t s) {
  if (adjoint) {
    const int64_t n = batch * ay.n_in * ax.n_in;
    hipLaunchKernelGGL((resample_adjoint_kernel<T>), dim3(resample_grid(n)), dim3(256), 0, s, src, dst, batch, ay,
                       ax, mode);
  } else {
    const int64_t n = batch * ay.n_out * ax.n_out;
    hipLaunchKernelGGL((resample_kernel<T>), dim3(resample_grid(n)), dim3(256), 0, s, src, dst, batch, ay, ax,
                       mode);
  }
  return hipGetLastError();
}

template struct Resample<float>;
template struct Resample<double>;

}  // namespace toprop
