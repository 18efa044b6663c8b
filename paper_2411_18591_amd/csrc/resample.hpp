// Resampling of fields onto another grid (see resample.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "fft.hpp"

namespace toprop {

// One axis of the map from output samples to fractional input indices:
// t(j) = ((j - half_out) * ratio + shift) + half_in.
struct AxisMap {
  int n_in, n_out;
  int half_in, half_out;  // n / 2 (integer division): the on-axis samples
  double ratio;           // d_out / d_in
  double shift;           // (o_out - o_in) / d_in
};

template <typename W>
struct AxisTap {  // taps of one output sample: w0 on sample i0, w1 on i0 + 1
  int i0;
  int pad;
  W w0, w1;
};
struct AxisRange {  // output samples [lo, hi] whose taps may include an input sample
  int lo, hi;
};

// Bytes of the per-axis tables of one call.
size_t resample_table_bytes(const AxisMap& ay, const AxisMap& ax);

template <typename T>
struct Resample {
  // dst[b] = R src[b] (src on the input grid, dst on the output grid), or
  // with `adjoint` dst[b] = R^T src[b] (src on the output grid, dst on the
  // input grid); mode 0 nearest, 1 bilinear.  `tables`: device workspace of
  // resample_table_bytes(ay, ax) bytes (rebuilt by every call).
  static hipError_t run(const cx<T>* src, cx<T>* dst, int64_t batch, const AxisMap& ay, const AxisMap& ax,
                        int mode, bool adjoint, void* tables, hipStream_t s);
};

}  // namespace toprop
