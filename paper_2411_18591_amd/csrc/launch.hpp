// Host-side launchers for the propagation kernels: map a runtime transform
// length to the kernel instantiation and its launch shape.  Instantiated per
// real type in inst_f32.hip / inst_f64.hip.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace toprop {

constexpr int kMinLen = 8;
constexpr int kMaxLen = 8192;

// Row passes: R points per thread, G rows per workgroup.
template <int L>
struct RowCfg {
  static constexpr int R = L <= 16 ? L : (L <= 2048 ? 8 : 16);
  static constexpr int TT = L / R;
  static constexpr int G = TT >= 256 ? 1 : 256 / TT;
  static constexpr int threads = G * TT;
};

// Column pass: R points per thread, TC columns per workgroup, sized so that
// the LDS exchange buffer (L * TC complex values) stays within 128 KiB.
template <typename T, int L>
struct ColCfg {
  static constexpr int R = L <= 16 ? L : (L <= 256 ? 8 : 16);
  static constexpr int TT = L / R;
  static constexpr int lds_elems = (int)(131072 / sizeof(cx<T>));
  static constexpr int tc0 = lds_elems / L > 16 ? 16 : lds_elems / L;
  static constexpr int tc1 = tc0 < 1 ? 1 : tc0;
  static constexpr int TC = tc1 * TT > 1024 ? 1024 / TT : tc1;
  static constexpr int threads = TC * TT;
};

// Column-tile width for a given column length (runtime query).
int col_tile_width(int ly, bool is_double);

template <typename T>
struct Launch {
  static hipError_t row_fwd(int lx, bool half, int nc, int ny, int nfields, const RowFwdArgs<T>& a,
                            hipStream_t s);
  static hipError_t col(int ly, bool half, int ncols_tiles, int nfields, const ColArgs<T>& a,
                        hipStream_t s);
  static hipError_t row_inv(int lx, bool half, int nc, int ny, int nblocks_y,
                            const RowInvArgs<T>& a, hipStream_t s);
  static hipError_t modulate(int nc, const cx<T>* in, cx<T>* out, int64_t fstride, int64_t cstride,
                             int ny, int nx, int nfields, int adjoint, const ElementParams<T>& el,
                             hipStream_t s);
};

hipError_t launch_reduce_add(const double* src, int64_t n, double scale, double* dst,
                             hipStream_t s);

}  // namespace toprop
