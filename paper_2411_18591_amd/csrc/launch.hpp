// Host-side launchers for the propagation kernels: map a runtime transform
// length to the kernel instantiation and its launch shape.  Instantiated per
// real type in inst_f32.hip / inst_f64.hip.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace toprop {

constexpr int kMinLen = 8;
constexpr int kMaxLen = 8192;

// Row passes: R points per thread, G rows per workgroup.  Heavy kernels
// (the backward row_inv epilogue, three coupled components) keep R = 8 from
// length 2048 on, where R = 16 would cost them occupancy (three coupled
// components at 4096 points: 344 and 408 VGPRs, one wave per SIMD, against
// 187 and 212); so does complex128 at 2048.
// OneRow: one row per workgroup at 2048 points (half the threads, a barrier
// over two waves instead of four); measured faster for the fused forward
// boundary (89.5 -> 84.9 us per launch of 8 fields) and the forward
// row_inv (65.4 -> 63.5 us), slower for row_fwd and the fused backward
// boundary, which keep two rows.
template <typename T, int L, bool Heavy = false, bool OneRow = false>
struct RowCfg {
  using Real = T;
  static constexpr int Len = L;
  static constexpr int R =
      L <= 16 ? L : (L <= 1024 ? 8 : (((L >= 2048 && Heavy) || (L == 2048 && sizeof(T) == 8)) ? 8 : 16));
  static constexpr int TT = L / R;
  static constexpr int G = (OneRow && L == 2048 && R == 16) ? 1 : (TT >= 256 ? 1 : 256 / TT);
  static constexpr int threads = G * TT;
};

// Column pass: R points per thread, TC columns per workgroup, sized so that
// the LDS exchange buffer (L * TC complex values) stays within the variant's
// budget: V = 0: 128 KiB, R = 16; V = 1: 64 KiB, R = 16 (two workgroups per
// CU); V = 2: 64 KiB, R = 8; V = 3: as V = 1, with the next field's column
// segment loaded during the current field's transforms; V = 4: as V = 0,
// with R = 32 for columns of 8192 points (three passes of radix 32/32/8
// instead of 16/16/16/2, two LDS exchanges per transform instead of three,
// at half the waves per CU; at 4096 points it measured slower than V = 0).
constexpr int kColVariants = 5;
constexpr bool col_prefetch(int V) { return V == 3; }
template <typename T, int L, int V = 0>
struct ColCfg {
  static constexpr int R = L <= 16 ? L : (L <= 256 ? 8 : (V == 2 ? 8 : ((V == 4 && L >= 8192) ? 32 : 16)));
  static constexpr int TT = L / R;
  static constexpr int lds_elems = (int)((V == 0 || V == 4 ? 131072 : 65536) / sizeof(cx<T>));
  static constexpr bool PF = col_prefetch(V);
  static constexpr int tc0 = lds_elems / L > 16 ? 16 : lds_elems / L;
  static constexpr int tc1 = tc0 < 1 ? 1 : tc0;
  static constexpr int TC = tc1 * TT > 1024 ? 1024 / TT : tc1;
  static constexpr int threads = TC * TT;
};

// Column-tile width for a given column length and variant (runtime query).
int col_tile_width(int ly, bool is_double, int variant);
// Rows per workgroup of the row passes for a given row length.
int row_rows_per_block(int lx, bool is_double, bool heavy);
// Row-pass workgroups that fit on one CU at once (LDS and thread limits).
int row_blocks_per_cu(int lx, bool is_double, bool heavy);

template <typename T>
struct Launch {
  static hipError_t row_fwd(int lx, bool half, int nc, int ny, int nfields, const RowFwdArgs<T>& a,
                            hipStream_t s);
  static hipError_t col(int ly, bool half, int ncols_tiles, int nfields, int variant,
                        const ColArgs<T>& a, hipStream_t s);
  static hipError_t row_inv(int lx, bool half, int nc, int ny, int nblocks_y,
                            const RowInvArgs<T>& a, hipStream_t s);
  static hipError_t row_mid(int lx, bool half, int ny, int nblocks_y, const RowMidArgs<T>& a, hipStream_t s);
  static hipError_t row_mid_bwd(int lx, bool half, int ny, int nblocks_y, const RowMidBwdArgs<T>& a,
                                hipStream_t s);
  static hipError_t modulate(int nc, const cx<T>* in, cx<T>* out, int64_t fstride, int64_t cstride,
                             int ny, int nx, int nfields, int adjoint, const ElementParams<T>& el,
                             hipStream_t s);
};

hipError_t launch_reduce_add(const double* src, int64_t n, double scale, double* dst,
                             hipStream_t s);

// dst[i] += sum_g part[g * n + i] for g = 0 .. groups-1, in order.
template <typename T>
hipError_t launch_sum_parts(const T* part, int groups, int64_t n, T* dst, hipStream_t s);

hipError_t launch_tf_tables(cx<float>* ex, float* sx, int lx, double inv_lxdx, cx<float>* ey,
                            float* sy, int ly, double inv_lydy, double fres_a, double q_frac,
                            double lam2, hipStream_t s);

}  // namespace toprop
