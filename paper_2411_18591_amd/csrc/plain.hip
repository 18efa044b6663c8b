// Plain (unfused) form of the propagation, the comparison baseline for the
// fused kernels: one field per launch sequence and one kernel per step of
// the pipeline of Eq. (field_propagation_tf) — modulate, zero-pad into a
// full py x px array, row FFTs, column FFTs, multiply by a stored transfer
// function table, inverse column and row FFTs, crop and scale.  Every
// intermediate is a full array in HBM.  The FFT building blocks are the same
// Stockham register/LDS transforms as the fused path; only the fusion and the
// batching are absent.  It is also the path for padded extents that are not
// powers of two: their lines go through the mixed-radix transform (lengths
// 2^a 3^b 5^c 7^d, with the fused sequence of run_mixed) or Bluestein's.
#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/toprop.h"
#include "launch_impl.hpp"
#include "plain.hpp"

namespace toprop {

template <typename T>
__global__ void __launch_bounds__(256) plain_modulate_kernel(const cx<T>* in, cx<T>* out, int ny, int nx,
                                                             ElementParams<T> el, int conj) {
  const int64_t n = (int64_t)ny * nx;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(i / nx), x = (int)(i % nx);
    cx<T> m = scalar_modulation(el, ny, nx, y, x);
    if (conj) m.y = -m.y;
    out[i] = cmul(m, in[i]);
  }
}

template <typename T>
__global__ void __launch_bounds__(256) plain_pad_kernel(const cx<T>* in, cx<T>* pad, int ny, int nx, int py,
                                                        int px) {
  const int64_t n = (int64_t)py * px;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(i / px), x = (int)(i % px);
    pad[i] = (y < ny && x < nx) ? in[(int64_t)y * nx + x] : cx<T>{T(0), T(0)};
  }
}

template <typename T>
__global__ void __launch_bounds__(256) plain_crop_kernel(const cx<T>* pad, cx<T>* out, int ny, int nx, int px,
                                                         T scale) {
  const int64_t n = (int64_t)ny * nx;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(i / nx), x = (int)(i % nx);
    out[i] = cscale(pad[(int64_t)y * px + x], scale);
  }
}

// Transfer function of every bin of the padded grid, stored as a table.
template <typename T>
__global__ void __launch_bounds__(256) plain_table_kernel(cx<T>* H, int py, int px, TransferParams p,
                                                          int transposed) {
  const int64_t n = (int64_t)py * px;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int ky = transposed ? (int)(i % py) : (int)(i / px);
    const int kx = transposed ? (int)(i / py) : (int)(i % px);
    H[i] = transfer_at<T>(kx, ky, px, py, p);
  }
}

template <typename T>
__global__ void __launch_bounds__(256) plain_intensity_kernel(const cx<T>* u, T* I, int64_t n, T scale) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const cx<T> v = u[i];
    I[i] += scale * (v.x * v.x + v.y * v.y);
  }
}

template <typename T>
__global__ void __launch_bounds__(256) plain_mul_kernel(cx<T>* a, const cx<T>* H, int64_t n, int conj) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    cx<T> h = H[i];
    if (conj) h.y = -h.y;
    a[i] = cmul(a[i], h);
  }
}

// In-place FFTs of `rows` contiguous rows of length L.
template <typename T, int L, int R, int G, int D>
__global__ void __launch_bounds__(G * (L / R)) plain_row_fft_kernel(cx<T>* a, int rows, const cx<T>* tw) {
  constexpr int TT = L / R;
  __shared__ cx<T> lds[G * lds_len<1>(L)];
  const int g = threadIdx.x / TT, j = threadIdx.x % TT;
  const int row = blockIdx.x * G + g;
  const bool ok = row < rows;
  cx<T>* p = a + (int64_t)(ok ? row : 0) * L;
  cx<T> v[R];
#pragma unroll
  for (int m = 0; m < R; ++m) v[m] = ok ? p[j + m * TT] : cx<T>{T(0), T(0)};
  fft_wg<T, L, R, D, false, 1>(v, j, lds + g * lds_len<1>(L), tw);
  if (ok) {
#pragma unroll
    for (int m = 0; m < R; ++m) p[j + m * TT] = v[m];
  }
}

// In-place FFTs of the columns of a row-major [L][lx] array, TC columns per
// block.
template <typename T, int L, int R, int TC, int D>
__global__ void __launch_bounds__(TC * (L / R)) plain_col_fft_kernel(cx<T>* a, int lx, const cx<T>* tw) {
  constexpr int TT = L / R;
  __shared__ cx<T> lds[lds_len<TC>(L) * TC];
  const int c = threadIdx.x % TC, j = threadIdx.x / TC;
  const int col = blockIdx.x * TC + c;
  const bool ok = col < lx;
  cx<T> v[R];
#pragma unroll
  for (int m = 0; m < R; ++m) v[m] = ok ? a[(int64_t)(j + m * TT) * lx + col] : cx<T>{T(0), T(0)};
  fft_wg<T, L, R, D, false, TC>(v, j, lds + c, tw);
  if (ok) {
#pragma unroll
    for (int m = 0; m < R; ++m) a[(int64_t)(j + m * TT) * lx + col] = v[m];
  }
}

// MSE / weighted-intensity loss of one field: gradient and per-block loss
// partial sums.
template <typename T>
__global__ void __launch_bounds__(256) plain_loss_kernel(const cx<T>* u, const T* ref, cx<T>* grad,
                                                         double* partial, int64_t n, int kind, T scale) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const cx<T> v = u[i];
    const T I = v.x * v.x + v.y * v.y;
    if (kind == EPI_MSE) {
      const T d = I - ref[i];
      acc += (double)d * (double)d;
      grad[i] = cscale(v, T(4) * scale * d);
    } else {
      acc += (double)ref[i] * (double)I;
      grad[i] = cscale(v, T(2) * scale * ref[i]);
    }
  }
  const double s = block_sum<256>(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// grad_phase += Im(g conj(M u)) for one field (M = exp(i phi)).
template <typename T>
__global__ void __launch_bounds__(256) plain_phase_grad_kernel(const cx<T>* g, const cx<T>* u, T* gphi,
                                                               int ny, int nx, ElementParams<T> el) {
  const int64_t n = (int64_t)ny * nx;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(i / nx), x = (int)(i % nx);
    const cx<T> um = cmul(scalar_modulation(el, ny, nx, y, x), u[i]);
    gphi[i] += g[i].y * um.x - g[i].x * um.y;
  }
}

// Per-block partial sums, in FP64, of the lens focal-length gradient of
// one field: sum over pixels of d(lens phase)/df * Im(g conj(M u)), where
// M u is the modulated saved input.  Fixed grid and tree order:
// deterministic.
template <typename T>
__global__ void __launch_bounds__(256) plain_lens_grad_kernel(const cx<T>* g, const cx<T>* u, double* partial,
                                                              int ny, int nx, ElementParams<T> el, double f) {
  __shared__ double red[256];
  const int64_t n = (int64_t)ny * nx;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(i / nx), x = (int)(i % nx);
    const cx<T> um = cmul(scalar_modulation(el, ny, nx, y, x), u[i]);
    const double im = (double)g[i].y * (double)um.x - (double)g[i].x * (double)um.y;
    acc += lens_dphase_df(el, ny, nx, y, x, f) * im;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

namespace {
int grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (int)(b > 16384 ? 16384 : (b < 1 ? 1 : b));
}
}  // namespace

template <typename T>
hipError_t Plain<T>::run_mixed(const PlainJob<T>& pj, hipStream_t s) {
  const int ny = pj.ny, nx = pj.nx, py = pj.py, px = pj.px;
  const int64_t nb = pj.nbatch;
  MixedPlan qx = pj.fx.mp, qy = pj.fy.mp;  // power-of-two extents: plans of radix 16, 8, 4, 2
  if ((!qx.np && !mixed_plan(px, &qx, true)) || (!qy.np && !mixed_plan(py, &qy, true)) || !pj.tr || nb < 1 ||
      nb * ny > INT32_MAX || nb * px > INT32_MAX)
    return hipErrorInvalidValue;
  hipError_t e;
  // rows: the ny field rows, modulated by the element and zero-extended to
  // px, into pad [ny][px]
  MixedArgs<T> r{};
  r.el = pj.el;
  r.el.flags &= EL_PHASE | EL_COMPLEX | EL_LENS;
  r.in = pj.in;
  r.in_ls = nx;
  r.in_es = 1;
  r.nin = nx;
  r.out = pj.pad;
  r.out_ls = px;
  r.out_es = 1;
  r.nout = px;
  r.scale = T(1);
  r.nlines = (int)(nb * ny);
  r.field_rows = ny;
  r.L = px;
  r.plan = qx;
  r.tw = pj.fx.tw;
  if ((e = Mixed<T>::launch(r, -1, s)) != hipSuccess) return e;
  // columns as rows of tr [px][ny]: zero-extended to py, forward, times the
  // transposed table, inverse, cropped to ny, in place
  if ((e = Mixed<T>::transpose(pj.pad, pj.tr, ny, px, nb, s)) != hipSuccess) return e;
  MixedArgs<T> c{};
  c.in = pj.tr;
  c.out = pj.tr;
  c.in_ls = c.out_ls = ny;
  c.in_es = c.out_es = 1;
  c.nin = c.nout = ny;
  c.h = pj.hcalc ? nullptr : pj.H;
  c.h_ls = py;
  c.conj = pj.conj;
  c.hcalc = pj.hcalc;
  c.tp = pj.tp;
  c.scale = T(1);
  c.nlines = (int)(nb * px);
  c.h_lines = px;
  c.L = py;
  c.plan = qy;
  c.tw = pj.fy.tw;
  if ((e = Mixed<T>::launch(c, 0, s)) != hipSuccess) return e;
  if ((e = Mixed<T>::transpose(pj.tr, pj.pad, px, ny, nb, s)) != hipSuccess) return e;
  // inverse rows, cropped to nx and scaled, into the output
  r.el.flags = 0;
  r.in = pj.pad;
  r.in_ls = px;
  r.nin = px;
  r.out = pj.out;
  r.out_ls = nx;
  r.nout = nx;
  r.scale = (T)(1.0 / ((double)py * (double)px));
  return Mixed<T>::launch(r, +1, s);
}

template <typename T>
hipError_t Plain<T>::run(const PlainJob<T>& pj, hipStream_t s) {
  if (pj.ht) return run_mixed(pj, s);
  const int ny = pj.ny, nx = pj.nx, py = pj.py, px = pj.px;
  const int64_t npad = (int64_t)py * px, nf = (int64_t)ny * nx;
  hipError_t e;
  // 1. modulation (forward: M in; backward: none here)
  const cx<T>* src = pj.in;
  if (pj.el.flags & (EL_PHASE | EL_COMPLEX | EL_LENS)) {
    hipLaunchKernelGGL((plain_modulate_kernel<T>), dim3(grid_for(nf)), dim3(256), 0, s, pj.in, pj.tmp,
                       ny, nx, pj.el, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    src = pj.tmp;
  }
  // 2. zero padding
  hipLaunchKernelGGL((plain_pad_kernel<T>), dim3(grid_for(npad)), dim3(256), 0, s, src, pj.pad, ny, nx, py,
                     px);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // 3-4. forward FFT: rows, then columns
  if ((e = rows_any(pj.fx, pj.pad, py, -1, s)) != hipSuccess) return e;
  if ((e = cols_any(pj.fy, pj.pad, px, -1, s, pj.tr)) != hipSuccess) return e;
  // 5. transfer function from the stored table
  hipLaunchKernelGGL((plain_mul_kernel<T>), dim3(grid_for(npad)), dim3(256), 0, s, pj.pad, pj.H, npad,
                     pj.conj);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // 6-7. inverse FFT: columns, then rows
  if ((e = cols_any(pj.fy, pj.pad, px, +1, s, pj.tr)) != hipSuccess) return e;
  if ((e = rows_any(pj.fx, pj.pad, py, +1, s)) != hipSuccess) return e;
  // 8. crop and scale
  hipLaunchKernelGGL((plain_crop_kernel<T>), dim3(grid_for(nf)), dim3(256), 0, s, pj.pad, pj.out, ny, nx,
                     px, (T)(1.0 / ((double)py * (double)px)));
  return hipGetLastError();
}

template <typename T>
hipError_t Plain<T>::table(cx<T>* H, int py, int px, const TransferParams& p, hipStream_t s, bool transposed) {
  hipLaunchKernelGGL((plain_table_kernel<T>), dim3(grid_for((int64_t)py * px)), dim3(256), 0, s, H, py, px,
                     p, transposed ? 1 : 0);
  return hipGetLastError();
}

template <typename T>
hipError_t Plain<T>::rows(int L, cx<T>* a, int nrows, int dir, const cx<T>* tw, hipStream_t s) {
  return dispatch_len(L, [&](auto Lc) -> hipError_t {
    constexpr int LL = decltype(Lc)::value;
    using C = RowCfg<T, LL>;
    dim3 grid((nrows + C::G - 1) / C::G);
    if (dir < 0)
      hipLaunchKernelGGL((plain_row_fft_kernel<T, LL, C::R, C::G, -1>), grid, dim3(C::threads), 0, s, a, nrows,
                         tw);
    else
      hipLaunchKernelGGL((plain_row_fft_kernel<T, LL, C::R, C::G, +1>), grid, dim3(C::threads), 0, s, a, nrows,
                         tw);
    return hipGetLastError();
  });
}

template <typename T>
hipError_t Plain<T>::cols(int L, cx<T>* a, int lx, int dir, const cx<T>* tw, hipStream_t s) {
  return dispatch_len(L, [&](auto Lc) -> hipError_t {
    constexpr int LL = decltype(Lc)::value;
    using C = ColCfg<T, LL, 1>;
    dim3 grid((lx + C::TC - 1) / C::TC);
    if (dir < 0)
      hipLaunchKernelGGL((plain_col_fft_kernel<T, LL, C::R, C::TC, -1>), grid, dim3(C::threads), 0, s, a, lx,
                         tw);
    else
      hipLaunchKernelGGL((plain_col_fft_kernel<T, LL, C::R, C::TC, +1>), grid, dim3(C::threads), 0, s, a, lx,
                         tw);
    return hipGetLastError();
  });
}

template <typename T>
hipError_t Plain<T>::rows_any(const LineFft<T>& f, cx<T>* a, int nrows, int dir, hipStream_t s) {
  if (f.mp.np > 0) return Mixed<T>::lines(f.L, f.mp, f.tw, a, nrows, f.L, 1, dir, s);
  return f.M == 0 ? rows(f.L, a, nrows, dir, f.tw, s) : Bluestein<T>::rows(f, a, nrows, dir, s);
}

template <typename T>
hipError_t Plain<T>::cols_any(const LineFft<T>& f, cx<T>* a, int lx, int dir, hipStream_t s, cx<T>* tr) {
  const bool mixed = f.mp.np > 0;
  if (!mixed && f.M == 0) return cols(f.L, a, lx, dir, f.tw, s);
  if (!tr)
    return mixed ? Mixed<T>::lines(f.L, f.mp, f.tw, a, lx, 1, lx, dir, s) : Bluestein<T>::cols(f, a, lx, dir, s);
  // strided columns gather poorly: transpose, transform rows, transpose back
  hipError_t e;
  if ((e = Bluestein<T>::transpose(a, tr, f.L, lx, s)) != hipSuccess) return e;
  if ((e = mixed ? Mixed<T>::lines(f.L, f.mp, f.tw, tr, lx, f.L, 1, dir, s) : Bluestein<T>::rows(f, tr, lx, dir, s)) !=
      hipSuccess)
    return e;
  return Bluestein<T>::transpose(tr, a, lx, f.L, s);
}

template <typename T>
hipError_t Plain<T>::lens_grad(const cx<T>* g, const cx<T>* u, double* partial, int ny, int nx,
                               const ElementParams<T>& el, double f, int* nblocks, hipStream_t s) {
  const int64_t n = (int64_t)ny * nx;
  *nblocks = grid_for(n) > 1024 ? 1024 : grid_for(n);
  hipLaunchKernelGGL((plain_lens_grad_kernel<T>), dim3(*nblocks), dim3(256), 0, s, g, u, partial, ny, nx, el, f);
  return hipGetLastError();
}

template <typename T>
hipError_t Plain<T>::intensity(const cx<T>* u, T* I, int64_t n, T scale, hipStream_t s) {
  hipLaunchKernelGGL((plain_intensity_kernel<T>), dim3(grid_for(n)), dim3(256), 0, s, u, I, n, scale);
  return hipGetLastError();
}

template <typename T>
hipError_t Plain<T>::loss(const cx<T>* u, const T* ref, cx<T>* grad, double* partial, int64_t n, int kind,
                          T scale, int* nblocks, hipStream_t s) {
  *nblocks = grid_for(n) > 1024 ? 1024 : grid_for(n);
  hipLaunchKernelGGL((plain_loss_kernel<T>), dim3(*nblocks), dim3(256), 0, s, u, ref, grad, partial, n, kind,
                     scale);
  return hipGetLastError();
}

template <typename T>
hipError_t Plain<T>::modulate(const cx<T>* in, cx<T>* out, int ny, int nx, const ElementParams<T>& el, int conj,
                              hipStream_t s) {
  hipLaunchKernelGGL((plain_modulate_kernel<T>), dim3(grid_for((int64_t)ny * nx)), dim3(256), 0, s, in, out,
                     ny, nx, el, conj);
  return hipGetLastError();
}

template <typename T>
hipError_t Plain<T>::phase_grad(const cx<T>* g, const cx<T>* u, T* gphi, int ny, int nx,
                                const ElementParams<T>& el, hipStream_t s) {
  hipLaunchKernelGGL((plain_phase_grad_kernel<T>), dim3(grid_for((int64_t)ny * nx)), dim3(256), 0, s, g, u,
                     gphi, ny, nx, el);
  return hipGetLastError();
}

template struct Plain<float>;
template struct Plain<double>;

}  // namespace toprop
