// Kernels for propagating a mutual coherence function (TorchOptics paper,
// section "Spatial coherence"): Gamma is stored as an n x n matrix with
// n = ny nx (row index r1 = (y1, x1), column index r2 = (y2, x2)).  The 4-D
// propagation Gamma_z = P Gamma P^H is carried out by the batched field
// propagation of the fused kernels (P along r2 for every row, P along r1 for
// every row of the transpose) around the tiled transposes below; these
// kernels supply the transposes, the element table, the diagonal-intensity
// loss and the mask-gradient reductions.
#include <hip/hip_runtime.h>

#include "coherence.hpp"

namespace toprop {

// out[b][a] = s(a, b) * in[a][b] for an n x n complex matrix, through a
// 64 x 64 LDS tile (padded against bank conflicts).  With `m` set,
// s(a, b) = conj(m[a]) m[b] (the element adjoint M^H G M of the adjoint
// propagation, applied to the un-transposed indices).
template <typename T>
__global__ void __launch_bounds__(256) coh_transpose_kernel(const cx<T>* __restrict__ in, cx<T>* __restrict__ out,
                                                            int n, const cx<T>* __restrict__ m) {
  __shared__ cx<T> tile[64][65];
  const int bx = blockIdx.x * 64, by = blockIdx.y * 64;  // source column / row block
  const int tx = threadIdx.x % 64, ty = threadIdx.x / 64;  // 64 x 4 threads
  for (int k = ty; k < 64; k += 4) {
    const int a = by + k, b = bx + tx;
    cx<T> v = {T(0), T(0)};
    if (a < n && b < n) {
      v = in[(int64_t)a * n + b];
      if (m) v = cmul(cmulc(m[b], m[a]), v);  // m[b] conj(m[a])
    }
    tile[k][tx] = v;
  }
  __syncthreads();
  for (int k = ty; k < 64; k += 4) {
    const int b = bx + k, a = by + tx;
    if (a < n && b < n) out[(int64_t)b * n + a] = tile[tx][k];
  }
}

// m[r] = M(r) (or conj(M(r))), the scalar modulation of the job's element at
// every pixel.
template <typename T>
__global__ void __launch_bounds__(256) coh_mtable_kernel(cx<T>* m, int ny, int nx, ElementParams<T> el,
                                                         int conj) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < ny * nx) {
    cx<T> v = scalar_modulation(el, ny, nx, r / nx, r % nx);
    if (conj) v.y = -v.y;
    m[r] = v;
  }
}

// g[a][b] *= conj(m[a]) m[b] in place (the element adjoint M^H G M).
template <typename T>
__global__ void __launch_bounds__(256) coh_scale_kernel(cx<T>* g, const cx<T>* m, int n) {
  const int64_t total = (int64_t)n * n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(i / n), b = (int)(i % n);
    g[i] = cmul(cmulc(m[b], m[a]), g[i]);
  }
}

// Diagonal-intensity loss of Gamma_out: I(r) = Re Gamma(r, r);
// MSE: loss += scale sum (I - T)^2, grad = 2 scale (I - T) on the diagonal;
// WEIGHTED: loss += scale sum W I, grad = scale W on the diagonal.  Off the
// diagonal the gradient is zero (written by the caller's memset-free clear:
// this kernel writes whole rows).
template <typename T>
__global__ void __launch_bounds__(256) coh_diag_loss_kernel(const cx<T>* __restrict__ g, const T* __restrict__ ref,
                                                            cx<T>* __restrict__ grad, double* partial, int n,
                                                            int kind, T scale) {
  // one block per row r of the gradient matrix
  __shared__ double red[256];
  const int r = blockIdx.x;
  // every thread forms the diagonal gradient (the one with b == r stores
  // it); thread 0 alone contributes the loss term
  double acc = 0.0;
  cx<T> dg;
  const T I = g[(int64_t)r * n + r].x;
  if (kind == EPI_MSE) {
    const T d = I - ref[r];
    if (threadIdx.x == 0) acc = (double)d * (double)d;
    dg = {T(2) * scale * d, T(0)};
  } else {
    if (threadIdx.x == 0) acc = (double)ref[r] * (double)I;
    dg = {scale * ref[r], T(0)};
  }
  for (int b = threadIdx.x; b < n; b += blockDim.x)
    grad[(int64_t)r * n + b] = (b == r) ? dg : cx<T>{T(0), T(0)};
  const double s = block_sum<256>(acc, red);
  if (threadIdx.x == 0) partial[r] = s;
}

// out[r] += scale * Re Gamma(r, r): the time-averaged intensity.
template <typename T>
__global__ void __launch_bounds__(256) coh_diag_intensity_kernel(const cx<T>* __restrict__ g, T* __restrict__ out,
                                                                 int n, T scale) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) out[r] += scale * g[(int64_t)r * n + r].x;
}

// t(a, b) = Im(G(a, b) conj(Gm(a, b))), Gm = m[a] conj(m[b]) Gamma(a, b).
template <typename T>
__device__ __forceinline__ double coh_grad_term(const cx<T>* G, const cx<T>* Gam, const cx<T>* m, int n, int a,
                                                int b) {
  const int64_t i = (int64_t)a * n + b;
  const cx<T> gm = cmul(cmulc(m[a], m[b]), Gam[i]);
  const cx<T> g = G[i];
  return (double)g.y * (double)gm.x - (double)g.x * (double)gm.y;
}

// Row sums: rowsum[a] = sum_b t(a, b), one block per row, fixed order.
template <typename T>
__global__ void __launch_bounds__(256) coh_rowsum_kernel(const cx<T>* G, const cx<T>* Gam, const cx<T>* m,
                                                         double* rowsum, int n) {
  __shared__ double red[256];
  const int a = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < n; b += 256) acc += coh_grad_term(G, Gam, m, n, a, b);
  const double s = block_sum<256>(acc, red);
  if (threadIdx.x == 0) rowsum[a] = s;
}

// Column sums in kCohRowChunks row chunks: colpart[c][b] = sum over the rows
// a of chunk c of t(a, b); a block covers 64 columns of one chunk with 4 row
// groups, fixed order (enough blocks to fill the GPU: columns x chunks).
template <typename T>
__global__ void __launch_bounds__(256) coh_colsum_kernel(const cx<T>* G, const cx<T>* Gam, const cx<T>* m,
                                                         double* colpart, int n) {
  __shared__ double red[4][64];
  const int tx = threadIdx.x % 64, ty = threadIdx.x / 64;
  const int b = blockIdx.x * 64 + tx;
  const int rows = (n + kCohRowChunks - 1) / kCohRowChunks;
  const int a0 = blockIdx.y * rows, a1 = min(a0 + rows, n);
  double acc = 0.0;
  if (b < n)
    for (int a = a0 + ty; a < a1; a += 4) acc += coh_grad_term(G, Gam, m, n, a, b);
  red[ty][tx] = acc;
  __syncthreads();
  if (ty == 0 && b < n)
    colpart[(int64_t)blockIdx.y * n + b] = ((red[0][tx] + red[1][tx]) + red[2][tx]) + red[3][tx];
}

// grad_phase[r] += rowsum[r] - sum over chunks (in order) of colpart[c][r].
template <typename T>
__global__ void __launch_bounds__(256) coh_grad_combine_kernel(const double* rowsum, const double* colpart, T* gphi,
                                                               int n) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double col = 0.0;
  for (int c = 0; c < kCohRowChunks; ++c) col += colpart[(int64_t)c * n + r];
  gphi[r] += (T)(rowsum[r] - col);
}

template <typename T>
hipError_t Coh<T>::transpose(const cx<T>* in, cx<T>* out, int n, const cx<T>* m, hipStream_t s) {
  dim3 grid((n + 63) / 64, (n + 63) / 64);
  hipLaunchKernelGGL((coh_transpose_kernel<T>), grid, dim3(256), 0, s, in, out, n, m);
  return hipGetLastError();
}

template <typename T>
hipError_t Coh<T>::mtable(cx<T>* m, int ny, int nx, const ElementParams<T>& el, int conj, hipStream_t s) {
  const int n = ny * nx;
  hipLaunchKernelGGL((coh_mtable_kernel<T>), dim3((n + 255) / 256), dim3(256), 0, s, m, ny, nx, el, conj);
  return hipGetLastError();
}

template <typename T>
hipError_t Coh<T>::scale(cx<T>* g, const cx<T>* m, int n, hipStream_t s) {
  const int64_t total = (int64_t)n * n;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL((coh_scale_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, s, g, m, n);
  return hipGetLastError();
}

template <typename T>
hipError_t Coh<T>::diag_loss(const cx<T>* g, const T* ref, cx<T>* grad, double* partial, int n, int kind, T scale,
                             hipStream_t s) {
  hipLaunchKernelGGL((coh_diag_loss_kernel<T>), dim3(n), dim3(256), 0, s, g, ref, grad, partial, n, kind, scale);
  return hipGetLastError();
}

template <typename T>
hipError_t Coh<T>::diag_intensity(const cx<T>* g, T* out, int n, T scale, hipStream_t s) {
  hipLaunchKernelGGL((coh_diag_intensity_kernel<T>), dim3((n + 255) / 256), dim3(256), 0, s, g, out, n, scale);
  return hipGetLastError();
}

template <typename T>
hipError_t Coh<T>::phase_grad(const cx<T>* G, const cx<T>* Gam, const cx<T>* m, double* rowsum, double* colsum,
                              T* gphi, int n, hipStream_t s) {
  hipLaunchKernelGGL((coh_rowsum_kernel<T>), dim3(n), dim3(256), 0, s, G, Gam, m, rowsum, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((coh_colsum_kernel<T>), dim3((n + 63) / 64, kCohRowChunks), dim3(256), 0, s, G, Gam, m, colsum,
                     n);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL((coh_grad_combine_kernel<T>), dim3((n + 255) / 256), dim3(256), 0, s, rowsum, colsum, gphi,
                     n);
  return hipGetLastError();
}

template struct Coh<float>;
template struct Coh<double>;

}  // namespace toprop
