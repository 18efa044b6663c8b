// Bluestein's chirp-z transform: for a length L that is not a power of two,
//   X[k] = sum_n x[n] exp(-2 pi i n k / L)
//        = conj(w[k]) sum_n (x[n] conj(w[n])) w[k - n],   w[m] = exp(i pi m^2 / L),
// since 2 n k = n^2 + k^2 - (k - n)^2.  The sum is a linear convolution,
// computed as a circular one of length M >= 2L - 1 (a power of two) with
// the library's own Stockham transforms: one forward FFT, a multiplication
// by Bf = DFT_M(b) (b[m] = w[m] for |m| < L, wrapped), one inverse FFT.  The
// inverse DFT is conj(DFT(conj(x))).  Chirp phases are reduced exactly in
// integers (m^2 mod 2L) and evaluated in FP64.  One workgroup transforms a
// whole line (rows) or a tile of columns, in registers and LDS.
#include <hip/hip_runtime.h>

#include "bluestein.hpp"
#include "launch.hpp"
#include "plain.hpp"

namespace toprop {

template <typename T>
__global__ void __launch_bounds__(256) bluestein_chirp_kernel(cx<T>* w, cx<T>* b, int L, int M) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  auto chirp = [&](int m) {
    const long long q = ((long long)m * m) % (2LL * L);
    double s, c;
    sincospi((double)q / (double)L, &s, &c);
    return cx<T>{(T)c, (T)s};
  };
  if (i < L) w[i] = chirp(i);
  const int m = i < L ? i : (i > M - L ? M - i : -1);
  b[i] = m >= 0 ? chirp(m) : cx<T>{T(0), T(0)};
}

// One line through the chirp-z pipeline.  v holds positions j + m TT.
template <typename T, int M, int R, int STRIDE>
__device__ __forceinline__ void bluestein_line(cx<T>* v, int j, int L, int dir, const cx<T>* __restrict__ w,
                                               const cx<T>* __restrict__ Bf, cx<T>* lds,
                                               const cx<T>* __restrict__ tw) {
  constexpr int TT = M / R;
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const int p = j + m * TT;
    cx<T> x = v[m];
    if (dir > 0) x.y = -x.y;
    v[m] = p < L ? cmulc(x, w[p]) : cx<T>{T(0), T(0)};
  }
  fft_wg<T, M, R, -1, false, STRIDE>(v, j, lds, tw);
#pragma unroll
  for (int m = 0; m < R; ++m) v[m] = cmul(v[m], Bf[j + m * TT]);
  fft_wg<T, M, R, +1, false, STRIDE>(v, j, lds, tw);
  const T sc = T(1) / T(M);
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const int p = j + m * TT;
    cx<T> y = p < L ? cscale(cmulc(v[m], w[p]), sc) : cx<T>{T(0), T(0)};
    if (dir > 0) y.y = -y.y;
    v[m] = y;
  }
}

template <typename T, int M, int R, int G>
__global__ void __launch_bounds__(G * (M / R)) bluestein_rows_kernel(cx<T>* a, int rows, int L, int dir,
                                                                     const cx<T>* w, const cx<T>* Bf,
                                                                     const cx<T>* tw) {
  constexpr int TT = M / R;
  __shared__ cx<T> lds[G * lds_len<1>(M)];
  const int g = threadIdx.x / TT, j = threadIdx.x % TT;
  const int row = blockIdx.x * G + g;
  const bool ok = row < rows;
  cx<T>* p = a + (int64_t)(ok ? row : 0) * L;
  cx<T> v[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const int q = j + m * TT;
    v[m] = (ok && q < L) ? p[q] : cx<T>{T(0), T(0)};
  }
  bluestein_line<T, M, R, 1>(v, j, L, dir, w, Bf, lds + g * lds_len<1>(M), tw);
  if (ok) {
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int q = j + m * TT;
      if (q < L) p[q] = v[m];
    }
  }
}

template <typename T, int M, int R, int TC>
__global__ void __launch_bounds__(TC * (M / R)) bluestein_cols_kernel(cx<T>* a, int L, int lx, int dir,
                                                                      const cx<T>* w, const cx<T>* Bf,
                                                                      const cx<T>* tw) {
  constexpr int TT = M / R;
  __shared__ cx<T> lds[lds_len<TC>(M) * TC];
  const int c = threadIdx.x % TC, j = threadIdx.x / TC;
  const int col = blockIdx.x * TC + c;
  const bool ok = col < lx;
  cx<T> v[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const int q = j + m * TT;
    v[m] = (ok && q < L) ? a[(int64_t)q * lx + col] : cx<T>{T(0), T(0)};
  }
  bluestein_line<T, M, R, TC>(v, j, L, dir, w, Bf, lds + c, tw);
  if (ok) {
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int q = j + m * TT;
      if (q < L) a[(int64_t)q * lx + col] = v[m];
    }
  }
}

// 32 x 32 tiles through LDS (one padding column: conflict-free columns).
template <typename T>
__global__ void __launch_bounds__(256) bluestein_transpose_kernel(const cx<T>* __restrict__ in,
                                                                  cx<T>* __restrict__ out, int rows, int cols) {
  __shared__ cx<T> tile[32][33];
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
#pragma unroll
  for (int k = 0; k < 32; k += 8) {
    const int r = r0 + ty + k, c = c0 + tx;
    if (r < rows && c < cols) tile[ty + k][tx] = in[(int64_t)r * cols + c];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 32; k += 8) {
    const int c = c0 + ty + k, r = r0 + tx;
    if (r < rows && c < cols) out[(int64_t)c * rows + r] = tile[tx][ty + k];
  }
}

namespace {
template <typename F>
hipError_t dispatch_pow2(int M, F&& f) {
  switch (M) {
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
}  // namespace

template <typename T>
hipError_t Bluestein<T>::build(int L, int M, cx<T>* w, cx<T>* Bf, const cx<T>* twM, hipStream_t s) {
  hipLaunchKernelGGL((bluestein_chirp_kernel<T>), dim3((M + 255) / 256), dim3(256), 0, s, w, Bf, L, M);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return Plain<T>::rows(M, Bf, 1, -1, twM, s);
}

template <typename T>
hipError_t Bluestein<T>::rows(const LineFft<T>& f, cx<T>* a, int nrows, int dir, hipStream_t s) {
  return dispatch_pow2(f.M, [&](auto Mc) -> hipError_t {
    constexpr int MM = decltype(Mc)::value;
    using C = RowCfg<T, MM>;
    hipLaunchKernelGGL((bluestein_rows_kernel<T, MM, C::R, C::G>), dim3((nrows + C::G - 1) / C::G),
                       dim3(C::threads), 0, s, a, nrows, f.L, dir, f.w, f.Bf, f.tw);
    return hipGetLastError();
  });
}

template <typename T>
hipError_t Bluestein<T>::cols(const LineFft<T>& f, cx<T>* a, int lx, int dir, hipStream_t s) {
  return dispatch_pow2(f.M, [&](auto Mc) -> hipError_t {
    constexpr int MM = decltype(Mc)::value;
    using C = ColCfg<T, MM, 1>;
    hipLaunchKernelGGL((bluestein_cols_kernel<T, MM, C::R, C::TC>), dim3((lx + C::TC - 1) / C::TC),
                       dim3(C::threads), 0, s, a, f.L, lx, dir, f.w, f.Bf, f.tw);
    return hipGetLastError();
  });
}

template <typename T>
hipError_t Bluestein<T>::transpose(const cx<T>* in, cx<T>* out, int rows, int cols, hipStream_t s) {
  hipLaunchKernelGGL((bluestein_transpose_kernel<T>), dim3((cols + 31) / 32, (rows + 31) / 32), dim3(256), 0, s, in,
                     out, rows, cols);
  return hipGetLastError();
}

template struct Bluestein<float>;
template struct Bluestein<double>;

}  // namespace toprop
