// Transfer-function tables.
//
// Direct integration (TorchOptics paper, section "Computational Fourier
// optics", Eq. (field_propagation) with the impulse response of
// Eq. (impulse_response)): the propagated field at a sample is the Riemann
// sum over the field's samples of h(x - x', y - y') u(x', y') dx dy, a
// linear convolution.  On the zero-padded grid (py >= 2 ny - 1,
// px >= 2 nx - 1) it is the circular convolution with the response sampled
// at the signed circular offsets, so the propagation pipeline applies it as
// a transfer function: the forward DFT of that sampled response.  The
// sampling kernel evaluates h in FP64; the DFT is the library's own
// row and column FFT passes in the table's precision.
#include <hip/hip_runtime.h>

#include "plain.hpp"
#include "transfer.hpp"

namespace toprop {

// h(oy, ox) dx dy at every entry of the padded grid; entry (ky, kx) holds the
// signed offset (sy dy, sx dx), sy = ky for ky < py/2 and ky - py otherwise.
// Offsets that no pair of field samples has (|sy| >= ny or |sx| >= nx) are 0.
//   h = z / (i lambda d) (1 + i / (k d)) exp(i k d) / d
//     = A (1 / (k d) - i) exp(2 pi i d / lambda),  A = z / (lambda d^2),
// with d / lambda = z/lambda + (z/lambda) s / (1 + sqrt(1 + s)),
// s = (oy^2 + ox^2) / z^2: the large integer part of z/lambda is replaced by
// its exact fractional part, so the FP64 phase keeps its fractional digits.
template <typename T>
__global__ void __launch_bounds__(256) di_sample_kernel(cx<T>* H, DiParams p) {
  const int64_t n = (int64_t)p.py * p.px;
  const double q = p.z / p.lam;
  const double area = p.dy * p.dx;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int ky = (int)(i / p.px), kx = (int)(i - (int64_t)ky * p.px);
    const int sy = 2 * ky < p.py ? ky : ky - p.py;
    const int sx = 2 * kx < p.px ? kx : kx - p.px;
    if (abs(sy) >= p.ny || abs(sx) >= p.nx) {
      H[i] = {T(0), T(0)};
      continue;
    }
    const double oy = (double)sy * p.dy, ox = (double)sx * p.dx;
    const double s = (oy * oy + ox * ox) / (p.z * p.z);
    const double root = sqrt(1.0 + s);
    const double d = p.z * root;
    const double cyc = p.q_frac + q * s / (1.0 + root);
    const cx<T> e = cis_cycles<T>(cyc);
    const double amp = area * p.z / (p.lam * d * d);
    const double kd = 6.283185307179586476925286766559 * d / p.lam;
    const cx<T> f = {(T)(amp / kd), (T)(-amp)};
    H[i] = cmul(f, e);
  }
}

namespace {
int table_grid(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (int)(b > 16384 ? 16384 : (b < 1 ? 1 : b));
}
}  // namespace

template <typename T>
hipError_t TransferTable<T>::direct_integration(cx<T>* H, const DiParams& p, const LineFft<T>& fx,
                                                const LineFft<T>& fy, hipStream_t s, cx<T>* tr) {
  hipLaunchKernelGGL((di_sample_kernel<T>), dim3(table_grid((int64_t)p.py * p.px)), dim3(256), 0, s, H, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = Plain<T>::rows_any(fx, H, p.py, -1, s)) != hipSuccess) return e;
  return Plain<T>::cols_any(fy, H, p.px, -1, s, tr);
}

template <typename T>
hipError_t TransferTable<T>::direct_integration_t(cx<T>* HT, cx<T>* tmp, const DiParams& p, const LineFft<T>& fx,
                                                  const LineFft<T>& fy, hipStream_t s) {
  hipLaunchKernelGGL((di_sample_kernel<T>), dim3(table_grid((int64_t)p.py * p.px)), dim3(256), 0, s, tmp, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = Plain<T>::rows_any(fx, tmp, p.py, -1, s)) != hipSuccess) return e;
  if ((e = Mixed<T>::transpose(tmp, HT, p.py, p.px, 1, s)) != hipSuccess) return e;
  return Plain<T>::rows_any(fy, HT, p.px, -1, s);
}

template <typename T>
hipError_t TransferTable<T>::analytic(cx<T>* H, int py, int px, const TransferParams& p, hipStream_t s) {
  return Plain<T>::table(H, py, px, p, s);
}

__global__ void __launch_bounds__(256) separable_tables_kernel(SepTableBatch b) {
  const SepTableDesc& d = b.d[blockIdx.y];
  cx<float>* ex = static_cast<cx<float>*>(d.base);
  cx<float>* ey = ex + d.lx;
  float* sx = reinterpret_cast<float*>(ey + d.ly);
  float* sy = sx + d.lx;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  tf_table_entry(i, ex, sx, d.lx, d.inv_lxdx, ey, sy, d.ly, d.inv_lydy, d.fres_a, d.q_frac, d.lam2);
}

hipError_t separable_tables(const SepTableBatch& b, hipStream_t s) {
  if (b.count <= 0) return hipSuccess;
  hipLaunchKernelGGL(separable_tables_kernel, dim3((b.maxlen + 255) / 256, b.count), dim3(256), 0, s, b);
  return hipGetLastError();
}

template struct TransferTable<float>;
template struct TransferTable<double>;

}  // namespace toprop
