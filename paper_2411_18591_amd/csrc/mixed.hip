// Mixed-radix Stockham FFT of lines of length L = 2^a 3^b 5^c 7^d.
//
// Pass p (radix R, NS = product of the radices before it) takes butterfly b
// (b < L/R) from positions b + r L/R, r < R, multiplies input r by
// w_{NS R}^{r (b mod NS)} (w_N = exp(D 2 pi i / N)), applies the R-point
// DFT and stores output r at (b - b mod NS) R + b mod NS + r NS.  After the
// last pass (NS R = L) the line holds its DFT in natural order (Stockham's
// self-sorting form: no index reversal).  The first pass reads the line
// from global memory, the last writes it back; in between the line lives in
// LDS (one padding element every 32, which keeps the strided stores of the
// first passes off shared banks).  A workgroup of 256 threads holds
// 256 / TL lines, TL = threads per line, the least power of two with
// L <= 16 TL, so each thread owns at most 16 points of a pass.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mixed.hpp"

namespace toprop {

bool mixed_plan(int L, MixedPlan* p, bool pow2) {
  p->np = 0;
  if (L < 2 || L > 4096 || (!pow2 && (L & (L - 1)) == 0)) return false;
  int a = L, e2 = 0;
  while (a % 2 == 0) a /= 2, ++e2;
  int r[kMixedMaxPasses], n = 0;
  for (; e2 >= 4; e2 -= 4) r[n++] = 16;
  if (e2 == 1 && n > 0)
    r[n - 1] = 8, r[n++] = 4;  // 16 * 2 as 8 * 4
  else if (e2 > 0)
    r[n++] = 1 << e2;
  for (int q : {5, 3, 7})
    while (a % q == 0) a /= q, r[n++] = q;
  if (a != 1) return false;
  p->np = n;
  for (int i = 0; i < n; ++i) p->r[i] = r[i];
  return true;
}

namespace {

constexpr int kLinePoints = 16;                         // points per thread and pass
constexpr int kMixedLds = 4096 + 4096 / 32;             // padded elements of one workgroup
__device__ __forceinline__ int pidx(int i) { return i + (i >> 5); }

// cos and sin of 2 pi m / R, 1 <= m <= (R - 1) / 2, for the odd radices.
constexpr double odd_cos(int R, int m) {
  return R == 3   ? -0.5
         : R == 5 ? (m == 1 ? 0.3090169943749474241022 : -0.8090169943749474241022)
                  : (m == 1 ? 0.6234898018587335305250 : m == 2 ? -0.2225209339563144042889 : -0.9009688679024191262361);
}
constexpr double odd_sin(int R, int m) {
  return R == 3   ? 0.8660254037844386467637
         : R == 5 ? (m == 1 ? 0.9510565162951535721164 : 0.5877852522924731291687)
                  : (m == 1 ? 0.7818314824680298087084 : m == 2 ? 0.9749279121818236070181 : 0.4338837391175581204757);
}

// R-point DFT (R odd) from the symmetric sums a_n = x_n + x_{R-n} and
// differences b_n = x_n - x_{R-n}:
//   X_k     = x_0 + sum_n a_n cos(2 pi n k / R) + D i sum_n b_n sin(2 pi n k / R)
//   X_{R-k} = x_0 + sum_n a_n cos(2 pi n k / R) - D i sum_n b_n sin(2 pi n k / R).
template <int R, int D, typename T>
__device__ __forceinline__ void odd_dft(cx<T>* v) {
  constexpr int H = (R - 1) / 2;
  cx<T> a[H], b[H];
  const cx<T> x0 = v[0];
  cx<T> s0 = x0;
#pragma unroll
  for (int n = 1; n <= H; ++n) {
    a[n - 1] = cadd(v[n], v[R - n]);
    b[n - 1] = csub(v[n], v[R - n]);
    s0 = cadd(s0, a[n - 1]);
  }
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    cx<T> re = x0, im{T(0), T(0)};
#pragma unroll
    for (int n = 1; n <= H; ++n) {
      const int m = (n * k) % R;
      const T c = (T)odd_cos(R, m <= H ? m : R - m);
      const T s = (T)(m <= H ? odd_sin(R, m) : -odd_sin(R, R - m));
      re = {re.x + a[n - 1].x * c, re.y + a[n - 1].y * c};
      im = {im.x + b[n - 1].x * s, im.y + b[n - 1].y * s};
    }
    const cx<T> t = D > 0 ? cx<T>{-im.y, im.x} : cx<T>{im.y, -im.x};  // D i im
    v[k] = cadd(re, t);
    v[R - k] = csub(re, t);
  }
  v[0] = s0;
}

template <int R, int D, typename T>
__device__ __forceinline__ void small_dft(cx<T>* v) {
  if constexpr ((R & (R - 1)) == 0)
    Dft<R, D, T>::run(v);
  else
    odd_dft<R, D, T>(v);
}

// One pass of radix R over the line owned by threads j < TL (see the file
// comment).  IN_G: the pass reads the line from global memory (element q <
// a.nin at in[q * in_es], zeros beyond), else from the LDS line `ll`.
// OUT_G: it writes elements q < a.nout, times a.scale, to out[q * out_es],
// else the whole line to `ll`.  MULH (a last forward pass, natural order):
// output q is multiplied by h[q] (conjugated if a.conj) before it is stored,
// or with HC by transfer_at(hline, q, h_lines, L, a.tp), formed in place.
template <typename T>
struct LineIo {
  const cx<T>* in;
  cx<T>* out;
  const cx<T>* h;
  int in_es, out_es;  // q * es < 2^31: checked on the host
  int line;           // row of the field (element modulation)
  int hline;          // row of the transfer table (line mod h_lines)
};

// b mod ns for b, ns <= 4096 from a float reciprocal of ns (uniform), with
// one correction step: the quotient estimate is off by at most one.
__device__ __forceinline__ int mod_small(int b, int ns, float inv_ns) {
  int k = b - (int)((float)b * inv_ns) * ns;
  k = k < 0 ? k + ns : k;
  return k >= ns ? k - ns : k;
}

template <typename T, int R, int D, bool IN_G, bool OUT_G, bool MULH, bool EL, bool HC = false>
__device__ __forceinline__ void mixed_pass(cx<T>* ll, const LineIo<T>& io, const MixedArgs<T>& a, bool ok, int NS,
                                           int j, int TL) {
  constexpr int NB = (kLinePoints + R - 1) / R;  // butterflies per thread
  const int L = a.L;
  const int nb = L / R;
  const int step = L / (NS * R);
  const float inv_ns = 1.0f / (float)NS;
  cx<T> v[NB][R];
  int kk[NB];
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    const int b = j + t * TL;
    const bool act = b < nb;
    kk[t] = NS > 1 ? mod_small(b, NS, inv_ns) : 0;
    // Loads are unconditional (from a valid address) so that no branch
    // surrounds them: a butterfly past nb is computed on whatever it read
    // and never stored; padding (q >= nin) and absent lines select zero.
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int q = act ? b + r * nb : 0;
      if constexpr (IN_G) {
        const bool valid = ok && q < a.nin;
        cx<T> x = io.in[(valid ? q : 0) * io.in_es];
        if constexpr (EL) x = cmul(scalar_modulation(a.el, a.field_rows, a.nin, io.line, valid ? q : 0), x);
        v[t][r] = valid ? x : cx<T>{T(0), T(0)};
      } else {
        v[t][r] = ll[pidx(q)];
      }
    }
    if (NS > 1) {
      // w^r for r < R from w = exp(D 2 pi i k / (NS R)): one table load, the
      // rest by products (squares for even r)
      cx<T> w[R];
      w[1] = a.tw[kk[t] * step];  // k step < L
      if (D > 0) w[1].y = -w[1].y;
#pragma unroll
      for (int r = 2; r < R; ++r) w[r] = (r % 2 == 0) ? cmul(w[r / 2], w[r / 2]) : cmul(w[r - 1], w[1]);
#pragma unroll
      for (int r = 1; r < R; ++r) v[t][r] = cmul(v[t][r], w[r]);
    }
    small_dft<R, D, T>(v[t]);
  }
  if constexpr (!IN_G && !OUT_G) __syncthreads();  // every read of this pass is done
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    const int b = j + t * TL;
    if (b >= nb) continue;
    const int k = kk[t];
    const int base = (b - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int q = base + r * NS;
      cx<T> y = v[t][r];
      if constexpr (MULH && HC) {
        y = cmul(y, transfer_at<T>(io.hline, q, a.h_lines, L, a.tp));
      } else if constexpr (MULH) {
        cx<T> h = io.h[q];
        if (a.conj) h.y = -h.y;
        y = cmul(y, h);
      }
      if constexpr (OUT_G) {
        if (ok && q < a.nout) io.out[q * io.out_es] = cscale(y, a.scale);
      } else {
        ll[pidx(q)] = y;
      }
    }
  }
  if constexpr (!OUT_G) __syncthreads();
}

template <typename T, int D, bool IN_G, bool OUT_G, bool MULH, bool EL = false, bool HC = false>
__device__ __forceinline__ void mixed_pass_r(int R, cx<T>* ll, const LineIo<T>& io, const MixedArgs<T>& a, bool ok,
                                             int NS, int j, int TL) {
  switch (R) {
    case 2: mixed_pass<T, 2, D, IN_G, OUT_G, MULH, EL, HC>(ll, io, a, ok, NS, j, TL); break;
    case 3: mixed_pass<T, 3, D, IN_G, OUT_G, MULH, EL, HC>(ll, io, a, ok, NS, j, TL); break;
    case 4: mixed_pass<T, 4, D, IN_G, OUT_G, MULH, EL, HC>(ll, io, a, ok, NS, j, TL); break;
    case 5: mixed_pass<T, 5, D, IN_G, OUT_G, MULH, EL, HC>(ll, io, a, ok, NS, j, TL); break;
    case 7: mixed_pass<T, 7, D, IN_G, OUT_G, MULH, EL, HC>(ll, io, a, ok, NS, j, TL); break;
    case 8: mixed_pass<T, 8, D, IN_G, OUT_G, MULH, EL, HC>(ll, io, a, ok, NS, j, TL); break;
    default: mixed_pass<T, 16, D, IN_G, OUT_G, MULH, EL, HC>(ll, io, a, ok, NS, j, TL); break;
  }
}

// The passes of one transform: the first reads global memory (IN_G), the
// last writes it (OUT_G) and/or multiplies by h (MULH).
template <typename T, int D, bool IN_G, bool OUT_G, bool MULH, bool EL = false, bool HC = false>
__device__ __forceinline__ void mixed_transform(cx<T>* ll, const LineIo<T>& io, const MixedArgs<T>& a, bool ok,
                                                int j, int TL) {
  const MixedPlan& p = a.plan;
  if (p.np == 1) {
    mixed_pass_r<T, D, IN_G, OUT_G, MULH, EL, HC>(p.r[0], ll, io, a, ok, 1, j, TL);
    return;
  }
  mixed_pass_r<T, D, IN_G, false, false, EL>(p.r[0], ll, io, a, ok, 1, j, TL);
  int ns = p.r[0];
  for (int i = 1; i < p.np - 1; ++i) {
    mixed_pass_r<T, D, false, false, false>(p.r[i], ll, io, a, ok, ns, j, TL);
    ns *= p.r[i];
  }
  mixed_pass_r<T, D, false, OUT_G, MULH, false, HC>(p.r[p.np - 1], ll, io, a, ok, ns, j, TL);
}

// MODE -1 / +1: one forward / inverse transform per line; MODE 0: forward
// transform, multiplication by the line's h (HC: the transfer function
// formed in place), inverse transform.  EL: the forward transform applies
// a.el to what it reads.
template <typename T, int MODE, bool EL, bool HC = false>
__global__ void __launch_bounds__(256) mixed_lines_kernel(MixedArgs<T> a) {
  __shared__ cx<T> lds[kMixedLds];
  const int TL = 1 << a.tl_shift, G = 256 >> a.tl_shift;
  const int g = threadIdx.x >> a.tl_shift, j = threadIdx.x & (TL - 1);
  const int line = blockIdx.x * G + g;
  const bool ok = line < a.nlines;
  const int64_t li = ok ? line : 0;
  const LineIo<T> io{a.in + li * a.in_ls, a.out + li * a.out_ls, a.h ? a.h + (li % a.h_lines) * a.h_ls : nullptr,
                     (int)a.in_es, (int)a.out_es, (int)(li % a.field_rows), (int)(li % a.h_lines)};
  cx<T>* ll = lds + g * (pidx(a.L - 1) + 1);
  if constexpr (MODE == 0) {
    mixed_transform<T, -1, true, false, true, false, HC>(ll, io, a, ok, j, TL);
    mixed_transform<T, +1, false, true, false>(ll, io, a, ok, j, TL);
  } else {
    mixed_transform<T, MODE, true, true, false, EL>(ll, io, a, ok, j, TL);
  }
}

// ---------------------------------------------------------------------------
// Lengths fixed at compile time (the paper's grids 1000, 250, 50 and their
// 2x padding 2000, 500, 100): the plan, strides and divisors are constants, every LDS and
// global offset of a pass is an immediate from one per-butterfly base, and
// the line needs no LDS padding: the first pass, whose natural stores
// (position b R1 + r) would stride across the banks, stores output r of
// butterfly b at r L/R1 + b instead, and the second pass reads position p
// from (p mod R1) L/R1 + p / R1.  Global element strides are 1.
// ---------------------------------------------------------------------------
struct CPlan {
  int np;
  int r[kMixedMaxPasses];
};
constexpr CPlan cplan(int L) {
  CPlan p{};
  int a = L, e2 = 0;
  while (a % 2 == 0) a /= 2, ++e2;
  for (; e2 >= 4; e2 -= 4) p.r[p.np++] = 16;
  if (e2 == 1 && p.np > 0)
    p.r[p.np - 1] = 8, p.r[p.np++] = 4;
  else if (e2 > 0)
    p.r[p.np++] = 1 << e2;
  for (int q : {5, 3, 7})
    while (a % q == 0) a /= q, p.r[p.np++] = q;
  return p;
}
constexpr int threads_per_line(int L) {
  int t = 1;
  while (kLinePoints * t < L) t *= 2;
  return t;
}

template <typename T, int L, int R, int NS, int D, int R1, bool IN_G, bool OUT_G, bool MULH, bool IN_T, bool OUT_T,
          bool EL, bool HC>
__device__ __forceinline__ void fixed_pass(cx<T>* ll, const LineIo<T>& io, const MixedArgs<T>& a, bool ok, int j) {
  constexpr int TL = threads_per_line(L);
  constexpr int NB = (kLinePoints + R - 1) / R;
  constexpr int nb = L / R;
  constexpr int step = L / (NS * R);
  constexpr int nb1 = L / R1;
  cx<T> v[NB][R];
  int bb[NB], kk[NB];
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    const int b = j + t * TL;
    const int bs = (t * TL + TL <= nb || b < nb) ? b : 0;  // an absent butterfly reads butterfly 0
    bb[t] = b;
    kk[t] = bs % NS;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int q = bs + r * nb;
      if constexpr (IN_G) {
        const bool valid = ok && q < a.nin;
        cx<T> x = io.in[valid ? q : 0];
        if constexpr (EL) x = cmul(scalar_modulation(a.el, a.field_rows, a.nin, io.line, valid ? q : 0), x);
        v[t][r] = valid ? x : cx<T>{T(0), T(0)};
      } else if constexpr (IN_T) {
        v[t][r] = ll[(q % R1) * nb1 + q / R1];
      } else {
        v[t][r] = ll[q];
      }
    }
    if constexpr (NS > 1) {
      cx<T> w[R];
      w[1] = a.tw[kk[t] * step];
      if (D > 0) w[1].y = -w[1].y;
#pragma unroll
      for (int r = 2; r < R; ++r) w[r] = (r % 2 == 0) ? cmul(w[r / 2], w[r / 2]) : cmul(w[r - 1], w[1]);
#pragma unroll
      for (int r = 1; r < R; ++r) v[t][r] = cmul(v[t][r], w[r]);
    }
    small_dft<R, D, T>(v[t]);
  }
  if constexpr (!IN_G && !OUT_G) __syncthreads();
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    const int b = bb[t];
    if (t * TL + TL > nb && b >= nb) continue;
    const int k = kk[t];
    const int base = (b - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      cx<T> y = v[t][r];
      if constexpr (OUT_T) {
        ll[b + r * nb] = y;
      } else {
        const int q = base + r * NS;
        if constexpr (MULH && HC) {
          y = cmul(y, transfer_at<T>(io.hline, q, a.h_lines, L, a.tp));
        } else if constexpr (MULH) {
          cx<T> h = io.h[q];
          if (a.conj) h.y = -h.y;
          y = cmul(y, h);
        }
        if constexpr (OUT_G) {
          if (ok && q < a.nout) io.out[q] = cscale(y, a.scale);
        } else {
          ll[q] = y;
        }
      }
    }
  }
  if constexpr (!OUT_G) __syncthreads();
}

template <typename T, int L, int D, int P, int NS, bool IN_G, bool OUT_G, bool MULH, bool EL = false, bool HC = false>
__device__ __forceinline__ void fixed_passes(cx<T>* ll, const LineIo<T>& io, const MixedArgs<T>& a, bool ok,
                                             int j) {
  constexpr CPlan pl = cplan(L);
  constexpr int R = pl.r[P];
  constexpr bool first = P == 0, last = P == pl.np - 1;
  fixed_pass<T, L, R, NS, D, pl.r[0], first && IN_G, last && OUT_G, last && MULH, P == 1, first && !last,
             first && EL, HC>(ll, io, a, ok, j);
  if constexpr (!last) fixed_passes<T, L, D, P + 1, NS * R, IN_G, OUT_G, MULH, EL, HC>(ll, io, a, ok, j);
}

// The column launch of complex64 that reads a table holds 128 registers
// (four waves per SIMD; forming H in place needs a few more).
template <typename T, int L, int MODE, bool EL, bool HC = false>
__global__ void __launch_bounds__(256, (MODE == 0 && !HC && sizeof(T) == 4) ? 4 : 1)
    mixed_fixed_kernel(MixedArgs<T> a) {
  constexpr int TL = threads_per_line(L), G = 256 / TL;
  __shared__ cx<T> lds[G * L];
  const int g = threadIdx.x / TL, j = threadIdx.x % TL;
  const int line = blockIdx.x * G + g;
  const bool ok = line < a.nlines;
  const int64_t li = ok ? line : 0;
  const LineIo<T> io{a.in + li * a.in_ls, a.out + li * a.out_ls, a.h ? a.h + (li % a.h_lines) * a.h_ls : nullptr, 1,
                     1, (int)(li % a.field_rows), (int)(li % a.h_lines)};
  cx<T>* ll = lds + g * L;
  if constexpr (MODE == 0) {
    fixed_passes<T, L, -1, 0, 1, true, false, true, false, HC>(ll, io, a, ok, j);
    fixed_passes<T, L, +1, 0, 1, false, true, false>(ll, io, a, ok, j);
  } else {
    fixed_passes<T, L, MODE, 0, 1, true, true, false, EL>(ll, io, a, ok, j);
  }
}

template <typename T, int L>
hipError_t launch_fixed(const MixedArgs<T>& a, int mode, hipStream_t s) {
  constexpr int G = 256 / threads_per_line(L);
  const dim3 grid((a.nlines + G - 1) / G);
  if (mode < 0 && a.el.flags)
    hipLaunchKernelGGL((mixed_fixed_kernel<T, L, -1, true>), grid, dim3(256), 0, s, a);
  else if (mode < 0)
    hipLaunchKernelGGL((mixed_fixed_kernel<T, L, -1, false>), grid, dim3(256), 0, s, a);
  else if (mode > 0)
    hipLaunchKernelGGL((mixed_fixed_kernel<T, L, +1, false>), grid, dim3(256), 0, s, a);
  else if (a.hcalc)
    hipLaunchKernelGGL((mixed_fixed_kernel<T, L, 0, false, true>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((mixed_fixed_kernel<T, L, 0, false>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(256) mixed_twiddle_kernel(cx<T>* tw, int L) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= L) return;
  // exp(-2 pi i m / L) = exp(-i pi q / L) with q = 2m reduced to (-L, L]
  const int q = 2 * m > L ? 2 * m - 2 * L : 2 * m;
  double s, c;
  sincospi((double)q / (double)L, &s, &c);
  tw[m] = cx<T>{(T)c, (T)(-s)};
}

// 32 x 32 tiles through LDS (one padding column), blockIdx.z = array of
// the batch (offset by z0).
template <typename T>
__global__ void __launch_bounds__(256) mixed_transpose_kernel(const cx<T>* __restrict__ in, cx<T>* __restrict__ out,
                                                              int rows, int cols, int64_t z0) {
  __shared__ cx<T> tile[32][33];
  const int64_t off = (z0 + blockIdx.z) * (int64_t)rows * cols;
  in += off;
  out += off;
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

}  // namespace

template <typename T>
hipError_t Mixed<T>::twiddles(int L, cx<T>* tw, hipStream_t s) {
  hipLaunchKernelGGL((mixed_twiddle_kernel<T>), dim3((L + 255) / 256), dim3(256), 0, s, tw, L);
  return hipGetLastError();
}

template <typename T>
hipError_t Mixed<T>::launch(MixedArgs<T> a, int mode, hipStream_t s) {
  const MixedPlan& p = a.plan;
  if (p.np < 1 || p.np > kMixedMaxPasses || a.L < 2 || a.L > 4096) return hipErrorInvalidValue;
  int prod = 1;
  for (int i = 0; i < p.np; ++i) {
    const int r = p.r[i];
    if (r != 2 && r != 3 && r != 4 && r != 5 && r != 7 && r != 8 && r != 16) return hipErrorInvalidValue;
    prod *= r;
  }
  if (prod != a.L || a.nin < 0 || a.nin > a.L || a.nout < 0 || a.nout > a.L) return hipErrorInvalidValue;
  if (a.nin < 1 || a.nout < 1) return hipErrorInvalidValue;
  if (a.in_es < 1 || a.out_es < 1 || a.in_es * a.L >= (int64_t(1) << 31) || a.out_es * a.L >= (int64_t(1) << 31))
    return hipErrorInvalidValue;  // element offsets are 32-bit in the kernel
  if ((mode == 0 && !a.h && !a.hcalc) || (mode > 0 && a.el.flags)) return hipErrorInvalidValue;
  if (a.hcalc && (mode != 0 || (a.tp.method != 0 && a.tp.method != 1))) return hipErrorInvalidValue;
  if (a.el.flags & ~(uint32_t)(EL_PHASE | EL_COMPLEX | EL_LENS)) return hipErrorInvalidValue;
  if (a.nlines <= 0) return hipSuccess;
  if (a.h_lines <= 0) a.h_lines = a.nlines;
  if (a.field_rows <= 0) a.field_rows = a.nlines;
  if (a.in_es == 1 && a.out_es == 1) {
    switch (a.L) {
      case 2000: return launch_fixed<T, 2000>(a, mode, s);
      case 1000: return launch_fixed<T, 1000>(a, mode, s);
      case 500: return launch_fixed<T, 500>(a, mode, s);
      case 250: return launch_fixed<T, 250>(a, mode, s);
      case 100: return launch_fixed<T, 100>(a, mode, s);
      case 50: return launch_fixed<T, 50>(a, mode, s);
      default: break;
    }
  }
  int shift = 0;
  while ((kLinePoints << shift) < a.L) ++shift;  // L <= 16 TL, TL <= 256
  a.tl_shift = shift;
  const int G = 256 >> shift;
  const dim3 grid((a.nlines + G - 1) / G);
  if (mode < 0 && a.el.flags)
    hipLaunchKernelGGL((mixed_lines_kernel<T, -1, true>), grid, dim3(256), 0, s, a);
  else if (mode < 0)
    hipLaunchKernelGGL((mixed_lines_kernel<T, -1, false>), grid, dim3(256), 0, s, a);
  else if (mode > 0)
    hipLaunchKernelGGL((mixed_lines_kernel<T, +1, false>), grid, dim3(256), 0, s, a);
  else if (a.hcalc)
    hipLaunchKernelGGL((mixed_lines_kernel<T, 0, false, true>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((mixed_lines_kernel<T, 0, false>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t Mixed<T>::lines(int L, const MixedPlan& p, const cx<T>* tw, cx<T>* a, int nlines, int64_t lstride,
                           int64_t estride, int dir, hipStream_t s) {
  MixedArgs<T> m{};
  m.in = a;
  m.out = a;
  m.in_ls = m.out_ls = lstride;
  m.in_es = m.out_es = estride;
  m.nin = m.nout = L;
  m.scale = T(1);
  m.nlines = nlines;
  m.L = L;
  m.plan = p;
  m.tw = tw;
  return launch(m, dir < 0 ? -1 : 1, s);
}

template <typename T>
hipError_t Mixed<T>::transpose(const cx<T>* in, cx<T>* out, int rows, int cols, int64_t batch, hipStream_t s) {
  if (rows <= 0 || cols <= 0 || batch <= 0) return hipSuccess;
  for (int64_t z0 = 0; z0 < batch; z0 += 65535) {
    const unsigned nz = (unsigned)std::min<int64_t>(65535, batch - z0);
    hipLaunchKernelGGL((mixed_transpose_kernel<T>), dim3((cols + 31) / 32, (rows + 31) / 32, nz), dim3(256), 0, s,
                       in, out, rows, cols, z0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template struct Mixed<float>;
template struct Mixed<double>;

}  // namespace toprop
