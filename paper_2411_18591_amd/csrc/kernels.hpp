// Propagation kernels: zero-padded angular-spectrum / Fresnel transfer-
// function propagation of batches of fields, with the element modulation
// fused into the first pass and the crop, scaling and loss epilogues fused
// into the last pass (TorchOptics paper, section "Computational Fourier
// optics": Eq. (field_modulation), Eq. (field_propagation_tf),
// Eq. (transfer_function); section "Polarization" for the Jones product).
//
// A propagation of an ny x nx field on an LY x LX padded grid runs three
// kernels over a chunk of fields:
//   row_fwd : per field row y < ny: load nx samples, modulate, zero-extend
//             to LX, forward FFT, store all LX bins to the scratch buffer;
//   col     : per column tile of TC bins: forward FFT along y (ny non-zero
//             inputs, LY points), multiply by H (or conj H), inverse FFT,
//             keep the first ny rows, store back in place;
//   row_inv : per row y < ny: inverse FFT of the LX bins, keep the first nx
//             samples, scale by 1/(LX LY), epilogue.
// The field sits in the corner of the padded grid: the operator is a
// circular convolution, so the window position cancels between pad and
// crop.
//
// Scratch layout ("column tiles"): [field][LX/TC][ny][TC] complex, so that a
// column tile is one contiguous block for the column kernel and a row reads
// or writes TC contiguous bins per tile.
#pragma once
#include "fft.hpp"

namespace toprop {

// Element flags (mirrors the public header).
enum : uint32_t { EL_PHASE = 1u, EL_COMPLEX = 2u, EL_LENS = 4u, EL_JONES = 8u };
enum : int { EPI_NONE = 0, EPI_MSE = 1, EPI_WEIGHTED = 2 };

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>());
    static_for<B + 1, E>(f);
  }
}

// ---------------------------------------------------------------------------
// Trigonometric helpers.  Phases are carried in cycles; sincospi takes half
// cycles.
// ---------------------------------------------------------------------------
__device__ __forceinline__ cx<float> cis_cycles_reduced(double fr, float) {
  // fr in [-0.5, 0.5]
  float s, c;
  sincospif((float)(2.0 * fr), &s, &c);
  return {c, s};
}
__device__ __forceinline__ cx<double> cis_cycles_reduced(double fr, double) {
  double s, c;
  sincospi(2.0 * fr, &s, &c);
  return {c, s};
}
// exp(2 pi i c) for any c (cycles), reduced to [-0.5, 0.5] first in FP64.
template <typename T>
__device__ __forceinline__ cx<T> cis_cycles(double c) {
  double fr = c - rint(c);
  return cis_cycles_reduced(fr, T());
}
__device__ __forceinline__ cx<float> cis_rad(float a) {
  float s, c;
  sincosf(a, &s, &c);
  return {c, s};
}
__device__ __forceinline__ cx<double> cis_rad(double a) {
  double s, c;
  sincos(a, &s, &c);
  return {c, s};
}

// ---------------------------------------------------------------------------
// Parameters
// ---------------------------------------------------------------------------
struct TransferParams {
  int method;       // 0 = angular spectrum, 1 = Fresnel transfer function
  int conj;         // multiply by conj(H) (adjoint)
  double lam2;      // lambda^2
  double q;         // z / lambda
  double q_frac;    // frac(z / lambda), computed exactly on the host
  double fres_a;    // lambda z / 2
  double inv_lxdx;  // 1 / (LX dx)
  double inv_lydy;  // 1 / (LY dy)
};

// Transfer function at padded-grid bin (kx, ky), FFT order.
//   AS: H = exp(2 pi i z sqrt(1/lambda^2 - fx^2 - fy^2)) = exp(2 pi i c) with
//       c = q - q s / (1 + sqrt(1 - s)),  s = lambda^2 (fx^2 + fy^2),  q = z/lambda,
//       zero where s > 1 (evanescent).  The form avoids cancellation; frac(q)
//       replaces q so that the large integer part never enters the sum.
//   Fresnel TF: c = z/lambda - (lambda z / 2)(fx^2 + fy^2).
template <typename T>
__device__ __forceinline__ cx<T> transfer_at(int kx, int ky, int lx, int ly, const TransferParams& p) {
  const int kxs = kx < lx / 2 ? kx : kx - lx;
  const int kys = ky < ly / 2 ? ky : ky - ly;
  const double fx = (double)kxs * p.inv_lxdx;
  const double fy = (double)kys * p.inv_lydy;
  const double rho2 = fx * fx + fy * fy;
  double c;
  if (p.method == 0) {
    const double s = p.lam2 * rho2;
    if (s > 1.0) return {T(0), T(0)};
    c = p.q_frac - p.q * s / (1.0 + sqrt(1.0 - s));
  } else {
    c = p.q_frac - p.fres_a * rho2;
  }
  cx<T> h = cis_cycles<T>(c);
  if (p.conj) h.y = -h.y;
  return h;
}

template <typename T>
struct ElementParams {
  uint32_t flags;
  const T* phase;         // [ny][nx] radians
  const cx<T>* cmask;     // [ny][nx]
  double lens_a;          // 1 / (2 lambda f): lens phase = -r^2 * lens_a cycles
  double dy, dx, y0, x0;  // grid spacing and offset of the optical axis
  cx<T> jones[9];         // row-major 3x3
};

// Scalar modulation at pixel (y, x): phase mask, complex mask, thin lens.
template <typename T>
__device__ __forceinline__ cx<T> scalar_modulation(const ElementParams<T>& e, int ny, int nx, int y,
                                                   int x) {
  cx<T> m = {T(1), T(0)};
  const int64_t pix = (int64_t)y * nx + x;
  if (e.flags & EL_PHASE) m = cis_rad(e.phase[pix]);
  if (e.flags & EL_COMPLEX) m = cmul(m, e.cmask[pix]);
  if (e.flags & EL_LENS) {
    const double xc = (double)(x - nx / 2) * e.dx + e.x0;
    const double yc = (double)(y - ny / 2) * e.dy + e.y0;
    m = cmul(m, cis_cycles<T>(-(xc * xc + yc * yc) * e.lens_a));
  }
  return m;
}

// d(lens phase)/df in radians per metre at pixel (y, x): pi r^2 / (lambda f^2)
// = 2 pi r^2 lens_a / f.
template <typename T>
__device__ __forceinline__ double lens_dphase_df(const ElementParams<T>& e, int ny, int nx, int y,
                                                 int x, double f) {
  const double xc = (double)(x - nx / 2) * e.dx + e.x0;
  const double yc = (double)(y - ny / 2) * e.dy + e.y0;
  return 6.283185307179586476925286766559 * (xc * xc + yc * yc) * e.lens_a / f;
}

// ---------------------------------------------------------------------------
// The in-workgroup FFT: all passes of a length-L transform whose elements are
// spread over T = L/R threads, exchanging through LDS between passes.
// `lds` points at element 0 of this transform's LDS region; element `pos`
// lives at lds[pos * STRIDE].
// ---------------------------------------------------------------------------
template <typename T, int L, int R, int D, bool HALF_IN, int STRIDE>
__device__ __forceinline__ void fft_wg(cx<T>* v, int j, cx<T>* lds, const cx<T>* __restrict__ tw) {
  using S = Schedule<L, R>;
  constexpr int TT = S::T;
  static_for<0, S::npass>([&](auto pc) {
    constexpr int P = decltype(pc)::value;
    constexpr int RP = S::radix(P);
    constexpr int NS = S::ns(P);
    constexpr int NB = R / RP;
    stockham_butterflies<T, L, R, RP, NS, D, HALF_IN && P == 0>(v, j, tw);
    if constexpr (P + 1 < S::npass) {
      __syncthreads();
#pragma unroll
      for (int t = 0; t < NB; ++t)
#pragma unroll
        for (int i = 0; i < RP; ++i)
          lds[stockham_out_pos<L, R, RP, NS>(j, t, i) * STRIDE] = v[t + i * NB];
      __syncthreads();
#pragma unroll
      for (int m = 0; m < R; ++m) v[m] = lds[(j + m * TT) * STRIDE];
    }
  });
}

// ---------------------------------------------------------------------------
// Kernel arguments
// ---------------------------------------------------------------------------
template <typename T>
struct RowFwdArgs {
  const cx<T>* in;      // first field of the chunk; fields `in_stride` apart
  cx<T>* scratch;       // first field of the chunk in the scratch buffer
  int64_t in_stride;    // elements between consecutive fields (or field groups for NC=3)
  int64_t comp_stride;  // elements between components (NC = 3)
  int64_t s_stride;     // scratch elements per field (per component for NC = 3)
  int ny, nx;
  int tc_shift;         // log2 of the column-tile width
  int nfields;          // fields in this chunk (field groups for NC = 3)
  ElementParams<T> el;
  const cx<T>* tw;      // twiddles of length LX
};

template <typename T>
struct ColArgs {
  cx<T>* scratch;
  int64_t s_stride;
  int ny;
  int lx;               // padded row length (for the signed x frequency)
  int tcl;              // column-tile width of the scratch layout, <= TC
  int nfields;
  TransferParams h;
  const cx<T>* tw;      // twiddles of length LY
};

template <typename T>
struct RowInvArgs {
  const cx<T>* scratch;
  int64_t s_stride;
  int64_t comp_stride;  // elements between components in out/saved/grad arrays (NC = 3)
  cx<T>* out;           // forward: propagated field; backward: dL/d(input), may be null
  int64_t out_stride;
  int ny, nx;
  int tc_shift;
  int nfields;
  T scale;              // 1 / (LX LY)
  const cx<T>* tw;
  // forward loss epilogues
  int epi;
  const T* epi_ref;     // MSE target or intensity weight, [ny][nx]
  T epi_scale;
  cx<T>* epi_grad;      // dL/d(out), same layout as out
  double* row_partial;  // per (field, row) loss partial sums
  // backward: element adjoint and parameter gradients
  int backward;
  ElementParams<T> el;
  const cx<T>* saved_in;  // forward input of the layer
  T* grad_phase;          // [ny][nx], accumulated
  double lens_f;
  double* lens_partial;   // per row partial sums of dL/df
};

// ---------------------------------------------------------------------------
// row_fwd
// ---------------------------------------------------------------------------
template <typename T, int L, int R, int G, bool HALF, int NC>
__global__ void __launch_bounds__(G * (L / R)) row_fwd_kernel(RowFwdArgs<T> a) {
  constexpr int TT = L / R;
  __shared__ cx<T> lds[G * L];
  const int g = threadIdx.x / TT;
  const int j = threadIdx.x % TT;
  const int y = blockIdx.x * G + g;
  const int f = blockIdx.y;
  const bool active = (y < a.ny) && (f < a.nfields);
  const int ny = a.ny, nx = a.nx;

  cx<T> v[NC][R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const int x = j + m * TT;
    const bool inside = active && x < nx && (!HALF || m < R / 2);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      cx<T> val = {T(0), T(0)};
      if (inside) val = a.in[f * a.in_stride + c * a.comp_stride + (int64_t)y * nx + x];
      v[c][m] = val;
    }
    if (inside && a.el.flags) {
      if constexpr (NC == 3) {
        if (a.el.flags & EL_JONES) {
          cx<T> o[3];
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            o[r] = cmul(a.el.jones[3 * r + 0], v[0][m]);
            o[r] = cadd(o[r], cmul(a.el.jones[3 * r + 1], v[1][m]));
            o[r] = cadd(o[r], cmul(a.el.jones[3 * r + 2], v[2][m]));
          }
#pragma unroll
          for (int r = 0; r < 3; ++r) v[r][m] = o[r];
        }
      }
      if (a.el.flags & (EL_PHASE | EL_COMPLEX | EL_LENS)) {
        const cx<T> mod = scalar_modulation(a.el, ny, nx, y, x);
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c][m] = cmul(mod, v[c][m]);
      }
    }
  }
  const int tcm = (1 << a.tc_shift) - 1;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    fft_wg<T, L, R, -1, HALF, 1>(v[c], j, lds + g * L, a.tw);
    if (active) {
      cx<T>* dst = a.scratch + (int64_t)(f * NC + c) * a.s_stride;
#pragma unroll
      for (int m = 0; m < R; ++m) {
        const int kx = j + m * TT;
        dst[((int64_t)(kx >> a.tc_shift) * ny + y) * (tcm + 1) + (kx & tcm)] = v[c][m];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// col: forward FFT along y, transfer function, inverse FFT, crop rows.
// ---------------------------------------------------------------------------
template <typename T, int L, int R, int TC, bool HALF>
__global__ void __launch_bounds__(TC * (L / R)) col_kernel(ColArgs<T> a) {
  constexpr int TT = L / R;
  __shared__ cx<T> lds[L * TC];
  const int c = threadIdx.x % TC;
  const int j = threadIdx.x / TC;
  const int tile = blockIdx.x;
  const int f = blockIdx.y;
  const int ny = a.ny;
  const int tcl = a.tcl;  // tile width of the scratch layout (<= TC when the rows are short)
  cx<T>* base = a.scratch + (int64_t)f * a.s_stride + (int64_t)tile * ny * tcl;
  const bool active = f < a.nfields && c < tcl;

  cx<T> v[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const int y = j + m * TT;
    cx<T> val = {T(0), T(0)};
    if (active && y < ny && (!HALF || m < R / 2)) val = base[(int64_t)y * tcl + c];
    v[m] = val;
  }
  fft_wg<T, L, R, -1, HALF, TC>(v, j, lds + c, a.tw);
  const int kx = tile * tcl + c;
#pragma unroll
  for (int m = 0; m < R; ++m) v[m] = cmul(v[m], transfer_at<T>(kx, j + m * TT, a.lx, L, a.h));
  fft_wg<T, L, R, +1, false, TC>(v, j, lds + c, a.tw);
  if (active) {
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int y = j + m * TT;
      if ((!HALF || m < R / 2) && y < ny) base[(int64_t)y * tcl + c] = v[m];
    }
  }
}

// ---------------------------------------------------------------------------
// Block reduction of one double per thread (fixed order: deterministic).
// ---------------------------------------------------------------------------
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
  __syncthreads();
  red[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  return red[0];
}

// Sum of the TT threads of one row group (threads g*TT .. g*TT+TT-1).
template <int TT, int G>
__device__ __forceinline__ double group_sum(double v, double* red) {
  __syncthreads();
  red[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int s = TT / 2; s > 0; s >>= 1) {
    if ((int)(threadIdx.x % TT) < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  return red[(threadIdx.x / TT) * TT];
}

// ---------------------------------------------------------------------------
// row_inv: inverse FFT along x, crop, scale and epilogue.
//   Forward (backward == 0): store the field; optionally the loss gradient
//     and per-row loss partials (MSE of |u|^2 against a target, or a
//     weighted intensity).
//   Backward (backward == 1): the rows hold g_mod = P^H g.  Store
//     dL/d(input) = M^H g_mod, accumulate dL/dphi += Im(g_mod conj(M u_in))
//     over the chunk's fields, and per-row partials of dL/df for a lens.
//     Fields are looped inside the block so each pixel's gradient is summed
//     by one thread in a fixed order.
// ---------------------------------------------------------------------------
template <typename T, int L, int R, int G, bool HALF, int NC>
__global__ void __launch_bounds__(G * (L / R)) row_inv_kernel(RowInvArgs<T> a) {
  constexpr int TT = L / R;
  constexpr int NT = G * TT;
  constexpr int RO = HALF ? R / 2 : R;  // output registers that can hold x < nx
  __shared__ cx<T> lds[G * L];
  __shared__ double red[NT];
  const int g = threadIdx.x / TT;
  const int j = threadIdx.x % TT;
  const int y = blockIdx.x * G + g;
  const int ny = a.ny, nx = a.nx;
  const bool rowok = y < ny;
  const int tcm = (1 << a.tc_shift) - 1;
  const bool loop_fields = a.backward != 0;
  const int f_begin = loop_fields ? 0 : blockIdx.y;
  const int f_end = loop_fields ? a.nfields : min((int)blockIdx.y + 1, a.nfields);

  T gphase[RO];
#pragma unroll
  for (int m = 0; m < RO; ++m) gphase[m] = T(0);
  double lens_acc = 0.0;

  for (int f = f_begin; f < (loop_fields ? f_end : f_begin + 1); ++f) {
    const bool active = rowok && f < f_end;
    cx<T> v[NC][R];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const cx<T>* src = a.scratch + (int64_t)(f * NC + c) * a.s_stride;
#pragma unroll
      for (int m = 0; m < R; ++m) {
        const int kx = j + m * TT;
        cx<T> val = {T(0), T(0)};
        if (active) val = src[((int64_t)(kx >> a.tc_shift) * ny + y) * (tcm + 1) + (kx & tcm)];
        v[c][m] = val;
      }
      fft_wg<T, L, R, +1, false, 1>(v[c], j, lds + g * L, a.tw);
    }
    double loss_acc = 0.0;
    if (active) {
#pragma unroll
      for (int m = 0; m < RO; ++m) {
        const int x = j + m * TT;
        if (x >= nx) continue;
        const int64_t pix = (int64_t)y * nx + x;
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c][m] = cscale(v[c][m], a.scale);
        if (!a.backward) {
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const int64_t o = f * a.out_stride + c * a.comp_stride + pix;
            a.out[o] = v[c][m];
            if (a.epi == EPI_MSE) {
              const T I = v[c][m].x * v[c][m].x + v[c][m].y * v[c][m].y;
              const T d = I - a.epi_ref[pix];
              loss_acc += (double)d * (double)d;
              a.epi_grad[o] = cscale(v[c][m], T(4) * a.epi_scale * d);
            } else if (a.epi == EPI_WEIGHTED) {
              const T I = v[c][m].x * v[c][m].x + v[c][m].y * v[c][m].y;
              const T w = a.epi_ref[pix];
              loss_acc += (double)w * (double)I;
              a.epi_grad[o] = cscale(v[c][m], T(2) * a.epi_scale * w);
            }
          }
        } else {
          // g_mod is v; the modulated forward field is M u_in.
          cx<T> mod = {T(1), T(0)};
          const uint32_t fl = a.el.flags;
          if (fl & (EL_PHASE | EL_COMPLEX | EL_LENS)) mod = scalar_modulation(a.el, ny, nx, y, x);
          if ((fl & (EL_PHASE | EL_LENS)) && a.saved_in) {
            cx<T> u[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) u[c] = a.saved_in[f * a.out_stride + c * a.comp_stride + pix];
            if constexpr (NC == 3) {
              if (fl & EL_JONES) {
                cx<T> o[3];
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                  o[r] = cmul(a.el.jones[3 * r + 0], u[0]);
                  o[r] = cadd(o[r], cmul(a.el.jones[3 * r + 1], u[1]));
                  o[r] = cadd(o[r], cmul(a.el.jones[3 * r + 2], u[2]));
                }
#pragma unroll
                for (int r = 0; r < 3; ++r) u[r] = o[r];
              }
            }
            T im = T(0);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
              const cx<T> um = cmul(mod, u[c]);
              im += v[c][m].y * um.x - v[c][m].x * um.y;  // Im(g conj(um))
            }
            if (fl & EL_PHASE) gphase[m] += im;
            if (fl & EL_LENS) lens_acc += (double)im * lens_dphase_df(a.el, ny, nx, y, x, a.lens_f);
          }
          if (a.out) {
            cx<T> gi[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) gi[c] = cmulc(v[c][m], mod);  // conj(M) g
            if constexpr (NC == 3) {
              if (fl & EL_JONES) {  // J^H g
                cx<T> o[3];
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                  o[r] = cmulc(gi[0], a.el.jones[0 * 3 + r]);
                  o[r] = cadd(o[r], cmulc(gi[1], a.el.jones[1 * 3 + r]));
                  o[r] = cadd(o[r], cmulc(gi[2], a.el.jones[2 * 3 + r]));
                }
#pragma unroll
                for (int r = 0; r < 3; ++r) gi[r] = o[r];
              }
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) a.out[f * a.out_stride + c * a.comp_stride + pix] = gi[c];
          }
        }
      }
    }
    if (!a.backward && a.epi != EPI_NONE) {
      const double s = group_sum<TT, G>(loss_acc, red);
      if (active && j == 0) a.row_partial[(int64_t)f * ny + y] = s;
    }
  }
  if (a.backward) {
    if (rowok && (a.el.flags & EL_PHASE) && a.grad_phase && a.saved_in) {
#pragma unroll
      for (int m = 0; m < RO; ++m) {
        const int x = j + m * TT;
        if (x < nx) a.grad_phase[(int64_t)y * nx + x] += gphase[m];
      }
    }
    if ((a.el.flags & EL_LENS) && a.lens_partial) {
      const double s = group_sum<TT, G>(lens_acc, red);
      if (rowok && j == 0) a.lens_partial[y] = s;
    }
  }
}

// Sum `n` doubles in a fixed order and add scale * sum to *dst (one block).
template <int NT>
__global__ void __launch_bounds__(NT) reduce_add_kernel(const double* src, int64_t n, double scale,
                                                        double* dst) {
  __shared__ double red[NT];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += NT) acc += src[i];
  const double s = block_sum<NT>(acc, red);
  if (threadIdx.x == 0) *dst += scale * s;
}

// Plain modulation out = M in (or M^H in for the adjoint), no propagation.
template <typename T, int NC>
__global__ void __launch_bounds__(256) modulate_kernel(const cx<T>* in, cx<T>* out, int64_t fstride,
                                                       int64_t cstride, int ny, int nx, int nfields,
                                                       int adjoint, ElementParams<T> el) {
  const int64_t npix = (int64_t)ny * nx;
  const int64_t total = npix * nfields;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t f = i / npix, pix = i % npix;
    const int y = (int)(pix / nx), x = (int)(pix % nx);
    cx<T> v[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = in[f * fstride + c * cstride + pix];
    cx<T> mod = {T(1), T(0)};
    if (el.flags & (EL_PHASE | EL_COMPLEX | EL_LENS)) mod = scalar_modulation(el, ny, nx, y, x);
    if (adjoint) mod.y = -mod.y;
    if (!adjoint) {
      if constexpr (NC == 3) {
        if (el.flags & EL_JONES) {
          cx<T> o[3];
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            o[r] = cmul(el.jones[3 * r + 0], v[0]);
            o[r] = cadd(o[r], cmul(el.jones[3 * r + 1], v[1]));
            o[r] = cadd(o[r], cmul(el.jones[3 * r + 2], v[2]));
          }
#pragma unroll
          for (int r = 0; r < 3; ++r) v[r] = o[r];
        }
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) v[c] = cmul(mod, v[c]);
    } else {
#pragma unroll
      for (int c = 0; c < NC; ++c) v[c] = cmul(mod, v[c]);
      if constexpr (NC == 3) {
        if (el.flags & EL_JONES) {
          cx<T> o[3];
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            o[r] = cmulc(v[0], el.jones[0 * 3 + r]);
            o[r] = cadd(o[r], cmulc(v[1], el.jones[1 * 3 + r]));
            o[r] = cadd(o[r], cmulc(v[2], el.jones[2 * 3 + r]));
          }
#pragma unroll
          for (int r = 0; r < 3; ++r) v[r] = o[r];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) out[f * fstride + c * cstride + pix] = v[c];
  }
}

}  // namespace toprop
