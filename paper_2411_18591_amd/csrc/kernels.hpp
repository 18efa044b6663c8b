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
enum : uint32_t { EL_PHASE = 1u, EL_COMPLEX = 2u, EL_LENS = 4u, EL_JONES = 8u, EL_JONES_MAP = 16u };
enum : int { EPI_NONE = 0, EPI_MSE = 1, EPI_WEIGHTED = 2, EPI_INTENSITY = 3 };

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>());
    static_for<B + 1, E>(f);
  }
}

// Workgroups of a launch are dispatched round-robin over the 8 XCDs of the
// MI355X (block b runs on XCD b mod 8), and each XCD has its own L2.  This
// maps the dispatch index to a logical index so that every XCD receives one
// contiguous range: neighbouring rows, whose column-tile segments share
// cache lines, are then processed under the same L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
  constexpr int kXcd = 8;
  const int per = n / kXcd, rem = n % kXcd;
  const int x = b % kXcd, k = b / kXcd;
  return x * per + min(x, rem) + k;
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
// exp(i a) for a phase in radians: converted to cycles and reduced to
// [-0.5, 0.5] first, so sincospi needs no large-argument reduction.  The
// conversion rounds a * (1/2pi) to FP32, an error below one ulp of a itself.
__device__ __forceinline__ cx<float> cis_rad(float a) {
  const float c = a * 0.15915494309189533577f;
  const float fr = c - rintf(c);
  float s, co;
  sincospif(2.0f * fr, &s, &co);
  return {co, s};
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
  int method;       // 0 = angular spectrum, 1 = Fresnel transfer function,
                    // 2 = table (direct integration: H read from `table`)
  int conj;         // multiply by conj(H) (adjoint)
  const void* table;  // method 2: complex of the field type, [LY][LX], FFT order
  double lam2;      // lambda^2
  double q;         // z / lambda
  double q_frac;    // frac(z / lambda), computed exactly on the host
  double fres_a;    // lambda z / 2
  double inv_lxdx;  // 1 / (LX dx)
  double inv_lydy;  // 1 / (LY dy)
  // Separable form (complex64 path only, chosen by the host when accurate):
  //   H = ey[ky] ex[kx] exp(-2 pi i (q/2) t^2),  t = s / (1 + sqrt(1 - s)),
  //   s = sx[kx] + sy[ky] = lambda^2 (fx^2 + fy^2)
  // where ex = exp(-2 pi i (lambda z/2) fx^2) and ey = exp(2 pi i (frac(z/lambda)
  // - (lambda z/2) fy^2)) are built in FP64 by tf_tables_kernel.  The last
  // factor is the non-paraxial remainder of the angular spectrum, since
  // z sqrt(1/lambda^2 - f^2) = z/lambda - (lambda z/2) f^2 - (q/2) t^2; the
  // host uses this path only when (q/2) t^2 stays below one cycle, so FP32
  // evaluates it to ~1e-7 cycles.  Fresnel: the remainder is absent.
  int fast;
  float qh;               // q / 2
  const cx<float>* ex;
  const cx<float>* ey;
  const float* sx;
  const float* sy;
};

// Transfer function at padded-grid bin (kx, ky), FFT order.
//   AS: H = exp(2 pi i z sqrt(1/lambda^2 - fx^2 - fy^2)) = exp(2 pi i c) with
//       c = q - q s / (1 + sqrt(1 - s)),  s = lambda^2 (fx^2 + fy^2),  q = z/lambda,
//       zero where s > 1 (evanescent).  The form avoids cancellation; frac(q)
//       replaces q so that the large integer part never enters the sum.
//   Fresnel TF: c = z/lambda - (lambda z / 2)(fx^2 + fy^2).
//
// complex64: the same phase with the square root and the quotient formed
// from the hardware FP64 reciprocal square root and reciprocal, each
// refined by two Newton steps (relative error a few ulp of FP64, i.e.
// below 1e-10 cycles on a term of at most ~1e5 cycles), and the reduced
// phase turned into cos/sin by the hardware FP32 sine and cosine, whose
// argument is in revolutions (absolute error ~1.2e-7 on [-1, 1]); far
// cheaper than the correctly rounded FP64 sqrt, division and FP32
// sincospi, and accurate to FP32 rounding of H.  complex128 keeps the
// correctly rounded operations throughout.
__device__ __forceinline__ double asm_t_c64(double s) {
  // t = s / (1 + sqrt(1 - s)), 0 <= s <= 1
  const double r = 1.0 - s;
  double y = __builtin_amdgcn_rsq(r > 0.0 ? r : 1.0);  // 1/sqrt(r)
  double g = r * y, hy = 0.5 * y;
#pragma unroll
  for (int it = 0; it < 2; ++it) {  // Newton on (g, hy) -> (sqrt r, 1 / (2 sqrt r))
    const double e = fma(-g, hy, 0.5);
    g = fma(g, e, g);
    hy = fma(hy, e, hy);
  }
  const double sq = r > 0.0 ? g : 0.0;
  const double d = 1.0 + sq;
  double x = __builtin_amdgcn_rcp(d);
#pragma unroll
  for (int it = 0; it < 2; ++it) x = fma(x, fma(-d, x, 1.0), x);
  return s * x;
}

template <typename T>
__device__ __forceinline__ cx<T> transfer_at(int kx, int ky, int lx, int ly, const TransferParams& p) {
  const int kxs = 2 * kx < lx ? kx : kx - lx;
  const int kys = 2 * ky < ly ? ky : ky - ly;
  const double fx = (double)kxs * p.inv_lxdx;
  const double fy = (double)kys * p.inv_lydy;
  const double rho2 = fx * fx + fy * fy;
  double c;
  if (p.method == 0) {
    const double s = p.lam2 * rho2;
    if (s > 1.0) return {T(0), T(0)};
    if constexpr (std::is_same<T, float>::value)
      c = p.q_frac - p.q * asm_t_c64(s);
    else
      c = p.q_frac - p.q * s / (1.0 + sqrt(1.0 - s));
  } else {
    c = p.q_frac - p.fres_a * rho2;
  }
  cx<T> h;
  if constexpr (std::is_same<T, float>::value) {
    const float fr = (float)(c - rint(c));
    h = {__builtin_amdgcn_cosf(fr), __builtin_amdgcn_sinf(fr)};
  } else {
    h = cis_cycles<T>(c);
  }
  if (p.conj) h.y = -h.y;
  return h;
}

// Separable complex64 transfer function (see TransferParams).  `exk`/`sxk`
// are the column's table entries.
__device__ __forceinline__ cx<float> transfer_fast(cx<float> exk, float sxk, int ky, int ly,
                                                   float lam_fy_unit, const TransferParams& p) {
  cx<float> h = cmul(exk, p.ey[ky]);
  if (p.method == 0) {
    // s = lambda^2 (fx^2 + fy^2); the y part from the bin index in FP32
    // (relative error ~1e-7 on a remainder below one cycle)
    const float gy = (float)(2 * ky < ly ? ky : ky - ly) * lam_fy_unit;
    const float s = fmaf(gy, gy, sxk);
    // v_sqrt / v_rcp (~1 ulp) and v_sin / v_cos, whose argument is in
    // revolutions (|theta| <= 1 here; absolute error ~1.2e-7): the
    // remainder needs ~1e-6 relative accuracy only.
    const float t = s * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_sqrtf(1.0f - s));
    const float theta = -p.qh * t * t;
    h = cmul(h, cx<float>{__builtin_amdgcn_cosf(theta), __builtin_amdgcn_sinf(theta)});
  }
  if (p.conj) h.y = -h.y;
  return h;
}

// Entry i of the FP64-built tables of the separable transfer function of one
// propagation: entries 0..lx-1 are the x tables, lx..lx+ly-1 the y tables.
__device__ __forceinline__ void tf_table_entry(int i, cx<float>* ex, float* sx, int lx, double inv_lxdx,
                                               cx<float>* ey, float* sy, int ly, double inv_lydy,
                                               double fres_a, double q_frac, double lam2) {
  if (i < lx) {
    const int ks = 2 * i < lx ? i : i - lx;
    const double f = (double)ks * inv_lxdx;
    const double c = -fres_a * f * f;
    double s, co;
    sincospi(2.0 * (c - rint(c)), &s, &co);
    ex[i] = {(float)co, (float)s};
    sx[i] = (float)(lam2 * f * f);
  } else if (i < lx + ly) {
    const int k = i - lx;
    const int ks = 2 * k < ly ? k : k - ly;
    const double f = (double)ks * inv_lydy;
    const double c = q_frac - fres_a * f * f;
    double s, co;
    sincospi(2.0 * (c - rint(c)), &s, &co);
    ey[k] = {(float)co, (float)s};
    sy[k] = (float)(lam2 * f * f);
  }
}

template <typename T>
__global__ void __launch_bounds__(256) tf_tables_kernel(cx<float>* ex, float* sx, int lx,
                                                        double inv_lxdx, cx<float>* ey, float* sy,
                                                        int ly, double inv_lydy, double fres_a,
                                                        double q_frac, double lam2) {
  tf_table_entry(blockIdx.x * blockDim.x + threadIdx.x, ex, sx, lx, inv_lxdx, ey, sy, ly, inv_lydy, fres_a,
                 q_frac, lam2);
}

template <typename T>
struct ElementParams {
  uint32_t flags;
  const T* phase;         // [ny][nx] radians
  const cx<T>* cmask;     // [ny][nx]
  double lens_a;          // 1 / (2 lambda f): lens phase = -r^2 * lens_a cycles
  double dy, dx, y0, x0;  // grid spacing and offset of the optical axis
  cx<T> jones[9];         // row-major 3x3
  const cx<T>* jones_map; // EL_JONES_MAP: [3][3][ny][nx], entry (r, c) at plane 3 r + c
  int64_t plane;          // ny * nx
};

// Jones matrix entry k = 3 r + c at pixel `pix` (uniform or mapped).
template <typename T>
__device__ __forceinline__ cx<T> jones_entry(const ElementParams<T>& e, int64_t pix, int k) {
  return (e.flags & EL_JONES_MAP) ? e.jones_map[k * e.plane + pix] : e.jones[k];
}

// v <- J v at pixel `pix`.
template <typename T>
__device__ __forceinline__ void apply_jones(const ElementParams<T>& e, int64_t pix, cx<T>* v) {
  cx<T> o[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    o[r] = cmul(jones_entry(e, pix, 3 * r + 0), v[0]);
    o[r] = cadd(o[r], cmul(jones_entry(e, pix, 3 * r + 1), v[1]));
    o[r] = cadd(o[r], cmul(jones_entry(e, pix, 3 * r + 2), v[2]));
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) v[r] = o[r];
}

// v <- J^H v at pixel `pix`.
template <typename T>
__device__ __forceinline__ void apply_jones_adjoint(const ElementParams<T>& e, int64_t pix, cx<T>* v) {
  cx<T> o[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    o[r] = cmulc(v[0], jones_entry(e, pix, 0 * 3 + r));
    o[r] = cadd(o[r], cmulc(v[1], jones_entry(e, pix, 1 * 3 + r)));
    o[r] = cadd(o[r], cmulc(v[2], jones_entry(e, pix, 2 * 3 + r)));
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) v[r] = o[r];
}

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
// LDS position of transform element `pos`, padded against bank conflicts
// (64 banks of 4 bytes, 64-bit accesses).  Rows (STRIDE 1): two pad slots
// every 32 elements plus one every 128; column tiles (STRIDE = columns per
// block, element (pos, c) at lds_pos(pos) * STRIDE + c): one pad row every 16
// rows, which makes every Stockham write and read pattern conflict-free.
template <int STRIDE>
__device__ __forceinline__ constexpr int lds_pos(int pos) {
  if constexpr (STRIDE == 1)
    return pos + 2 * (pos >> 5) + (pos >> 7);
  else
    return pos + (pos >> 4);
}
// STRIDE = -1: a single transform (stride 1) with the column-tile padding,
// which the split row transforms use (their exchange patterns are
// conflict-free or nearly so under it, not under the row padding).
template <int STRIDE>
__device__ __forceinline__ constexpr int lds_mul() {
  return STRIDE < 0 ? 1 : STRIDE;
}
template <int STRIDE>
constexpr int lds_len(int L) {  // elements (per column) of a padded exchange buffer
  return STRIDE == 1 ? L + 2 * (L >> 5) + (L >> 7) : L + (L >> 4);
}

// Orders this wavefront's LDS accesses before and after it without a
// workgroup barrier: the LDS unit executes one wave's instructions in issue
// order, so only the compiler's reordering has to be stopped.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// WAVE: every thread of the transform sits in the calling thread's
// wavefront, so the exchanges between passes need no workgroup barrier.
template <typename T, int L, int R, int D, bool HALF_IN, int STRIDE, bool WAVE = false>
__device__ __forceinline__ void fft_wg(cx<T>* v, int j, cx<T>* lds, const cx<T>* __restrict__ tw) {
  using S = Schedule<L, R>;
  constexpr int TT = S::T;
  auto sync = [] {
    if constexpr (WAVE)
      wave_sync();
    else
      __syncthreads();
  };
  static_for<0, S::npass>([&](auto pc) {
    constexpr int P = decltype(pc)::value;
    constexpr int RP = S::radix(P);
    constexpr int NS = S::ns(P);
    constexpr int NB = R / RP;
    stockham_butterflies<T, L, R, RP, NS, D, HALF_IN && P == 0>(v, j, tw);
    if constexpr (P + 1 < S::npass) {
      // The padding adds floor(p/32)*2 + floor(p/128) (rows) or floor(p/16)
      // (column tiles) slots.  Output i of a butterfly sits at p0 + i NS with
      // p0 = Q + r, Q a multiple of NS RP and r < NS, and no carry out of the
      // low bits can occur in that sum, so lds_pos(p0 + i NS) =
      // lds_pos(p0) + lds_pos(i NS); likewise lds_pos(j + m TT) =
      // lds_pos(j) + lds_pos(m TT) for j < TT.  Every element offset is
      // therefore a compile-time immediate on one per-thread base.
      sync();
#pragma unroll
      for (int t = 0; t < NB; ++t) {
        const int p0 = stockham_out_pos<L, R, RP, NS>(j, t, 0);
        const int b0 = lds_pos<STRIDE>(p0) * lds_mul<STRIDE>();
#pragma unroll
        for (int i = 0; i < RP; ++i) lds[b0 + lds_pos<STRIDE>(i * NS) * lds_mul<STRIDE>()] = v[t + i * NB];
      }
      sync();
      const int r0 = lds_pos<STRIDE>(j) * lds_mul<STRIDE>();
#pragma unroll
      for (int m = 0; m < R; ++m) v[m] = lds[r0 + lds_pos<STRIDE>(m * TT) * lds_mul<STRIDE>()];
    }
  });
}

// ---------------------------------------------------------------------------
// Split transform: a length-L transform as one radix-R pass across the whole
// transform and R sub-transforms of M = L/R points, each held by TS = M/R
// consecutive threads (X[R k + g] = sum_a w_M^{a k} w_L^{a g} sum_b
// x[a + M b] w_R^{b g}).  When a sub-transform's threads share one
// wavefront, its exchanges need no workgroup barrier.  Two orders:
//  natural: thread j holds element j + m M in register m (as fft_wg);
//  split:   thread j = g TS + s holds element R (s + m TS) + g, i.e.
//           base(j) + m M.
// split_dif takes natural order to split order (the radix-R pass first);
// split_dit takes split order to natural order (the sub-transforms first).
// A forward split_dif + inverse split_dit pair (or inverse + forward) costs
// three workgroup barriers instead of 4 (npass - 1).
// ---------------------------------------------------------------------------
template <int L, int R, int STRIDE, int WAVE_THREADS>
struct Split {
  static constexpr int M = L / R;
  static constexpr int TS = M / R;
  // WAVE_THREADS: threads of one sub-transform (with all STRIDE columns of a
  // column tile) that must fit one wavefront; lds_pos splits over g M + p
  // when M is a multiple of the padding period (16 for the column-tile
  // padding, which the split rows use too (STRIDE = -1); 128 for the row
  // padding)
  static constexpr bool ok = L >= R * R && R >= 4 && WAVE_THREADS <= 64 && (64 % WAVE_THREADS) == 0 &&
                             M % (STRIDE == 1 ? 128 : 16) == 0;
  __device__ __forceinline__ static int base(int j) { return R * (j % TS) + j / TS; }
};
template <int L, int R, int TC>
using ColSplit = Split<L, R, TC, (L / R / R) * TC>;
template <int L, int R>
using RowSplit = Split<L, R, -1, L / R / R>;

// Radix-R pass over registers m (elements j + m M), then the twiddles
// w_L^{D j g} on output g.
template <typename T, int L, int R, int D, bool HALF_IN>
__device__ __forceinline__ void split_outer(cx<T>* v, int j, const cx<T>* __restrict__ tw) {
  const rsrc_t twr = buf_rsrc(tw, (uint32_t)(L * sizeof(cx<T>)));
  if constexpr (HALF_IN)
    DftHalfZero<R, D, T>::run(v);
  else
    Dft<R, D, T>::run(v);
#pragma unroll
  for (int g = 1; g < R; ++g) {
    cx<T> w = buf_ld<T>(twr, __umul24((uint32_t)j, (uint32_t)(g * sizeof(cx<T>))), 0u);
    if (D > 0) w.y = -w.y;
    v[g] = cmul(v[g], w);
  }
}

// Positions g M + j (j < M) and s + m TS (s < TS; TS, 32 and 128 powers of
// two) add without a carry into the padding bits, so lds_pos splits into a
// per-thread base plus a compile-time offset.
template <typename T, int L, int R, int D, bool HALF_IN, int STRIDE>
__device__ __forceinline__ void split_dif(cx<T>* v, int j, cx<T>* lds, const cx<T>* __restrict__ tw) {
  using SP = Split<L, R, STRIDE, 1>;
  constexpr int M = SP::M, TS = SP::TS;
  split_outer<T, L, R, D, HALF_IN>(v, j, tw);
  const int wb = lds_pos<STRIDE>(j) * lds_mul<STRIDE>();
  __syncthreads();  // earlier readers of the buffer are done
#pragma unroll
  for (int g = 0; g < R; ++g) lds[wb + lds_pos<STRIDE>(g * M) * lds_mul<STRIDE>()] = v[g];
  __syncthreads();
  const int g = j / TS, s = j % TS;
  cx<T>* sub = lds + lds_pos<STRIDE>(g * M) * lds_mul<STRIDE>();
  const int rb = lds_pos<STRIDE>(s) * lds_mul<STRIDE>();
#pragma unroll
  for (int m = 0; m < R; ++m) v[m] = sub[rb + lds_pos<STRIDE>(m * TS) * lds_mul<STRIDE>()];
  // the sub-transform's twiddles: the length-M table (packed before L's)
  fft_wg<T, M, R, D, false, STRIDE, true>(v, s, sub, tw - (L - M));
}

// HALF_IN: registers m >= R/2 are zero (elements from L/2 on, in split order
// as in natural order).  Since the last workgroup barrier only this
// wavefront may have touched its sub-transform's region.
template <typename T, int L, int R, int D, bool HALF_IN, int STRIDE>
__device__ __forceinline__ void split_dit(cx<T>* v, int j, cx<T>* lds, const cx<T>* __restrict__ tw) {
  using SP = Split<L, R, STRIDE, 1>;
  constexpr int M = SP::M, TS = SP::TS;
  const int g = j / TS, s = j % TS;
  cx<T>* sub = lds + lds_pos<STRIDE>(g * M) * lds_mul<STRIDE>();
  wave_sync();
  fft_wg<T, M, R, D, HALF_IN, STRIDE, true>(v, s, sub, tw - (L - M));
  wave_sync();
  const int rb = lds_pos<STRIDE>(s) * lds_mul<STRIDE>();
#pragma unroll
  for (int m = 0; m < R; ++m) sub[rb + lds_pos<STRIDE>(m * TS) * lds_mul<STRIDE>()] = v[m];
  __syncthreads();
  const int wb = lds_pos<STRIDE>(j) * lds_mul<STRIDE>();
#pragma unroll
  for (int q = 0; q < R; ++q) v[q] = lds[wb + lds_pos<STRIDE>(q * M) * lds_mul<STRIDE>()];
  // w_L^{D j g} on input g, then the radix-R pass over g
  const rsrc_t twr = buf_rsrc(tw, (uint32_t)(L * sizeof(cx<T>)));
#pragma unroll
  for (int q = 1; q < R; ++q) {
    cx<T> w = buf_ld<T>(twr, __umul24((uint32_t)j, (uint32_t)(q * sizeof(cx<T>))), 0u);
    if (D > 0) w.y = -w.y;
    v[q] = cmul(v[q], w);
  }
  Dft<R, D, T>::run(v);
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
  int fpb;              // fields per block (the modulation is evaluated once for them)
  // Coherence rows: field f of the chunk is row r1 = f_off + f of a mutual
  // coherence matrix; the modulation is coh_m[r1] conj(coh_m[pixel]).
  const cx<T>* coh_m;
  int64_t f_off;
  ElementParams<T> el;
  const cx<T>* tw;      // twiddles of length LX
};

template <typename T>
struct ColArgs {
  cx<T>* scratch;
  int64_t s_stride;
  int ny;
  int lx;               // padded row length (for the signed x frequency)
  int tm;               // column-tile width of the scratch layout
  int cpb;              // columns transformed per block (<= TC, divides tm)
  int nfields;
  int fpc;              // fields per block: the transfer function is formed once for them
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
  T* epi_out;           // intensity epilogue: [field][ny][nx], accumulated
  double* row_partial;  // per (field, row) loss partial sums
  // backward: element adjoint and parameter gradients
  int backward;
  int fpb;                // forward: fields per block (backward: all fields of the chunk)
  ElementParams<T> el;
  const cx<T>* saved_in;  // forward input of the layer
  T* grad_phase;          // [ny][nx], accumulated
  double lens_f;
  double* lens_partial;   // per row partial sums of dL/df
};

// Waves per SIMD that fit on a CU given a workgroup's LDS footprint (160 KiB
// of LDS per CU, 4 SIMDs): the register budget the compiler may assume.
constexpr int waves_per_simd(int threads, int lds_bytes) {
  const int wg = lds_bytes > 0 ? 163840 / lds_bytes : 8;
  const int w = (wg < 1 ? 1 : wg) * threads / 256;
  return w < 1 ? 1 : (w > 8 ? 8 : w);
}

// ---------------------------------------------------------------------------
// Addressing shared by the row passes.
//
// A row pass owns rows of the padded grid: thread j of a row holds the
// elements x = j + m TT, m < R.  Threads of one row are whole waves when
// TT >= 64, so the row index is then wave-uniform (readfirstlane), and so is
// every branch on it.  Field rows ([..][ny][nx], x fastest) put element m at
// lane offset (y nx + j) plus a uniform m TT; scratch rows in the
// column-tile layout [LX/tm][ny][tm] put element kx = j + m TT at
// ((kx / tm) ny + y) tm + kx % tm, which with TT a multiple of tm (TT >= 16
// >= tm) is a lane offset plus a uniform m TT ny.  Both go to buffer
// accesses whose uniform part sits in a scalar register.
//
// EX ("exact width"): the field fills exactly the registers that can hold
// it (nx == RI TT, RI = R/2 on a half-padded row, else R), so the test
// x < nx reduces to the compile-time m < RI.
// ---------------------------------------------------------------------------
// LDS bytes of a row-pass workgroup: G padded rows (+ a double per thread
// for the reductions of the kernels that have them).
template <typename T, int L, int R, int G, bool RED>
constexpr int row_lds_bytes() {
  return G * lds_len<1>(L) * (int)sizeof(cx<T>) + (RED ? G * (L / R) * 8 : 0);
}

// Occupancy the row passes ask the compiler to keep: the waves per SIMD
// their LDS allows, at most four (128 registers).  Three-component passes,
// which hold three rows of registers, are left to the compiler.
constexpr int row_min_waves(int nc, int w) { return nc == 1 ? (w < 4 ? w : 4) : 1; }

template <int TT>
__device__ __forceinline__ int row_group(int tid = (int)threadIdx.x) {
  const int g = tid / TT;
  if constexpr (TT >= 64) return __builtin_amdgcn_readfirstlane(g);
  return g;
}

template <typename T, int TT>
struct TileRow {
  uint32_t vo;  // lane part (bytes)
  int j, y, ny, shift;
  __device__ __forceinline__ TileRow(int j_, int y_, int ny_, int shift_) : j(j_), y(y_), ny(ny_), shift(shift_) {
    if constexpr (TT >= 16)
      vo = (uint32_t)(((((j >> shift) * ny + y) << shift) + (j & ((1 << shift) - 1))) * (int)sizeof(cx<T>));
    else
      vo = 0;
  }
  // lane and uniform byte offsets of register m
  __device__ __forceinline__ uint32_t v(int m) const {
    if constexpr (TT >= 16) {
      return vo;
    } else {
      const int kx = j + m * TT;
      return (uint32_t)(((((kx >> shift) * ny + y) << shift) + (kx & ((1 << shift) - 1))) * (int)sizeof(cx<T>));
    }
  }
  __device__ __forceinline__ uint32_t s(int m) const {
    if constexpr (TT >= 16)
      return (uint32_t)m * (uint32_t)(TT * ny) * (uint32_t)sizeof(cx<T>);
    else
      return 0u;
  }
};

// ---------------------------------------------------------------------------
// row_fwd
// ---------------------------------------------------------------------------
// The body of a workgroup of the pass, at block (bx, by) of a grid gx
// blocks wide, for thread `tid` of the workgroup: the kernel below runs it at
// its own block index, the job-queue kernel at the index of each item it
// takes (with an opaque copy of the thread index, so that nothing derived
// from it is hoisted out of the item loop and held in registers).
template <typename T, int L, int R, int G, bool HALF, int NC, bool EX>
__device__ __forceinline__ void row_fwd_body(RowFwdArgs<T> a, int bx, int by, int gx, int tid) {
  constexpr int TT = L / R;
  __shared__ cx<T> lds[G * lds_len<1>(L)];
  constexpr int RI = HALF ? R / 2 : R;  // registers that can hold a sample x < nx
  const int g = row_group<TT>(tid);
  const int j = tid % TT;
  const int y = xcd_remap(bx, gx) * G + g;
  const bool rowok = y < a.ny;
  const int ny = a.ny, nx = a.nx;
  const int f0 = by * a.fpb;
  const int f1 = min(f0 + a.fpb, a.nfields);
  const TileRow<T, TT> tr(j, y, ny, a.tc_shift);
  const uint32_t row_vo = (uint32_t)((y * nx + j) * (int)sizeof(cx<T>));
  const uint32_t in_bytes = (uint32_t)(((int64_t)(NC - 1) * a.comp_stride + (int64_t)ny * nx) * sizeof(cx<T>));
  const uint32_t s_bytes = (uint32_t)(a.s_stride * sizeof(cx<T>));

  // Scalar modulation of this thread's pixels, shared by every field.
  const bool scalar_el = (a.el.flags & (EL_PHASE | EL_COMPLEX | EL_LENS)) != 0 || a.coh_m;
  cx<T> mod[RI];
#pragma unroll
  for (int m = 0; m < RI; ++m) {
    const int x = j + m * TT;
    mod[m] = {T(1), T(0)};
    if (a.coh_m) {
      if (rowok && (EX || x < nx)) mod[m] = cconj(a.coh_m[y * nx + x]);
    } else if (scalar_el && rowok && (EX || x < nx)) {
      mod[m] = scalar_modulation(a.el, ny, nx, y, x);
    }
    // one pixel at a time: interleaving the sincos chains only costs registers
    __builtin_amdgcn_sched_barrier(0);
  }

  // Loads of one field's row samples (zero outside the field).  Rows past
  // the field (ny not a multiple of G) still run the transforms, whose
  // barriers every wave must reach, on zeros, and store nothing.
  auto load_row = [&](int f, cx<T> (&dst)[NC][RI]) {
    const rsrc_t in_r = buf_rsrc(a.in + (int64_t)f * a.in_stride, in_bytes);
#pragma unroll
    for (int m = 0; m < RI; ++m) {
      const bool inside = rowok && (EX || j + m * TT < nx);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        cx<T> val = {T(0), T(0)};
        if (inside)
          val = buf_ld<T>(in_r, row_vo,
                          (uint32_t)((c * a.comp_stride + m * TT) * (int64_t)sizeof(cx<T>)));
        dst[c][m] = val;
      }
    }
  };
  // Software pipeline over the block's fields: the next field's loads are
  // issued before the current field's transform, so their latency overlaps
  // the FFT passes.
  cx<T> cur[NC][RI];
  if (f0 < f1) load_row(f0, cur);

#pragma unroll 1
  for (int f = f0; f < f1; ++f) {
    // Opaque copy of the thread index for the transforms: their twiddle
    // addresses are recomputed per field instead of being hoisted and kept
    // live across the loop.
    int jv = j;
    asm volatile("" : "+v"(jv));
    cx<T> nxt[NC][RI];
    if (f + 1 < f1) {
      load_row(f + 1, nxt);
    } else {
#pragma unroll
      for (int m = 0; m < RI; ++m)
#pragma unroll
        for (int c = 0; c < NC; ++c) nxt[c][m] = {T(0), T(0)};
    }
    cx<T> v[NC][R];
    const cx<T> fmod = a.coh_m ? a.coh_m[a.f_off + f] : cx<T>{T(1), T(0)};
#pragma unroll
    for (int m = 0; m < R; ++m) {
#pragma unroll
      for (int c = 0; c < NC; ++c) v[c][m] = m < RI ? cur[c][m] : cx<T>{T(0), T(0)};
      if (m < RI && a.coh_m) {
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c][m] = cmul(fmod, v[c][m]);
      }
      if (m < RI) {
        if constexpr (NC == 3) {
          if ((a.el.flags & (EL_JONES | EL_JONES_MAP)) && (EX || j + m * TT < nx)) {
            cx<T> w[3] = {v[0][m], v[1][m], v[2][m]};
            apply_jones(a.el, (int64_t)y * nx + (j + m * TT), w);
#pragma unroll
            for (int r = 0; r < 3; ++r) v[r][m] = w[r];
          }
        }
        if (scalar_el) {
#pragma unroll
          for (int c = 0; c < NC; ++c) v[c][m] = cmul(mod[m], v[c][m]);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      fft_wg<T, L, R, -1, HALF, 1>(v[c], jv, lds + g * lds_len<1>(L), a.tw);
      if (rowok) {
        const rsrc_t sr = buf_rsrc(a.scratch + (int64_t)(f * NC + c) * a.s_stride, s_bytes);
#pragma unroll
        for (int m = 0; m < R; ++m) buf_st(sr, tr.v(m), tr.s(m), v[c][m]);
      }
    }
#pragma unroll
    for (int m = 0; m < RI; ++m)
#pragma unroll
      for (int c = 0; c < NC; ++c) cur[c][m] = nxt[c][m];
  }
}

template <typename T, int L, int R, int G, bool HALF, int NC, bool EX>
__global__ void __launch_bounds__(G * (L / R))
    __attribute__((amdgpu_waves_per_eu(row_min_waves(NC, waves_per_simd(G * (L / R), row_lds_bytes<T, L, R, G, false>())),
                                       waves_per_simd(G * (L / R), row_lds_bytes<T, L, R, G, false>()))))
    row_fwd_kernel(RowFwdArgs<T> a) {
  row_fwd_body<T, L, R, G, HALF, NC, EX>(a, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, (int)threadIdx.x);
}

// ---------------------------------------------------------------------------
// col: forward FFT along y, transfer function, inverse FFT, crop rows.
// ---------------------------------------------------------------------------
// EX: the field's rows fill exactly the registers that can hold them
// (ny == R/2 TT on a half-padded column, ny == L otherwise), so y < ny is the
// compile-time m < R/2 (or always true).
// PF: the next field's column segment is loaded while the current one is
// transformed (software pipeline over the block's fields).
template <typename T, int L, int R, int TC, bool HALF, bool EX, bool PF>
__device__ __forceinline__ void col_body(ColArgs<T> a, int bx, int by, int gx, int tid) {
  constexpr int TT = L / R;
  __shared__ cx<T> lds[lds_len<TC>(L) * TC];
  const int c = tid % TC;
  const int j = tid / TC;
  // The scratch layout stores column tiles `tm` bins wide (a full cache line
  // per row segment); a block transforms `cpb` (<= TC) of them.  Blocks that
  // share a tile get consecutive logical indices, hence the same XCD and L2.
  const int lb = xcd_remap(bx, gx);
  const int tm = a.tm, cpb = a.cpb;
  const int per = tm / cpb;
  const int tile = lb / per, h = lb - tile * per;
  const int ny = a.ny;
  const int f_begin = by * a.fpc;
  const int f_end = min(f_begin + a.fpc, a.nfields);
  const bool active = c < cpb;

  // Transfer function at this thread's bins, formed once and applied to
  // every field of the block.  The split transform leaves frequency row
  // jf + m TT in register m.
  // (complex64 only, and not with the prefetching variant: there the extra
  // registers spill or halve the waves per SIMD)
  constexpr bool SPLIT = ColSplit<L, R, TC>::ok && !PF && sizeof(T) == 4;
  const int jf = SPLIT ? ColSplit<L, R, TC>::base(j) : j;
  __builtin_assume(jf >= 0 && jf < TT);
  const int kx = tile * tm + h * cpb + c;
  cx<T> hv[R];
  bool done = false;
  if constexpr (std::is_same<T, float>::value) {
    if (a.h.fast) {
      const int kxc = kx < a.lx ? kx : 0;
      const cx<float> exk = a.h.ex[kxc];
      const float sxk = a.h.sx[kxc];
      const float lam_fy_unit = (float)(sqrt(a.h.lam2) * a.h.inv_lydy);
#pragma unroll
      for (int m = 0; m < R; ++m) hv[m] = transfer_fast(exk, sxk, jf + m * TT, L, lam_fy_unit, a.h);
      done = true;
    }
  }
  if (!done && a.h.table) {
    // tabulated H (direct integration): one contiguous row segment of the
    // table per bin row
    const cx<T>* tab = static_cast<const cx<T>*>(a.h.table) + (active ? kx : 0);
#pragma unroll
    for (int m = 0; m < R; ++m) {
      cx<T> t = tab[(int64_t)(jf + m * TT) * a.lx];
      if (a.h.conj) t.y = -t.y;
      hv[m] = t;
    }
    done = true;
  }
  if (!done) {
#pragma unroll
    for (int m = 0; m < R; ++m) hv[m] = transfer_at<T>(kx, jf + m * TT, a.lx, L, a.h);
  }

  // Element (y, c) of the block's columns: lane part (j tm + c), uniform
  // part (tile ny tm + h cpb + m TT tm), in bytes from the field's scratch.
  const uint32_t s_bytes = (uint32_t)(a.s_stride * sizeof(cx<T>));
  const uint32_t col_vo = (uint32_t)((j * tm + c) * (int)sizeof(cx<T>));
  const uint32_t col_so = (uint32_t)(((int64_t)tile * ny * tm + h * cpb) * sizeof(cx<T>));
  const uint32_t m_so = (uint32_t)(TT * tm * (int)sizeof(cx<T>));
  auto kept = [&](int m) { return active && (EX ? (!HALF || m < R / 2) : ((!HALF || m < R / 2) && j + m * TT < ny)); };
  constexpr int RL = HALF ? R / 2 : R;  // registers that can hold a row y < ny
  auto load_col = [&](int f, cx<T> (&dst)[RL]) {
    const rsrc_t fr = buf_rsrc(a.scratch + (int64_t)f * a.s_stride, s_bytes);
#pragma unroll
    for (int m = 0; m < RL; ++m) {
      cx<T> val = {T(0), T(0)};
      if (kept(m)) val = buf_ld<T>(fr, col_vo, col_so + (uint32_t)m * m_so);
      dst[m] = val;
    }
  };
  cx<T> pre[PF ? RL : 1];
  if constexpr (PF) {
    if (f_begin < f_end) load_col(f_begin, pre);
  }
  for (int f = f_begin; f < f_end; ++f) {
    // Opaque per-field copy of j: the twiddle loads (addresses depend on j
    // only) are not hoisted out of the field loop, which would hold every
    // twiddle of both transforms in registers.
    int j1 = j;
    asm volatile("" : "+v"(j1));
    const rsrc_t fr = buf_rsrc(a.scratch + (int64_t)f * a.s_stride, s_bytes);
    cx<T> v[R];
    if constexpr (PF) {
#pragma unroll
      for (int m = 0; m < R; ++m) v[m] = m < RL ? pre[m < RL ? m : 0] : cx<T>{T(0), T(0)};
      if (f + 1 < f_end) load_col(f + 1, pre);
    } else {
      cx<T> cur[RL];
      load_col(f, cur);
#pragma unroll
      for (int m = 0; m < R; ++m) v[m] = m < RL ? cur[m < RL ? m : 0] : cx<T>{T(0), T(0)};
    }
    if constexpr (SPLIT)
      split_dif<T, L, R, -1, HALF, TC>(v, j1, lds + c, a.tw);
    else
      fft_wg<T, L, R, -1, HALF, TC>(v, j1, lds + c, a.tw);
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = cmul(v[m], hv[m]);
    // Opaque copy of j: the inverse transform reloads its twiddles instead
    // of keeping the forward transform's (same addresses) live across the
    // multiply.
    int j2 = j;
    asm volatile("" : "+v"(j2));
    if constexpr (SPLIT)
      split_dit<T, L, R, +1, false, TC>(v, j2, lds + c, a.tw);
    else
      fft_wg<T, L, R, +1, false, TC>(v, j2, lds + c, a.tw);
#pragma unroll
    for (int m = 0; m < R; ++m)
      if (kept(m)) buf_st(fr, col_vo, col_so + (uint32_t)m * m_so, v[m]);
  }
}

template <typename T, int L, int R, int TC, bool HALF, bool EX, bool PF>
__global__ void __launch_bounds__(TC * (L / R))
    __attribute__((amdgpu_waves_per_eu(PF ? waves_per_simd(TC * (L / R), lds_len<TC>(L) * TC * (int)sizeof(cx<T>)) : 1,
                                       waves_per_simd(TC * (L / R), lds_len<TC>(L) * TC * (int)sizeof(cx<T>)))))
    col_kernel(ColArgs<T> a) {
  col_body<T, L, R, TC, HALF, EX, PF>(a, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, (int)threadIdx.x);
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
template <typename T, int L, int R, int G, bool HALF, int NC, bool BWD, bool EX>
__device__ __forceinline__ void row_inv_body(RowInvArgs<T> a, int bx, int by, int gx, int tid) {
  constexpr bool kBwd = BWD;
  constexpr int TT = L / R;
  constexpr int NT = G * TT;
  constexpr int RO = HALF ? R / 2 : R;  // output registers that can hold x < nx
  constexpr uint32_t CB = sizeof(cx<T>), RB = sizeof(T);
  __shared__ cx<T> lds[G * lds_len<1>(L)];
  __shared__ double red[NT];
  const int g = row_group<TT>(tid);
  const int j = tid % TT;
  const int y = xcd_remap(bx, gx) * G + g;
  const int ny = a.ny, nx = a.nx;
  const bool rowok = y < ny;
  const TileRow<T, TT> tr(j, y, ny, a.tc_shift);
  const uint32_t s_bytes = (uint32_t)(a.s_stride * CB);
  const int64_t npix = (int64_t)ny * nx;
  // field-layout arrays: element m of this thread at lane offset (y nx + j)
  // plus the uniform m TT (+ c comp_stride)
  const uint32_t pix0 = (uint32_t)(y * nx + j);
  const uint32_t f_bytes = (uint32_t)(((int64_t)(NC - 1) * a.comp_stride + npix) * CB);
  const rsrc_t ref_r = buf_rsrc(a.epi_ref, (uint32_t)(npix * RB));
  auto xin = [&](int m) { return EX || j + m * TT < nx; };
  // Backward: one block owns its rows' parameter gradients, so it loops over
  // every field of the chunk; forward: `fpb` fields per block.
  const int f_begin = kBwd ? 0 : by * a.fpb;
  const int f_end = kBwd ? a.nfields : min(f_begin + a.fpb, a.nfields);
  // One field component's scratch row (tile layout); zeros past the field.
  auto load_row = [&](int f, int c, cx<T> (&dst)[R]) {
    const rsrc_t sr = buf_rsrc(a.scratch + (int64_t)(f * NC + c) * a.s_stride, s_bytes);
#pragma unroll
    for (int m = 0; m < R; ++m) {
      cx<T> val = {T(0), T(0)};
      if (rowok) val = buf_ld<T>(sr, tr.v(m), tr.s(m));
      dst[m] = val;
    }
  };
  // Scalar rows are software-pipelined: the next field's row is loaded
  // while the current one is transformed.
  constexpr bool kPipe = NC == 1;
  cx<T> pre[kPipe ? R : 1];
  if constexpr (kPipe) {
    if (f_begin < f_end) load_row(f_begin, 0, pre);
  }

  T gphase[RO];
  cx<T> modr[RO];  // backward: scalar modulation of this thread's pixels (all fields)
  double dpsi[RO];  // backward: d(lens phase)/df of this thread's pixels
#pragma unroll
  for (int m = 0; m < RO; ++m) {
    gphase[m] = T(0);
    modr[m] = {T(1), T(0)};
    dpsi[m] = 0.0;
    const int x = j + m * TT;
    if (kBwd && rowok && xin(m)) {
      if (a.el.flags & (EL_PHASE | EL_COMPLEX | EL_LENS)) modr[m] = scalar_modulation(a.el, ny, nx, y, x);
      if (a.el.flags & EL_LENS) dpsi[m] = lens_dphase_df(a.el, ny, nx, y, x, a.lens_f);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  double lens_acc = 0.0;

#pragma unroll 1
  for (int f = f_begin; f < f_end; ++f) {
    // Opaque copy of the thread index for the transforms (twiddle addresses
    // recomputed per field rather than hoisted).
    int jv = j;
    asm volatile("" : "+v"(jv));
    const rsrc_t out_r = buf_rsrc(a.out + (int64_t)f * a.out_stride, a.out ? f_bytes : 0u);
    const rsrc_t in_r = buf_rsrc(a.saved_in + (int64_t)f * a.out_stride, a.saved_in ? f_bytes : 0u);
    cx<T> v[NC][R];
    // backward, scalar rows: this field's layer input, loaded before the
    // transform so its latency overlaps it
    cx<T> uin[kBwd && kPipe ? RO : 1];
    if constexpr (kBwd && kPipe) {
      const bool want = (a.el.flags & (EL_PHASE | EL_LENS)) && a.saved_in && rowok;
#pragma unroll
      for (int m = 0; m < RO; ++m) {
        uin[m] = {T(0), T(0)};
        if (want && xin(m)) uin[m] = buf_ld<T>(in_r, pix0 * CB, (uint32_t)(m * TT) * CB);
      }
    }
    if constexpr (kPipe) {
#pragma unroll
      for (int m = 0; m < R; ++m) v[0][m] = pre[m];
      if (f + 1 < f_end) load_row(f + 1, 0, pre);
      fft_wg<T, L, R, +1, false, 1>(v[0], jv, lds + g * lds_len<1>(L), a.tw);
    } else {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        load_row(f, c, v[c]);
        fft_wg<T, L, R, +1, false, 1>(v[c], jv, lds + g * lds_len<1>(L), a.tw);
      }
    }
    double loss_acc = 0.0;
    if (rowok) {
      const rsrc_t grad_r = buf_rsrc(a.epi_grad + (int64_t)f * a.out_stride, a.epi_grad ? f_bytes : 0u);
      const rsrc_t eo_r = buf_rsrc(a.epi_out + (int64_t)f * npix, a.epi_out ? (uint32_t)(npix * RB) : 0u);
#pragma unroll
      for (int m = 0; m < RO; ++m) {
        if (!xin(m)) continue;
        const uint32_t so = (uint32_t)(m * TT);  // elements
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c][m] = cscale(v[c][m], a.scale);
        if constexpr (!kBwd) {
          if (a.epi == EPI_INTENSITY) {
            T I = T(0);
#pragma unroll
            for (int c = 0; c < NC; ++c) I += v[c][m].x * v[c][m].x + v[c][m].y * v[c][m].y;
            const T prev = buf_ldr(eo_r, pix0 * RB, so * RB, T());
            buf_str(eo_r, pix0 * RB, so * RB, prev + a.epi_scale * I);
          }
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const uint32_t oc = (uint32_t)((c * a.comp_stride + so) * CB);
            if (a.out) buf_st(out_r, pix0 * CB, oc, v[c][m]);
            if (a.epi == EPI_MSE) {
              const T I = v[c][m].x * v[c][m].x + v[c][m].y * v[c][m].y;
              const T d = I - buf_ldr(ref_r, pix0 * RB, so * RB, T());
              loss_acc += (double)d * (double)d;
              buf_st(grad_r, pix0 * CB, oc, cscale(v[c][m], T(4) * a.epi_scale * d));
            } else if (a.epi == EPI_WEIGHTED) {
              const T I = v[c][m].x * v[c][m].x + v[c][m].y * v[c][m].y;
              const T w = buf_ldr(ref_r, pix0 * RB, so * RB, T());
              loss_acc += (double)w * (double)I;
              buf_st(grad_r, pix0 * CB, oc, cscale(v[c][m], T(2) * a.epi_scale * w));
            }
          }
        } else {
          // g_mod is v; the modulated forward field is M u_in.
          const cx<T> mod = modr[m];
          const uint32_t fl = a.el.flags;
          const uint32_t pix = pix0 + so;
          if ((fl & (EL_PHASE | EL_LENS)) && a.saved_in) {
            cx<T> u[NC];
            if constexpr (kPipe) {
              u[0] = uin[m];
            } else {
#pragma unroll
              for (int c = 0; c < NC; ++c) u[c] = buf_ld<T>(in_r, pix0 * CB, (uint32_t)((c * a.comp_stride + so) * CB));
            }
            if constexpr (NC == 3) {
              if (fl & (EL_JONES | EL_JONES_MAP)) apply_jones(a.el, (int64_t)pix, u);
            }
            T im = T(0);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
              const cx<T> um = cmul(mod, u[c]);
              im += v[c][m].y * um.x - v[c][m].x * um.y;  // Im(g conj(um))
            }
            if (fl & EL_PHASE) gphase[m] += im;
            if (fl & EL_LENS) lens_acc += (double)im * dpsi[m];
          }
          if (a.out) {
            cx<T> gi[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) gi[c] = cmulc(v[c][m], mod);  // conj(M) g
            if constexpr (NC == 3) {
              if (fl & (EL_JONES | EL_JONES_MAP)) apply_jones_adjoint(a.el, (int64_t)pix, gi);  // J^H g
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) buf_st(out_r, pix0 * CB, (uint32_t)((c * a.comp_stride + so) * CB), gi[c]);
          }
        }
      }
    }
    if (!kBwd && (a.epi == EPI_MSE || a.epi == EPI_WEIGHTED)) {
      const double s = group_sum<TT, G>(loss_acc, red);
      if (rowok && j == 0) a.row_partial[(int64_t)f * ny + y] = s;
    }
  }
  if constexpr (kBwd) {
    if (rowok && (a.el.flags & EL_PHASE) && a.grad_phase && a.saved_in) {
#pragma unroll
      for (int m = 0; m < RO; ++m) {
        const int x = j + m * TT;
        if (xin(m)) a.grad_phase[(int64_t)y * nx + x] += gphase[m];
      }
    }
    if ((a.el.flags & EL_LENS) && a.lens_partial) {
      const double s = group_sum<TT, G>(lens_acc, red);
      if (rowok && j == 0) a.lens_partial[y] = s;
    }
  }
}

template <typename T, int L, int R, int G, bool HALF, int NC, bool BWD, bool EX>
__global__ void __launch_bounds__(G * (L / R))
    __attribute__((amdgpu_waves_per_eu(row_min_waves(NC, waves_per_simd(G * (L / R), row_lds_bytes<T, L, R, G, true>())),
                                       waves_per_simd(G * (L / R), row_lds_bytes<T, L, R, G, true>()))))
    row_inv_kernel(RowInvArgs<T> a) {
  row_inv_body<T, L, R, G, HALF, NC, BWD, EX>(a, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, (int)threadIdx.x);
}

// ---------------------------------------------------------------------------
// Job-queue launches.  One launch of a pass serves up to kQueueJobs
// independent propagations of one shape class (same padded lengths, pruning
// and kernel configuration; scalar fields, no element, no epilogue).  Each
// job contributes the workgroups of its own grid as items, numbered job
// after job; the launch holds at most as many workgroups as are resident at
// once, and each walks the items in strides of the grid size.  An item runs
// exactly the workgroup of the job's own launch at that block index, so the
// results equal those of the per-job launches bit for bit.  The job records
// travel in the kernel arguments: nothing is uploaded, and a launch captured
// in a graph carries its own copy.
// ---------------------------------------------------------------------------
constexpr int kQueueJobs = 16;

template <typename T>
struct QueueJob {
  const cx<T>* in;   // row_fwd: the field (or gradient) read
  cx<T>* out;        // row_inv: the field written (null: not formed)
  cx<T>* scratch;    // the job's padded intermediate, [field][LX/tm][ny][tm]
  int ny, nx;
  int nfields;
  int fpb;           // fields per workgroup of this pass (col: per column block)
  int first;         // first item; the job owns items first .. first + gx gy - 1
  int gx, gy;        // the job's grid of this pass
};

template <typename T>
struct QueueArgs {
  int njobs;
  int items;         // one past the last job's last item
  int lx;            // padded row length
  int tc_shift;      // log2 of the scratch tile width
  int tm, cpb;       // column pass: scratch tile width, columns per workgroup
  T scale;           // row_inv: 1 / (LX LY)
  const cx<T>* tw;   // twiddles of this pass's transform length
  QueueJob<T> job[kQueueJobs];
};

template <typename T>
struct ColQueueArgs {
  QueueArgs<T> q;
  TransferParams h[kQueueJobs];  // per job (adjoint: conj set)
};

// Runs body(k, bx, by, tid) for the items of this workgroup: blockIdx.x,
// blockIdx.x + gridDim.x, ...  Items in the alignment gap after a job's grid
// are skipped.  Every value involved is uniform over the workgroup.
template <typename T, typename F>
__device__ __forceinline__ void queue_walk(const QueueArgs<T>& q, F&& body) {
  int k = 0;
#pragma unroll 1
  for (int it = (int)blockIdx.x; it < q.items; it += (int)gridDim.x) {
    while (k + 1 < q.njobs && it >= q.job[k + 1].first) ++k;
    const int local = it - q.job[k].first;
    const int by = local / q.job[k].gx;
    if (by >= q.job[k].gy) continue;
    __syncthreads();  // the previous item's LDS reads are complete
    // The item's thread index, opaque to the compiler: what the body derives
    // from it is recomputed per item instead of being hoisted out of the
    // item loop and held in registers across it.
    int tid = (int)threadIdx.x;
    asm volatile("" : "+v"(tid));
    body(k, local - by * q.job[k].gx, by, tid);
  }
}

template <typename T, int L, int R, int G, bool HALF, bool EX>
__global__ void __launch_bounds__(G * (L / R))
    __attribute__((amdgpu_waves_per_eu(row_min_waves(1, waves_per_simd(G * (L / R), row_lds_bytes<T, L, R, G, false>())),
                                       waves_per_simd(G * (L / R), row_lds_bytes<T, L, R, G, false>()))))
    row_fwd_queue_kernel(QueueArgs<T> q) {
  queue_walk(q, [&](int k, int bx, int by, int tid) {
    const QueueJob<T>& jb = q.job[k];
    RowFwdArgs<T> a{};
    a.in = jb.in;
    a.scratch = jb.scratch;
    a.in_stride = (int64_t)jb.ny * jb.nx;
    a.comp_stride = a.in_stride;
    a.s_stride = (int64_t)q.lx * jb.ny;
    a.ny = jb.ny;
    a.nx = jb.nx;
    a.tc_shift = q.tc_shift;
    a.nfields = jb.nfields;
    a.fpb = jb.fpb;
    a.tw = q.tw;
    row_fwd_body<T, L, R, G, HALF, 1, EX>(a, bx, by, jb.gx, tid);
  });
}

template <typename T, int L, int R, int TC, bool HALF, bool EX, bool PF>
__global__ void __launch_bounds__(TC * (L / R))
    __attribute__((amdgpu_waves_per_eu(PF ? waves_per_simd(TC * (L / R), lds_len<TC>(L) * TC * (int)sizeof(cx<T>)) : 1,
                                       waves_per_simd(TC * (L / R), lds_len<TC>(L) * TC * (int)sizeof(cx<T>)))))
    col_queue_kernel(ColQueueArgs<T> cq) {
  const QueueArgs<T>& q = cq.q;
  queue_walk(q, [&](int k, int bx, int by, int tid) {
    const QueueJob<T>& jb = q.job[k];
    ColArgs<T> a;
    a.scratch = jb.scratch;
    a.s_stride = (int64_t)q.lx * jb.ny;
    a.ny = jb.ny;
    a.lx = q.lx;
    a.tm = q.tm;
    a.cpb = q.cpb;
    a.nfields = jb.nfields;
    a.fpc = jb.fpb;
    a.h = cq.h[k];
    a.tw = q.tw;
    col_body<T, L, R, TC, HALF, EX, PF>(a, bx, by, jb.gx, tid);
  });
}

template <typename T, int L, int R, int G, bool HALF, bool BWD, bool EX>
__global__ void __launch_bounds__(G * (L / R))
    __attribute__((amdgpu_waves_per_eu(row_min_waves(1, waves_per_simd(G * (L / R), row_lds_bytes<T, L, R, G, true>())),
                                       waves_per_simd(G * (L / R), row_lds_bytes<T, L, R, G, true>()))))
    row_inv_queue_kernel(QueueArgs<T> q) {
  queue_walk(q, [&](int k, int bx, int by, int tid) {
    const QueueJob<T>& jb = q.job[k];
    RowInvArgs<T> a{};
    a.scratch = jb.scratch;
    a.s_stride = (int64_t)q.lx * jb.ny;
    a.comp_stride = (int64_t)jb.ny * jb.nx;
    a.out = jb.out;
    a.out_stride = a.comp_stride;
    a.ny = jb.ny;
    a.nx = jb.nx;
    a.tc_shift = q.tc_shift;
    a.nfields = jb.nfields;
    a.scale = q.scale;
    a.tw = q.tw;
    a.epi = EPI_NONE;
    a.backward = BWD ? 1 : 0;
    a.fpb = jb.fpb;
    row_inv_body<T, L, R, G, HALF, 1, BWD, EX>(a, bx, by, jb.gx, tid);
  });
}

// ---------------------------------------------------------------------------
// row_mid: the boundary between two propagations of a chain (the output of
// one layer is the input of the next), fused: per row, the inverse FFT of
// the finished layer, crop and 1/(LX LY) scale, store of that layer's
// output, the next layer's element, the forward FFT of the next layer, back
// into the same scratch row.  Equal to row_inv followed by row_fwd (bit for
// bit where both take the same factorisation: not for complex64 rows that
// take the split transforms here).
// ---------------------------------------------------------------------------
template <typename T>
struct RowMidArgs {
  cx<T>* scratch;       // the chunk's intermediate, read and rewritten in place
  int64_t s_stride;
  cx<T>* out;           // the finished layer's output (first field of the chunk)
  int64_t out_stride;   // elements between fields of `out`
  int ny, nx;
  int tc_shift;
  int nfields;
  int fpb;              // fields per block (the element is evaluated once for them)
  T scale;              // 1 / (LX LY)
  ElementParams<T> el;  // element in front of the next layer
  const cx<T>* tw;
};

template <typename T, int L, int R, int G, bool HALF, bool EX>
__global__ void __launch_bounds__(G * (L / R))
    __attribute__((amdgpu_waves_per_eu(row_min_waves(1, waves_per_simd(G * (L / R), row_lds_bytes<T, L, R, G, false>())),
                                       waves_per_simd(G * (L / R), row_lds_bytes<T, L, R, G, false>()))))
    row_mid_kernel(RowMidArgs<T> a) {
  constexpr int TT = L / R;
  constexpr int RO = HALF ? R / 2 : R;  // registers that can hold x < nx
  constexpr uint32_t CB = sizeof(cx<T>);
  __shared__ cx<T> lds[G * lds_len<1>(L)];
  const int g = row_group<TT>();
  const int j = threadIdx.x % TT;
  // Split transforms (complex64): the inverse leaves pixel xj + m TT in
  // register m and the forward takes that order back to natural order.
  constexpr bool SPLIT = RowSplit<L, R>::ok && sizeof(T) == 4;
  const int xj = SPLIT ? RowSplit<L, R>::base(j) : j;
  const int y = xcd_remap((int)blockIdx.x, (int)gridDim.x) * G + g;
  const int ny = a.ny, nx = a.nx;
  const bool rowok = y < ny;
  const int f_begin = (int)blockIdx.y * a.fpb;
  const int f_end = min(f_begin + a.fpb, a.nfields);
  const TileRow<T, TT> tr(j, y, ny, a.tc_shift);
  const uint32_t s_bytes = (uint32_t)(a.s_stride * CB);
  const uint32_t o_bytes = (uint32_t)((int64_t)ny * nx * CB);
  const uint32_t pix0 = (uint32_t)(y * nx + xj);
  auto xin = [&](int m) { return EX || xj + m * TT < nx; };

  const bool scalar_el = (a.el.flags & (EL_PHASE | EL_COMPLEX | EL_LENS)) != 0;
  cx<T> mod[RO];
#pragma unroll
  for (int m = 0; m < RO; ++m) {
    const int x = xj + m * TT;
    mod[m] = {T(1), T(0)};
    if (scalar_el && rowok && xin(m)) mod[m] = scalar_modulation(a.el, ny, nx, y, x);
    __builtin_amdgcn_sched_barrier(0);
  }
  auto load_row = [&](int f, cx<T> (&dst)[R]) {
    const rsrc_t sr = buf_rsrc(a.scratch + (int64_t)f * a.s_stride, s_bytes);
#pragma unroll
    for (int m = 0; m < R; ++m) {
      cx<T> val = {T(0), T(0)};
      if (rowok) val = buf_ld<T>(sr, tr.v(m), tr.s(m));
      dst[m] = val;
    }
  };
  // The next field's row is loaded while the current one is transformed
  // (not with the split transforms: their registers leave no room for it).
  constexpr bool kPipe = !SPLIT;
  cx<T> pre[kPipe ? R : 1];
  if constexpr (kPipe) {
    if (f_begin < f_end) load_row(f_begin, pre);
  }

#pragma unroll 1
  for (int f = f_begin; f < f_end; ++f) {
    int jv = j;
    asm volatile("" : "+v"(jv));
    cx<T> v[R];
    if constexpr (kPipe) {
#pragma unroll
      for (int m = 0; m < R; ++m) v[m] = pre[m];
      if (f + 1 < f_end) load_row(f + 1, pre);
    } else {
      load_row(f, v);
    }
    if constexpr (SPLIT)
      split_dif<T, L, R, +1, false, -1>(v, jv, lds + g * lds_len<1>(L), a.tw);
    else
      fft_wg<T, L, R, +1, false, 1>(v, jv, lds + g * lds_len<1>(L), a.tw);
    const rsrc_t out_r = buf_rsrc(a.out + (int64_t)f * a.out_stride, o_bytes);
#pragma unroll
    for (int m = 0; m < R; ++m) {
      if (m < RO && rowok && xin(m)) {
        v[m] = cscale(v[m], a.scale);
        buf_st(out_r, pix0 * CB, (uint32_t)(m * TT) * CB, v[m]);
        if (scalar_el) v[m] = cmul(mod[m], v[m]);
      } else {
        v[m] = {T(0), T(0)};
      }
    }
    // fresh opaque index: the forward transform reloads its twiddles rather
    // than keeping the inverse transform's (same addresses) live
    int jw = jv;
    asm volatile("" : "+v"(jw));
    if constexpr (SPLIT)
      split_dit<T, L, R, -1, HALF, -1>(v, jw, lds + g * lds_len<1>(L), a.tw);
    else
      fft_wg<T, L, R, -1, HALF, 1>(v, jw, lds + g * lds_len<1>(L), a.tw);
    if (rowok) {
      const rsrc_t sr = buf_rsrc(a.scratch + (int64_t)f * a.s_stride, s_bytes);
#pragma unroll
      for (int m = 0; m < R; ++m) buf_st(sr, tr.v(m), tr.s(m), v[m]);
    }
  }
}

// ---------------------------------------------------------------------------
// row_mid_bwd: the same boundary in the backward pass of a chain.  Per row:
// inverse FFT of g_mod = P^H g of layer l, crop and scale, the layer's
// parameter gradients, g_l = M^H g_mod (stored when requested), which is the
// upstream gradient of layer l-1, then the forward FFT of g_l back into the
// scratch row.  Like row_inv's backward, a block loops over its fields so each pixel's gradient is summed by one thread in a fixed
// order.  A block takes `fpb` fields (a field group); with several groups
// each writes its own gradient partials, combined afterwards in group order.
// ---------------------------------------------------------------------------
template <typename T>
struct RowMidBwdArgs {
  cx<T>* scratch;
  int64_t s_stride;
  cx<T>* grad_in;         // g_l (first field of the chunk), or null
  const cx<T>* saved_in;  // the layer's forward input, or null (no parameter gradients)
  int64_t stride;         // elements between fields of grad_in / saved_in
  int ny, nx;
  int tc_shift;
  int nfields;
  T scale;
  ElementParams<T> el;    // layer l's element
  int fpb;                // fields per block (a field group)
  T* grad_phase;          // [ny][nx], accumulated, or null
  T* gphase_part;         // several field groups: [group][ny][nx] partials (overwritten)
  double lens_f;
  double* lens_partial;   // per (field group, row) partial sums of dL/df, or null
  const cx<T>* tw;
};

template <typename T, int L, int R, int G, bool HALF, bool EX>
__global__ void __launch_bounds__(G * (L / R))
    __attribute__((amdgpu_waves_per_eu(row_min_waves(1, waves_per_simd(G * (L / R), row_lds_bytes<T, L, R, G, true>())),
                                       waves_per_simd(G * (L / R), row_lds_bytes<T, L, R, G, true>()))))
    row_mid_bwd_kernel(RowMidBwdArgs<T> a) {
  constexpr int TT = L / R;
  constexpr int NT = G * TT;
  constexpr int RO = HALF ? R / 2 : R;
  constexpr uint32_t CB = sizeof(cx<T>);
  __shared__ cx<T> lds[G * lds_len<1>(L)];
  __shared__ double red[NT];
  const int g = row_group<TT>();
  const int j = threadIdx.x % TT;
  // Split transforms (complex64): the inverse leaves pixel xj + m TT in
  // register m and the forward takes that order back to natural order.
  // (not at 8192 points, where the split's registers spill)
  constexpr bool SPLIT = RowSplit<L, R>::ok && sizeof(T) == 4 && L <= 4096;
  const int xj = SPLIT ? RowSplit<L, R>::base(j) : j;
  const int y = xcd_remap((int)blockIdx.x, (int)gridDim.x) * G + g;
  const int ny = a.ny, nx = a.nx;
  const bool rowok = y < ny;
  const uint32_t fl = a.el.flags;
  const bool want_param = (fl & (EL_PHASE | EL_LENS)) && a.saved_in;
  const TileRow<T, TT> tr(j, y, ny, a.tc_shift);
  const uint32_t s_bytes = (uint32_t)(a.s_stride * CB);
  const uint32_t f_bytes = (uint32_t)((int64_t)ny * nx * CB);
  const uint32_t pix0 = (uint32_t)(y * nx + xj);
  auto xin = [&](int m) { return EX || xj + m * TT < nx; };

  T gphase[RO];
  cx<T> modr[RO];
#pragma unroll
  for (int m = 0; m < RO; ++m) {
    gphase[m] = T(0);
    modr[m] = {T(1), T(0)};
    const int x = xj + m * TT;
    if (rowok && xin(m)) {
      if (fl & (EL_PHASE | EL_COMPLEX | EL_LENS)) modr[m] = scalar_modulation(a.el, ny, nx, y, x);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  double lens_acc = 0.0;
  auto load_row = [&](int f, cx<T> (&dst)[R]) {
    const rsrc_t sr = buf_rsrc(a.scratch + (int64_t)f * a.s_stride, s_bytes);
#pragma unroll
    for (int m = 0; m < R; ++m) {
      cx<T> val = {T(0), T(0)};
      if (rowok) val = buf_ld<T>(sr, tr.v(m), tr.s(m));
      dst[m] = val;
    }
  };
  const int f_begin = (int)blockIdx.y * a.fpb;
  const int f_end = min(f_begin + a.fpb, a.nfields);
  // With 8 points per thread the next field's row is loaded while the
  // current one is transformed; with 16 (and the layer input, modulation
  // and gradient registers this pass holds) the row is loaded at the top of
  // its iteration, which keeps the kernel within 128 registers.
  constexpr bool kPipe = R <= 8;
  cx<T> pre[kPipe ? R : 1];
  if constexpr (kPipe) {
    if (f_begin < f_end) load_row(f_begin, pre);
  }

#pragma unroll 1
  for (int f = f_begin; f < f_end; ++f) {
    int jv = j;
    asm volatile("" : "+v"(jv));
    cx<T> v[R];
    if constexpr (kPipe) {
#pragma unroll
      for (int m = 0; m < R; ++m) v[m] = pre[m];
      if (f + 1 < f_end) load_row(f + 1, pre);
    } else {
      load_row(f, v);
    }
    // the layer input of this field's row, loaded before the transform so
    // its latency overlaps it
    const rsrc_t in_r = buf_rsrc(a.saved_in + (int64_t)f * a.stride, a.saved_in ? f_bytes : 0u);
    const rsrc_t gi_r = buf_rsrc(a.grad_in + (int64_t)f * a.stride, a.grad_in ? f_bytes : 0u);
    cx<T> uin[RO];
#pragma unroll
    for (int m = 0; m < RO; ++m) {
      uin[m] = {T(0), T(0)};
      if (want_param && rowok && xin(m)) uin[m] = buf_ld<T>(in_r, pix0 * CB, (uint32_t)(m * TT) * CB);
    }
    if constexpr (SPLIT)
      split_dif<T, L, R, +1, false, -1>(v, jv, lds + g * lds_len<1>(L), a.tw);
    else
      fft_wg<T, L, R, +1, false, 1>(v, jv, lds + g * lds_len<1>(L), a.tw);
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int x = xj + m * TT;
      if (m < RO && rowok && xin(m)) {
        v[m] = cscale(v[m], a.scale);  // g_mod
        const cx<T> mod = modr[m];
        if (want_param) {
          const cx<T> um = cmul(mod, uin[m]);
          const T im = v[m].y * um.x - v[m].x * um.y;  // Im(g conj(M u))
          if (fl & EL_PHASE) gphase[m] += im;
          // d(lens phase)/df, formed where needed (lens layers are rare)
          if (fl & EL_LENS) lens_acc += (double)im * lens_dphase_df(a.el, ny, nx, y, x, a.lens_f);
        }
        v[m] = cmulc(v[m], mod);  // g_l = conj(M) g_mod
        if (a.grad_in) buf_st(gi_r, pix0 * CB, (uint32_t)(m * TT) * CB, v[m]);
      } else {
        v[m] = {T(0), T(0)};
      }
    }
    // fresh opaque index: the forward transform reloads its twiddles rather
    // than keeping the inverse transform's (same addresses) live
    int jw = jv;
    asm volatile("" : "+v"(jw));
    if constexpr (SPLIT)
      split_dit<T, L, R, -1, HALF, -1>(v, jw, lds + g * lds_len<1>(L), a.tw);
    else
      fft_wg<T, L, R, -1, HALF, 1>(v, jw, lds + g * lds_len<1>(L), a.tw);
    if (rowok) {
      const rsrc_t sr = buf_rsrc(a.scratch + (int64_t)f * a.s_stride, s_bytes);
#pragma unroll
      for (int m = 0; m < R; ++m) buf_st(sr, tr.v(m), tr.s(m), v[m]);
    }
  }
  if (rowok && (fl & EL_PHASE) && a.grad_phase && a.saved_in) {
#pragma unroll
    for (int m = 0; m < RO; ++m) {
      const int x = xj + m * TT;
      if (xin(m)) {
        if (a.gphase_part)
          a.gphase_part[((int64_t)blockIdx.y * ny + y) * nx + x] = gphase[m];
        else
          a.grad_phase[(int64_t)y * nx + x] += gphase[m];
      }
    }
  }
  if ((fl & EL_LENS) && a.lens_partial) {
    const double s = group_sum<TT, G>(lens_acc, red);
    if (rowok && j == 0) a.lens_partial[(int64_t)blockIdx.y * ny + y] = s;
  }
}

// dst[i] += sum over g of part[g][i], g in order (deterministic combine of
// per-field-group gradient partials).
template <typename T>
__global__ void __launch_bounds__(256) sum_parts_kernel(const T* __restrict__ part, int groups, int64_t n,
                                                        T* __restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    T acc = part[i];
    for (int g = 1; g < groups; ++g) acc += part[(int64_t)g * n + i];
    dst[i] += acc;
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
        if (el.flags & (EL_JONES | EL_JONES_MAP)) apply_jones(el, pix, v);
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) v[c] = cmul(mod, v[c]);
    } else {
#pragma unroll
      for (int c = 0; c < NC; ++c) v[c] = cmul(mod, v[c]);
      if constexpr (NC == 3) {
        if (el.flags & (EL_JONES | EL_JONES_MAP)) apply_jones_adjoint(el, pix, v);
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) out[f * fstride + c * cstride + pix] = v[c];
  }
}

}  // namespace toprop
