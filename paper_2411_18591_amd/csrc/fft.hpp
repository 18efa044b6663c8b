// Device-side building blocks of the Stockham FFT used by the propagation
// kernels: a complex type, small in-register DFTs (radix 2..32) with
// compile-time twiddles, and the generic register/LDS Stockham pass.
//
// Conventions: forward transform X[k] = sum_n x[n] exp(-2 pi i n k / L)
// (direction D = -1), inverse without scaling (D = +1).  A transform of
// length L is owned by T = L / R threads; between passes thread j holds
// the elements at positions j + m*T, m < R ("strided ownership"), which is
// also the coalesced order for global loads and stores.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace toprop {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) { return {a.x, -a.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.x * s, a.y * s}; }

// cos(2 pi k / 64) for k = 0..16 (first quadrant), 40 significant digits.
__device__ constexpr long double kCos64[17] = {
    1.0000000000000000000000000000000000000000L, 0.9951847266721968862448369531094799215755L,
    0.9807852804032304491261822361342390369739L, 0.9569403357322088649357978869802699694828L,
    0.9238795325112867561281831893967882868224L, 0.8819212643483550297127568636603883495084L,
    0.8314696123025452370787883776179057567386L, 0.7730104533627369608109066097584698009710L,
    0.7071067811865475244008443621048490392848L, 0.6343932841636454982151716132254933706757L,
    0.5555702330196022247428308139485328743749L, 0.4713967368259976485563876259052543776575L,
    0.3826834323650897717284599840303988667613L, 0.2902846772544623676361923758173952746915L,
    0.1950903220161282678482848684770222409277L, 0.0980171403295606019941955638886418458611L,
    0.0000000000000000000000000000000000000000L};

// cos and sin of 2 pi k / N for N dividing 64, evaluated at compile time.
constexpr long double cos64(int i) {
  // i in [0, 64): reduce by quadrant symmetry to the table
  return (i <= 16)   ? kCos64[i]
         : (i <= 32) ? -kCos64[32 - i]
         : (i <= 48) ? -kCos64[i - 32]
                     : kCos64[64 - i];
}
template <int N, int K>
constexpr long double twc() { return cos64(((K % N) * (64 / N)) % 64); }
template <int N, int K>
constexpr long double tws() { return cos64(((K % N) * (64 / N) + 48) % 64); }  // sin x = cos(x - pi/2)

// v * exp(D * 2 pi i K / N), with the trivial angles done by swaps/negations.
template <int N, int K, int D, typename T>
__device__ __forceinline__ cx<T> rot(cx<T> v) {
  constexpr int k = ((K % N) + N) % N;
  if constexpr (k == 0) {
    return v;
  } else if constexpr (2 * k == N) {
    return {-v.x, -v.y};
  } else if constexpr (4 * k == N) {  // exp(D i pi/2) = D i
    return (D > 0) ? cx<T>{-v.y, v.x} : cx<T>{v.y, -v.x};
  } else if constexpr (4 * k == 3 * N) {  // exp(D i 3pi/2) = -D i
    return (D > 0) ? cx<T>{v.y, -v.x} : cx<T>{-v.y, v.x};
  } else if constexpr (8 * k == N || 8 * k == 3 * N || 8 * k == 5 * N || 8 * k == 7 * N) {
    // (+-1 +- i)/sqrt(2): two adds and two multiplies
    constexpr T s = (T)0.7071067811865475244008443621048490392848L;
    constexpr int sc = (8 * k == N || 8 * k == 7 * N) ? 1 : -1;   // sign of cos
    constexpr int ss = ((8 * k == N || 8 * k == 3 * N) ? 1 : -1) * D;  // sign of sin
    T re = (sc > 0 ? v.x : -v.x) - (ss > 0 ? v.y : -v.y);
    T im = (sc > 0 ? v.y : -v.y) + (ss > 0 ? v.x : -v.x);
    return {re * s, im * s};
  } else {
    constexpr T c = (T)twc<N, k>();
    constexpr T s = (T)(D * tws<N, k>());
    return {v.x * c - v.y * s, v.x * s + v.y * c};
  }
}

// In-register DFT of N points (N a power of two <= 32), natural order in
// and out, decimation in time.
template <int N, int D, typename T>
struct Dft {
  __device__ __forceinline__ static void run(cx<T>* v) {
    if constexpr (N == 1) {
      return;
    } else if constexpr (N == 2) {
      cx<T> a = v[0], b = v[1];
      v[0] = cadd(a, b);
      v[1] = csub(a, b);
    } else {
      cx<T> e[N / 2], o[N / 2];
#pragma unroll
      for (int k = 0; k < N / 2; ++k) {
        e[k] = v[2 * k];
        o[k] = v[2 * k + 1];
      }
      Dft<N / 2, D, T>::run(e);
      Dft<N / 2, D, T>::run(o);
      combine(e, o, v, std::integral_constant<int, 0>());
    }
  }
  template <int K>
  __device__ __forceinline__ static void combine(const cx<T>* e, const cx<T>* o, cx<T>* v,
                                                 std::integral_constant<int, K>) {
    if constexpr (K < N / 2) {
      cx<T> t = rot<N, K, D>(o[K]);
      v[K] = cadd(e[K], t);
      v[K + N / 2] = csub(e[K], t);
      combine(e, o, v, std::integral_constant<int, K + 1>());
    }
  }
};

// DFT of N points whose upper half v[N/2..N-1] is zero (zero-padded input):
// X[2m] = DFT_{N/2}(x)[m],  X[2m+1] = DFT_{N/2}(x[n] w_N^n)[m].
template <int N, int D, typename T>
struct DftHalfZero {
  __device__ __forceinline__ static void run(cx<T>* v) {
    if constexpr (N == 1) {
      return;
    } else if constexpr (N == 2) {
      v[1] = v[0];
    } else {
      cx<T> a[N / 2], b[N / 2];
#pragma unroll
      for (int k = 0; k < N / 2; ++k) a[k] = v[k];
      twiddle(a, b, std::integral_constant<int, 0>());
      Dft<N / 2, D, T>::run(a);
      Dft<N / 2, D, T>::run(b);
#pragma unroll
      for (int k = 0; k < N / 2; ++k) {
        v[2 * k] = a[k];
        v[2 * k + 1] = b[k];
      }
    }
  }
  template <int K>
  __device__ __forceinline__ static void twiddle(const cx<T>* a, cx<T>* b,
                                                 std::integral_constant<int, K>) {
    if constexpr (K < N / 2) {
      b[K] = rot<N, K, D>(a[K]);
      twiddle(a, b, std::integral_constant<int, K + 1>());
    }
  }
};

// ---------------------------------------------------------------------------
// Raw buffer access.  A buffer resource holds a wave-uniform base address
// and size in scalar registers; each access adds a per-lane byte offset
// (voff) and a wave-uniform byte offset (soff).  Strided register sets
// (element m at soff = m * stride) then cost no vector instructions for
// their addresses.  Word 3 is the gfx9 descriptor word for untyped access
// (32-bit data format).  The base must be wave-uniform and both offsets
// must stay below 2^32 and within `bytes`.
// ---------------------------------------------------------------------------
using rsrc_t = __amdgpu_buffer_rsrc_t;

__device__ __forceinline__ rsrc_t buf_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ cx<float> buf_ld(rsrc_t r, uint32_t voff, uint32_t soff, float) {
  return __builtin_bit_cast(cx<float>, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ cx<double> buf_ld(rsrc_t r, uint32_t voff, uint32_t soff, double) {
  return __builtin_bit_cast(cx<double>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
template <typename T>
__device__ __forceinline__ cx<T> buf_ld(rsrc_t r, uint32_t voff, uint32_t soff) {
  return buf_ld(r, voff, soff, T());
}
__device__ __forceinline__ void buf_st(rsrc_t r, uint32_t voff, uint32_t soff, cx<float> v) {
  using V = unsigned int __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, voff, soff, 0);
}
// A complex128 element is stored as two 64-bit halves.  A buffer store of
// more than 64 bits whose offset is a scalar register can still be reading
// its data registers when the next instruction overwrites them (seen on
// gfx950 as wrong values in lanes 12-15 of every 16-lane group, only under
// load), and the compiler inserts no wait state for that form; a 64-bit
// store reads its data at issue.
__device__ __forceinline__ void buf_st(rsrc_t r, uint32_t voff, uint32_t soff, cx<double> v) {
  using V = unsigned int __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v.x), r, voff, soff, 0);
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v.y), r, voff, soff + 8u, 0);
}
// Real scalars (masks, targets, weights, gradients).
__device__ __forceinline__ void buf_str(rsrc_t r, uint32_t voff, uint32_t soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, voff, soff, 0);
}
__device__ __forceinline__ void buf_str(rsrc_t r, uint32_t voff, uint32_t soff, double v) {
  using V = unsigned int __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, voff, soff, 0);
}
__device__ __forceinline__ float buf_ldr(rsrc_t r, uint32_t voff, uint32_t soff, float) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ double buf_ldr(rsrc_t r, uint32_t voff, uint32_t soff, double) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

// ---------------------------------------------------------------------------
// Pass schedule.  A length-L transform with R points per thread runs passes
// of radix R while they fit, and one final pass of the remaining radix.
// ---------------------------------------------------------------------------
constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n / 2); }

template <int L, int R>
struct Schedule {
  static constexpr int T = L / R;  // threads per transform
  static constexpr int full = ilog2c(L) / ilog2c(R);           // passes of radix R
  static constexpr int rem = 1 << (ilog2c(L) - full * ilog2c(R));  // last radix (1 = none)
  static constexpr int npass = full + (rem > 1 ? 1 : 0);
  static constexpr int radix(int p) { return p < full ? R : rem; }
  static constexpr int ns(int p) {  // product of the radices before pass p
    int n = 1;
    for (int q = 0; q < p; ++q) n *= radix(q);
    return n;
  }
};

// Butterflies of one Stockham pass on the registers of one thread.
// Butterfly t (t < R/RP) of thread j has global index b = j + t*T and uses
// registers m = t + i*(R/RP), i < RP, which hold X[b + i*L/RP].  Twiddles
// w_L^{i * (b mod NS) * L/(NS*RP)} come from `tw` (exp(-2 pi i m/L), m < L;
// conjugated for the inverse).  FIRST_HALF_ZERO: registers m >= R/2 are
// known to be zero (only valid for the first pass, NS == 1).
template <typename T, int L, int R, int RP, int NS, int D, bool FIRST_HALF_ZERO>
__device__ __forceinline__ void stockham_butterflies(cx<T>* v, int j, const cx<T>* __restrict__ tw) {
  constexpr int TT = L / R;
  constexpr int NB = R / RP;
  const rsrc_t twr = buf_rsrc(tw, (uint32_t)(L * sizeof(cx<T>)));
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    cx<T> u[RP];
#pragma unroll
    for (int i = 0; i < RP; ++i) u[i] = v[t + i * NB];
    if constexpr (NS > 1) {
      const int b = j + t * TT;
      const int k = b % NS;
      constexpr int step = L / (NS * RP);
#pragma unroll
      for (int i = 1; i < RP; ++i) {
        // twiddle index i k step < L; byte offset k * (i step size), both
        // factors below 2^24 (one full-rate 24-bit multiply)
        cx<T> w = buf_ld<T>(twr, __umul24((uint32_t)k, (uint32_t)(i * step * sizeof(cx<T>))), 0u);
        if (D > 0) w.y = -w.y;
        u[i] = cmul(u[i], w);
      }
    }
    if constexpr (FIRST_HALF_ZERO && NS == 1 && NB == 1)
      DftHalfZero<RP, D, T>::run(u);
    else
      Dft<RP, D, T>::run(u);
#pragma unroll
    for (int i = 0; i < RP; ++i) v[t + i * NB] = u[i];
  }
}

// Position in the transform of output i of butterfly t after a pass with
// product NS: (b / NS) * NS * RP + (b mod NS) + i * NS.
template <int L, int R, int RP, int NS>
__device__ __forceinline__ int stockham_out_pos(int j, int t, int i) {
  constexpr int TT = L / R;
  const int b = j + t * TT;
  return (b / NS) * NS * RP + (b % NS) + i * NS;
}

}  // namespace toprop
