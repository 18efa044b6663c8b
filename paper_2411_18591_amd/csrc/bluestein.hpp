// Transforms of lines whose length is not a power of two (Bluestein's
// chirp-z method on power-of-two FFTs), used by the plain pipeline for
// padded grids of any extent.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "mixed.hpp"

namespace toprop {

// How the lines of one length are transformed.
template <typename T>
struct LineFft {
  int L;            // transform length
  int M;            // 0: L is a power of two or mixed-radix; else the convolution length (power of two >= 2L - 1)
  const cx<T>* tw;  // twiddles of length L (power of two or mixed-radix) or M
  const cx<T>* w;   // chirp exp(i pi n^2 / L), n < L (Bluestein only)
  const cx<T>* Bf;  // length-M DFT of the chirp kernel (Bluestein only)
  MixedPlan mp;     // mp.np > 0: L = 2^a 3^b 5^c 7^d, transformed by the mixed-radix passes
};

template <typename T>
struct Bluestein {
  // Chirp w[0..L) and the kernel's DFT Bf[0..M) (in place in Bf), on `s`.
  static hipError_t build(int L, int M, cx<T>* w, cx<T>* Bf, const cx<T>* twM, hipStream_t s);
  // In-place DFTs (dir -1 forward, +1 inverse, unnormalised) of `nrows`
  // contiguous rows of length f.L, or of the f.L-long columns of a
  // row-major [f.L][lx] array.
  static hipError_t rows(const LineFft<T>& f, cx<T>* a, int nrows, int dir, hipStream_t s);
  static hipError_t cols(const LineFft<T>& f, cx<T>* a, int lx, int dir, hipStream_t s);
  // out[c][r] = in[r][c] for a row-major rows x cols array.
  static hipError_t transpose(const cx<T>* in, cx<T>* out, int rows, int cols, hipStream_t s);
};

}  // namespace toprop
