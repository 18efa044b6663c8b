// Transforms of lines whose length is not a power of two but factors into
// 2, 3, 5 and 7 (the paper's padded grids: 2000 = 16 * 5^3, 500, 100): a
// mixed-radix Stockham FFT held in LDS, used by the plain pipeline in place
// of Bluestein's transform for such lengths.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft.hpp"
#include "kernels.hpp"

namespace toprop {

constexpr int kMixedMaxPasses = 12;  // 4096 = 2^12 is the longest line

// Radices of the passes of one length, first pass first.  np == 0: the
// length is not transformed this way.
struct MixedPlan {
  int np;
  int r[kMixedMaxPasses];
};

// The plan of L = 2^a 3^b 5^c 7^d (L <= 4096): the power-of-two part in
// passes of 16 (the remainder as 8, 4 or 2; 16 * 2 as 8 * 4), then the
// radix-5, 3 and 7 passes.  Returns false (np = 0) for any other length,
// and for powers of two unless `pow2` is set.
bool mixed_plan(int L, MixedPlan* p, bool pow2 = false);

// One launch over `nlines` lines of length L.  Line i is read from
// in + i * in_ls (element q < nin at in[q * in_es], zeros beyond: the zero
// padding) and written, elements q < nout times `scale` (the crop), to
// out + i * out_ls (out[q * out_es]); in == out with equal strides is in
// place.  With a transfer table h (the convolution mode), the forward
// transform of line i is multiplied by h[(i mod h_lines) * h_ls + k]
// (conjugated if `conj`) and transformed back.  A forward launch applies the
// element `el` (phase mask, complex mask, lens; flags 0: none) to the field
// it reads, taking line i as row i mod field_rows of a field_rows x nin
// field (batches of fields are consecutive lines).  h_lines and field_rows
// of 0 mean nlines.
template <typename T>
struct MixedArgs {
  const cx<T>* in;
  cx<T>* out;
  const cx<T>* h;
  int64_t in_ls, in_es, out_ls, out_es, h_ls;
  int nin, nout, conj, nlines, L, tl_shift, h_lines, field_rows;
  T scale;
  MixedPlan plan;
  const cx<T>* tw;  // exp(-2 pi i m / L), m < L
  ElementParams<T> el;
  // hcalc: the convolution mode forms the transfer function itself,
  // transfer_at(line mod h_lines, k, h_lines, L, tp) (conjugated by tp.conj),
  // instead of reading h
  int hcalc;
  TransferParams tp;
};

template <typename T>
struct Mixed {
  // tw[m] = exp(-2 pi i m / L), m < L, on `s` (phases reduced exactly in
  // integers, evaluated in FP64).
  static hipError_t twiddles(int L, cx<T>* tw, hipStream_t s);
  // In-place DFTs (dir -1 forward, +1 inverse, unnormalised) of `nlines`
  // lines of length L: element q of line i is a[i * lstride + q * estride].
  static hipError_t lines(int L, const MixedPlan& p, const cx<T>* tw, cx<T>* a, int nlines, int64_t lstride,
                          int64_t estride, int dir, hipStream_t s);
  // mode -1 / +1: forward / inverse transforms; 0: the convolution mode.
  static hipError_t launch(MixedArgs<T> a, int mode, hipStream_t s);
  // out[b][c][r] = in[b][r][c] for `batch` row-major rows x cols arrays.
  static hipError_t transpose(const cx<T>* in, cx<T>* out, int rows, int cols, int64_t batch, hipStream_t s);
};

}  // namespace toprop
