// Host interface of the coherence-propagation helper kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace toprop {

// Row chunks of the column sums of the mask gradient (partials summed in
// chunk order: deterministic).
constexpr int kCohRowChunks = 32;

template <typename T>
struct Coh {
  // out = transpose(in) (n x n), optionally scaled by conj(m[a]) m[b] at the
  // source position (a, b)
  static hipError_t transpose(const cx<T>* in, cx<T>* out, int n, const cx<T>* m, hipStream_t s);
  static hipError_t mtable(cx<T>* m, int ny, int nx, const ElementParams<T>& el, int conj, hipStream_t s);
  // g[a][b] *= conj(m[a]) m[b]
  static hipError_t scale(cx<T>* g, const cx<T>* m, int n, hipStream_t s);
  // out[r] += scale * Re g[r][r]
  static hipError_t diag_intensity(const cx<T>* g, T* out, int n, T scale, hipStream_t s);
  static hipError_t diag_loss(const cx<T>* g, const T* ref, cx<T>* grad, double* partial, int n, int kind,
                              T scale, hipStream_t s);
  // colsum: kCohRowChunks * n doubles of column partials
  static hipError_t phase_grad(const cx<T>* G, const cx<T>* Gam, const cx<T>* m, double* rowsum, double* colsum,
                               T* gphi, int n, hipStream_t s);
};

}  // namespace toprop
