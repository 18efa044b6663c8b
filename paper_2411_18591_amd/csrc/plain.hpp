// Host interface of the plain (unfused, one field per launch sequence)
// propagation used as the comparison baseline.
#pragma once
#include <hip/hip_runtime.h>

#include "bluestein.hpp"
#include "kernels.hpp"

namespace toprop {

template <typename T>
struct PlainJob {
  int ny, nx, py, px;
  const cx<T>* in;   // one field [ny][nx]
  cx<T>* out;        // one field [ny][nx]
  cx<T>* tmp;        // [ny][nx] workspace (modulated field)
  cx<T>* pad;        // [py][px] workspace
  const cx<T>* H;    // [py][px] transfer-function table
  int conj;          // multiply by conj(H)
  ElementParams<T> el;  // forward element (flags 0 = none)
  LineFft<T> fx;        // transforms of length px
  LineFft<T> fy;        // transforms of length py
  cx<T>* tr;            // [px][py] workspace for Bluestein columns, or null
};

template <typename T>
struct Plain {
  static hipError_t run(const PlainJob<T>& pj, hipStream_t s);
  static hipError_t table(cx<T>* H, int py, int px, const TransferParams& p, hipStream_t s);
  static hipError_t rows(int L, cx<T>* a, int nrows, int dir, const cx<T>* tw, hipStream_t s);
  static hipError_t cols(int L, cx<T>* a, int lx, int dir, const cx<T>* tw, hipStream_t s);
  // Any length: the power-of-two passes above, or Bluestein's transform.
  static hipError_t rows_any(const LineFft<T>& f, cx<T>* a, int nrows, int dir, hipStream_t s);
  // Bluestein columns run as rows of the transposed array when `tr` (f.L *
  // lx elements) is given, else column-wise.
  static hipError_t cols_any(const LineFft<T>& f, cx<T>* a, int lx, int dir, hipStream_t s, cx<T>* tr = nullptr);
  static hipError_t loss(const cx<T>* u, const T* ref, cx<T>* grad, double* partial, int64_t n, int kind,
                         T scale, int* nblocks, hipStream_t s);
  static hipError_t modulate(const cx<T>* in, cx<T>* out, int ny, int nx, const ElementParams<T>& el, int conj,
                             hipStream_t s);
  static hipError_t phase_grad(const cx<T>* g, const cx<T>* u, T* gphi, int ny, int nx,
                               const ElementParams<T>& el, hipStream_t s);
};

}  // namespace toprop
