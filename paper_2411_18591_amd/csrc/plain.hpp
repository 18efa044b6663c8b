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
  int ht;               // 1: H is stored transposed ([px][py]) and the job takes run_mixed
  int64_t nbatch = 1;   // run_mixed: consecutive fields of in / out in one pass (pad and tr hold as many)
  int hcalc = 0;        // run_mixed: form the transfer function from tp in the column launch (no table)
  TransferParams tp{};  // AS or Fresnel parameters, tp.conj for the adjoint
};

template <typename T>
struct Plain {
  static hipError_t run(const PlainJob<T>& pj, hipStream_t s);
  // Grids with an extent that is not a power of two and both extents of the
  // form 2^a 3^b 5^c 7^d (<= 4096): zero padding, crop, the transfer
  // function and both column transforms fused into three mixed-radix
  // launches around two transposes, and only the ny rows that are not zero
  // transformed.  Needs H transposed (pj.ht); pad and tr hold pj.nbatch *
  // ny * px elements, and the pj.nbatch fields go through each launch
  // together.
  static hipError_t run_mixed(const PlainJob<T>& pj, hipStream_t s);
  // The table of every bin, [py][px], or [px][py] with `transposed`.
  static hipError_t table(cx<T>* H, int py, int px, const TransferParams& p, hipStream_t s, bool transposed = false);
  static hipError_t rows(int L, cx<T>* a, int nrows, int dir, const cx<T>* tw, hipStream_t s);
  static hipError_t cols(int L, cx<T>* a, int lx, int dir, const cx<T>* tw, hipStream_t s);
  // Any length: the power-of-two passes above, or Bluestein's transform.
  static hipError_t rows_any(const LineFft<T>& f, cx<T>* a, int nrows, int dir, hipStream_t s);
  // Bluestein columns run as rows of the transposed array when `tr` (f.L *
  // lx elements) is given, else column-wise.
  static hipError_t cols_any(const LineFft<T>& f, cx<T>* a, int lx, int dir, hipStream_t s, cx<T>* tr = nullptr);
  // Lens focal-length gradient of one field (g = P^H grad_out, u the saved
  // input): per-block FP64 partial sums into partial[0 .. *nblocks), at most
  // 1024 blocks.
  static hipError_t lens_grad(const cx<T>* g, const cx<T>* u, double* partial, int ny, int nx,
                              const ElementParams<T>& el, double f, int* nblocks, hipStream_t s);
  // I[i] += scale |u[i]|^2, i < n (the intensity epilogue)
  static hipError_t intensity(const cx<T>* u, T* I, int64_t n, T scale, hipStream_t s);
  static hipError_t loss(const cx<T>* u, const T* ref, cx<T>* grad, double* partial, int64_t n, int kind,
                         T scale, int* nblocks, hipStream_t s);
  static hipError_t modulate(const cx<T>* in, cx<T>* out, int ny, int nx, const ElementParams<T>& el, int conj,
                             hipStream_t s);
  static hipError_t phase_grad(const cx<T>* g, const cx<T>* u, T* gphi, int ny, int nx,
                               const ElementParams<T>& el, hipStream_t s);
};

}  // namespace toprop
