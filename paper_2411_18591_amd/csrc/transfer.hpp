// Transfer-function tables: the direct-integration (DI) table, and the
// tabulated AS / Fresnel transfer function of a job.
#pragma once
#include <hip/hip_runtime.h>

#include "bluestein.hpp"
#include "kernels.hpp"

namespace toprop {

// Geometry of a DI table (see di_sample_kernel).
struct DiParams {
  int ny, nx;      // field grid: offsets |sy| < ny, |sx| < nx are sampled
  int py, px;      // padded grid
  double dy, dx;   // spacing [m]
  double z;        // distance [m], > 0
  double lam;      // wavelength [m]
  double q_frac;   // frac(z / lambda), computed exactly on the host
};

// Separable complex64 transfer-function tables (see TransferParams) of many
// propagations, built by one launch: table k is {ex[lx], ey[ly], sx[lx],
// sy[ly]} at `base[k]`.
struct SepTableDesc {
  void* base;
  int lx, ly;
  double inv_lxdx, inv_lydy, fres_a, q_frac, lam2;
};
constexpr int kSepBatch = 32;  // tables per launch (kernel arguments stay < 4 KiB)
struct SepTableBatch {
  int count;
  int maxlen;  // largest lx + ly of the batch
  SepTableDesc d[kSepBatch];
};
hipError_t separable_tables(const SepTableBatch& b, hipStream_t s);

template <typename T>
struct TransferTable {
  // DI: H = FFT2(sampled impulse response * dx dy), [py][px] row-major,
  // built in place in H.  With `tr` (py * px elements of scratch), columns
  // whose length is not a power of two are transformed as rows of the
  // transposed table; without it, in place with strided access.
  static hipError_t direct_integration(cx<T>* H, const DiParams& p, const LineFft<T>& fx, const LineFft<T>& fy,
                                       hipStream_t s, cx<T>* tr = nullptr);
  // The same table stored transposed, HT[kx][ky] ([px][py]), as the
  // any-length column launch reads it; `tmp` holds py * px elements.
  static hipError_t direct_integration_t(cx<T>* HT, cx<T>* tmp, const DiParams& p, const LineFft<T>& fx,
                                         const LineFft<T>& fy, hipStream_t s);
  // AS / Fresnel: H at every bin of the padded grid.
  static hipError_t analytic(cx<T>* H, int py, int px, const TransferParams& p, hipStream_t s);
};

}  // namespace toprop
