// Host-side launchers of the job-queue passes: one launch of a pass over
// the jobs of one shape class (kernels in kernels.hpp).  Instantiated per
// real type in queue_f32.hip / queue_f64.hip.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace toprop {

// Transform lengths of the job-queue column pass, and of jobs grouped into
// one launch: the jobs whose own launches are too small to fill the device.
// From 2048 points on, one job's column pass alone has as many workgroups as
// the device holds at once, and the per-job launches on the lanes measured
// as fast or faster.
constexpr int kQueueMinLen = 64;
constexpr int kQueueMaxLen = 1024;
inline bool queue_len_ok(int L) { return L >= kQueueMinLen && L <= kQueueMaxLen && (L & (L - 1)) == 0; }
// The row passes are built up to the longest transform: with one job and one
// workgroup per block (cus = 0 below) they are the per-job row passes of a
// job without element or epilogue, whose folded branches free registers
// (the 8192-point backward row pass: 104 VGPRs and no spills against 128
// VGPRs and 85 spilled).
constexpr int kQueueRowMaxLen = 8192;
inline bool queue_row_len_ok(int L) { return L >= kQueueMinLen && L <= kQueueRowMaxLen && (L & (L - 1)) == 0; }

// The caller fills q.njobs, the pass-independent fields of q and, per job,
// the pointers, ny, nx, nfields and fpb (fields per workgroup of this pass;
// backward row_inv: all of the job's fields).  The launcher sets each job's
// grid (gx, gy) from the kernel configuration, numbers the items (each job's
// first item a multiple of 8, so that item index and block index agree
// modulo the XCD count), and launches at most as many workgroups as are
// resident at once on `cus` CUs (cus <= 0: one workgroup per item).
// `exact`: every job's extent along the transformed axis fills its
// registers exactly (as for the per-job launch).
template <typename T>
struct QueueLaunch {
  static hipError_t row_fwd(int lx, bool half, bool exact, QueueArgs<T>& q, int cus, hipStream_t s);
  static hipError_t col(int ly, bool half, bool exact, int variant, ColQueueArgs<T>& q, int cus, hipStream_t s);
  static hipError_t row_inv(int lx, bool half, bool exact, bool bwd, QueueArgs<T>& q, int cus, hipStream_t s);
};

}  // namespace toprop
