// Internal interface between the no-allocation entry point (noalloc.hip)
// and the launch sequences of capi.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "../../include/toprop.h"

namespace toprop {

// Twiddle tables of every power-of-two length 8..8192 packed back to back,
// length L from entry L - 8: 2 * 8192 - 8 entries per precision.
constexpr int kTwPacked = 2 * 8192 - 8;

// Record `msg` (or the HIP error of `what`) as the calling thread's last
// error and return `st` (TO_E_HIP).
to_status set_error(to_status st, const char* msg);
to_status hip_error(hipError_t e, const char* what);

// to_propagate's argument checks (every job, plus the limits of the fixed
// area: power-of-two padded grids, one field's scratch within the area,
// direct integration only with a caller table).
to_status validate_forward(const to_job* jobs, int32_t njobs, to_dtype dtype, size_t ws_bytes);

// to_propagate's work on `s` alone with every workspace carved from the
// device area `ws` of `ws_bytes`; `tw` holds the complex64 then the
// complex128 twiddle tables in the packed layout.  Allocates nothing.
to_status propagate_fixed(const to_job* jobs, int32_t njobs, to_dtype dtype, hipStream_t s, const void* tw,
                          void* ws, size_t ws_bytes);

}  // namespace toprop
