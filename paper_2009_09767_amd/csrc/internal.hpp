// internal.hpp -- entry points of the host runtime shared between its source files.
#pragma once

#include <hip/hip_runtime.h>

#include "ranky.h"

namespace ranky {

// Sets the thread-local error text and returns st.
ranky_status set_error(ranky_status st, const char *fmt, ...);
// Device of a context.
int ctx_device(const ranky_ctx *ctx);
// ranky_svd on a workspace the caller does not own, with no allocation on the way: the context's
// staging must already be large enough (E_NOMEM otherwise) and the sweep is never captured.
ranky_status svd_fixed_workspace(ranky_ctx *ctx, const ranky_csc *A, int32_t M, int64_t N, int32_t k, double tol,
                                 const ranky_opts *opts, void *workspace, size_t ws_bytes, double *sigma, double *U,
                                 void *V, ranky_info *info, ranky_stream_t stream);
// The device address of the fixed scratch array on `device` (current), looked up once.
hipError_t noalloc_setup(int device);

}  // namespace ranky
