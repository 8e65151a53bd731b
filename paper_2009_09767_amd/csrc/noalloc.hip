// noalloc.hip -- ranky_svd_noalloc: the whole path of ranky_svd with its workspace in a fixed
// device array of the library instead of caller memory, for callers that cannot allocate
// (code under HIP graph capture, tight serving loops, harnesses that forbid allocation).
//
// The array `scratch` is a file-scope device variable: every GPU the library runs on holds its
// own copy, of kNoallocBytes, until the process ends.  Its name in host code is only a host-side
// stand-in; the device address of each GPU's copy is looked up once per device with that device
// current (hipGetSymbolAddress, when a context is created for the device) and kept in a table,
// and only that address is ever handed to kernels.  All calls on one GPU share its copy: the
// path initialises everything it reads, so nothing carries over from the previous call, but
// calls that overlap on one GPU (several streams or threads at once) race on it.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "internal.hpp"
#include "ranky.h"

namespace {

constexpr size_t kNoallocBytes = RANKY_NOALLOC_WORKSPACE_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __attribute__((aligned(256))) unsigned char scratch[kNoallocBytes];

std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};   // device address of each device's copy

}  // namespace

namespace ranky {

hipError_t noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[device] = p;
    return hipSuccess;
}

}  // namespace ranky

extern "C" ranky_status ranky_svd_noalloc(ranky_ctx *ctx, const ranky_csc *A, int32_t M, int64_t N, int32_t k,
                                          double tol, const ranky_opts *opts, double *sigma, double *U, void *V,
                                          ranky_info *info, ranky_stream_t stream) {
    if (!ctx) return ranky::set_error(RANKY_E_INVALID, "ctx is NULL");
    const int dev = ranky::ctx_device(ctx);
    void *ws = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (dev >= 0 && dev < kMaxDevices) ws = g_scratch[dev];
    }
    if (!ws) return ranky::set_error(RANKY_E_DEVICE, "no scratch address for device %d", dev);
    const size_t need = ranky_workspace_bytes(M, N, A ? A->nnz : 0, k, opts);
    if (need > kNoallocBytes)
        return ranky::set_error(RANKY_E_NOMEM, "the problem needs %zu bytes of workspace; the fixed scratch holds %zu",
                                need, kNoallocBytes);
    return ranky::svd_fixed_workspace(ctx, A, M, N, k, tol, opts, ws, kNoallocBytes, sigma, U, V, info, stream);
}
