// serve.cpp -- continuous-admission server for sparse SVD requests (ranky_serve_*).
//
// The scheduler (serve_core.hpp) queues requests FIFO and admits the head as soon as its
// footprint -- its CSC copy plus the path's workspace -- fits in the caller's device arena
// and a slot is free.  Each slot's executor here owns a context and a HIP stream: it copies
// the admitted CSC into the arena (so A and the Gram state stay resident there while it
// runs) and runs the same path as ranky_svd on the slot's stream.  Requests arriving while
// others are on the device are admitted as slots and memory free up, and the slots' kernels
// overlap on the GPU.  Nothing is shared between slots but the arena's allocator, so each
// result is bitwise the result of ranky_svd alone.
//
// Every slot's context and stream are created on the thread that calls ranky_serve_create,
// one after the other, before any slot thread starts: no slot sets up device state while
// another launches kernels.
#include <hip/hip_runtime.h>

#include <cstring>
#include <memory>
#include <vector>

#include "ranky.h"
#include "serve_core.hpp"

namespace {

using ranky_serve::align256;
using ranky_serve::Req;

size_t value_bytes(int32_t dtype) { return dtype == RANKY_F64 ? 8 : 4; }

class DeviceExec {
public:
    DeviceExec(const ranky_serve_cfg &cfg) : cfg_(cfg) {}
    ~DeviceExec() {
        if (stream_) hipStreamDestroy(stream_);
        if (ctx_) ranky_ctx_destroy(ctx_);
    }
    ranky_status init() {
        ranky_status st = ranky_ctx_create(cfg_.device, &ctx_);
        if (st != RANKY_OK) return st;
        if (hipStreamCreate(&stream_) != hipSuccess) return RANKY_E_DEVICE;
        return RANKY_OK;
    }
    ranky_status run(const Req &q, ranky_info *info) {
        char *base = static_cast<char *>(cfg_.arena) + q.off;
        const ranky_request &r = q.r;
        const size_t b_colptr = sizeof(int32_t) * (size_t)(r.N + 1);
        const size_t b_rowidx = sizeof(int32_t) * (size_t)r.A.nnz;
        const size_t b_vals = value_bytes(r.A.dtype) * (size_t)r.A.nnz;
        char *p_colptr = base;
        char *p_rowidx = p_colptr + align256(b_colptr);
        char *p_vals = p_rowidx + align256(b_rowidx);
        char *p_ws = base + q.csc_bytes;
        hipError_t e = hipMemcpyAsync(p_colptr, r.A.colptr, b_colptr, hipMemcpyDeviceToDevice, stream_);
        if (e == hipSuccess && b_rowidx) e = hipMemcpyAsync(p_rowidx, r.A.rowidx, b_rowidx, hipMemcpyDeviceToDevice, stream_);
        if (e == hipSuccess && b_vals) e = hipMemcpyAsync(p_vals, r.A.values, b_vals, hipMemcpyDeviceToDevice, stream_);
        if (e != hipSuccess) return RANKY_E_DEVICE;
        ranky_csc A;
        A.nnz = r.A.nnz;
        A.colptr = reinterpret_cast<const int32_t *>(p_colptr);
        A.rowidx = reinterpret_cast<const int32_t *>(p_rowidx);
        A.values = p_vals;
        A.dtype = r.A.dtype;
        return ranky_svd(ctx_, &A, r.M, r.N, r.k, r.tol, &cfg_.opts, p_ws, q.ws_bytes, r.sigma, r.U, r.V, info,
                         reinterpret_cast<ranky_stream_t>(stream_));
    }

private:
    ranky_serve_cfg cfg_;
    ranky_ctx *ctx_ = nullptr;
    hipStream_t stream_ = nullptr;
};

}  // namespace

struct ranky_server {
    ranky_serve_cfg cfg;
    std::unique_ptr<ranky_serve::Scheduler<DeviceExec>> sched;
};

extern "C" {

ranky_status ranky_serve_create(const ranky_serve_cfg *cfg, ranky_server **out) {
    if (!cfg || !out || !cfg->arena || cfg->arena_bytes == 0 || cfg->max_slots < 1 || cfg->max_queue < 1)
        return RANKY_E_INVALID;
    if (reinterpret_cast<uintptr_t>(cfg->arena) % 256) return RANKY_E_INVALID;   // carved workspaces keep it
    if (cfg->opts.block_start) return RANKY_E_INVALID;   // requests differ in N: no shared boundaries
    std::vector<std::unique_ptr<DeviceExec>> execs;
    for (int i = 0; i < cfg->max_slots; ++i) {
        execs.emplace_back(new DeviceExec(*cfg));
        const ranky_status st = execs.back()->init();
        if (st != RANKY_OK) return st;   // the executors made so far are destroyed here
    }
    auto *s = new ranky_server();
    s->cfg = *cfg;
    s->sched.reset(new ranky_serve::Scheduler<DeviceExec>(cfg->arena_bytes, cfg->max_queue));
    s->sched->start(std::move(execs));
    *out = s;
    return RANKY_OK;
}

ranky_status ranky_serve_submit(ranky_server *srv, const ranky_request *req, uint64_t *ticket) {
    if (!srv || !req || !ticket) return RANKY_E_INVALID;
    const ranky_request &r = *req;
    if (r.M < 1 || r.N < 1 || r.k < 1 || r.k > r.M || r.A.nnz < 0 || !r.A.colptr || !r.sigma || !r.U || !r.V ||
        !(r.tol >= 0.0) || (r.A.dtype != RANKY_F32 && r.A.dtype != RANKY_F64) ||
        (r.A.nnz > 0 && (!r.A.rowidx || !r.A.values)))
        return RANKY_E_INVALID;
    const size_t ws = ranky_workspace_bytes(r.M, r.N, r.A.nnz, r.k, &srv->cfg.opts);
    if (ws == 0) return RANKY_E_INVALID;
    const size_t csc = align256(sizeof(int32_t) * (size_t)(r.N + 1)) + align256(sizeof(int32_t) * (size_t)r.A.nnz) +
                       align256(value_bytes(r.A.dtype) * (size_t)r.A.nnz);
    return srv->sched->submit(r, csc, ws, ticket);
}

ranky_status ranky_serve_poll(ranky_server *srv, uint64_t ticket, ranky_info *info) {
    if (!srv) return RANKY_E_INVALID;
    return srv->sched->poll(ticket, info);
}

ranky_status ranky_serve_wait(ranky_server *srv, uint64_t ticket, int64_t timeout_us, ranky_info *info) {
    if (!srv) return RANKY_E_INVALID;
    return srv->sched->wait(ticket, timeout_us, info);
}

ranky_status ranky_serve_cancel(ranky_server *srv, uint64_t ticket) {
    if (!srv) return RANKY_E_INVALID;
    return srv->sched->cancel(ticket);
}

ranky_status ranky_serve_stats(ranky_server *srv, ranky_serve_summary *out) {
    if (!srv || !out) return RANKY_E_INVALID;
    srv->sched->stats(out);
    return RANKY_OK;
}

ranky_status ranky_serve_destroy(ranky_server *srv) {
    if (!srv) return RANKY_OK;
    srv->sched->stop();
    delete srv;
    return RANKY_OK;
}

}  // extern "C"
