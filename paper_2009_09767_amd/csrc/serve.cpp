// serve.cpp -- continuous-admission server for sparse SVD requests.
//
// Requests queue FIFO.  A worker slot (thread + its own context and HIP stream)
// admits the head of the queue as soon as the head's footprint -- its CSC copy plus
// the path's workspace -- fits in the caller's device arena; the CSC is copied into
// the arena (so A and the Gram state stay resident there while it runs) and the
// request runs the same path as ranky_svd on the slot's stream.  Requests arriving
// while others are on the device are admitted as slots and memory free up, and the
// slots' kernels overlap on the GPU.  Nothing is shared between slots but the
// arena's allocator, so each result is bitwise the result of ranky_svd alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ranky.h"

namespace {

using Clock = std::chrono::steady_clock;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// First-fit heap over [0, size) with coalescing of neighbouring free ranges.
class Arena {
public:
    void reset(size_t size) {
        free_.clear();
        free_[0] = size;
        used_ = peak_ = 0;
        size_ = size;
    }
    bool alloc(size_t n, size_t *off) {
        n = align256(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const size_t rest = it->second - n, at = it->first + n;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used_ += n;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = align256(n);
        used_ -= n;
        auto it = free_.emplace(off, n).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t size() const { return size_; }
    size_t peak() const { return peak_; }

private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0, peak_ = 0, size_ = 0;
};

enum ReqState { kQueued, kRunning, kDone };

struct Req {
    uint64_t id = 0;
    ranky_request r;
    size_t csc_bytes = 0, ws_bytes = 0, footprint = 0, off = 0;
    Clock::time_point t_submit, t_done;
    ReqState state = kQueued;
    bool cancel = false;
    ranky_status status = RANKY_PENDING;
    ranky_info info;
};

size_t value_bytes(int32_t dtype) { return dtype == RANKY_F64 ? 8 : 4; }

}  // namespace

struct ranky_server {
    ranky_serve_cfg cfg;
    Arena arena;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req *> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
    std::vector<std::thread> workers;
    bool stopping = false;
    uint64_t next_id = 1;
    int64_t submitted = 0, admitted = 0, completed = 0, failed = 0, cancelled = 0, rejected = 0;
    int64_t running = 0, peak_running = 0;
    double nnz_done = 0.0;
    std::vector<double> lat_us;
    bool any_submit = false;
    Clock::time_point first_submit, last_done;
    ranky_status worker_error = RANKY_OK;

    void worker(int slot);
};

void ranky_server::worker(int slot) {
    (void)slot;
    ranky_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    ranky_status st = ranky_ctx_create(cfg.device, &ctx);
    if (st == RANKY_OK && hipStreamCreate(&stream) != hipSuccess) st = RANKY_E_DEVICE;
    if (st != RANKY_OK) {
        std::lock_guard<std::mutex> lk(mu);
        worker_error = st;
    }
    for (;;) {
        Req *q = nullptr;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] {
                if (queue.empty()) return stopping;
                Req *h = queue.front();
                size_t off = 0;
                if (h->cancel || arena.alloc(h->footprint, &off)) {
                    if (!h->cancel) h->off = off;
                    return true;
                }
                return false;
            });
            if (queue.empty()) break;  // stopping and drained
            q = queue.front();
            queue.pop_front();
            if (q->cancel) {
                q->state = kDone;
                q->status = RANKY_E_CANCELLED;
                q->t_done = Clock::now();
                cancelled += 1;
                cv_done.notify_all();
                cv_work.notify_all();
                continue;
            }
            q->state = kRunning;
            admitted += 1;
            running += 1;
            peak_running = std::max(peak_running, running);
            cv_work.notify_all();  // the next head may fit as well
        }
        // copy the CSC into the arena, then run the path on this slot's stream
        ranky_status rs = st;
        ranky_info info;
        std::memset(&info, 0, sizeof(info));
        if (rs == RANKY_OK) {
            char *base = static_cast<char *>(cfg.arena) + q->off;
            const ranky_request &r = q->r;
            const size_t b_colptr = sizeof(int32_t) * (size_t)(r.N + 1);
            const size_t b_rowidx = sizeof(int32_t) * (size_t)r.A.nnz;
            const size_t b_vals = value_bytes(r.A.dtype) * (size_t)r.A.nnz;
            char *p_colptr = base;
            char *p_rowidx = p_colptr + align256(b_colptr);
            char *p_vals = p_rowidx + align256(b_rowidx);
            char *p_ws = base + q->csc_bytes;
            hipError_t e = hipMemcpyAsync(p_colptr, r.A.colptr, b_colptr, hipMemcpyDeviceToDevice, stream);
            if (e == hipSuccess && b_rowidx)
                e = hipMemcpyAsync(p_rowidx, r.A.rowidx, b_rowidx, hipMemcpyDeviceToDevice, stream);
            if (e == hipSuccess && b_vals) e = hipMemcpyAsync(p_vals, r.A.values, b_vals, hipMemcpyDeviceToDevice, stream);
            if (e != hipSuccess) {
                rs = RANKY_E_DEVICE;
            } else {
                ranky_csc A;
                A.nnz = r.A.nnz;
                A.colptr = reinterpret_cast<const int32_t *>(p_colptr);
                A.rowidx = reinterpret_cast<const int32_t *>(p_rowidx);
                A.values = p_vals;
                A.dtype = r.A.dtype;
                rs = ranky_svd(ctx, &A, r.M, r.N, r.k, r.tol, &cfg.opts, p_ws, q->ws_bytes, r.sigma, r.U, r.V, &info,
                               reinterpret_cast<ranky_stream_t>(stream));
            }
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            arena.release(q->off, q->footprint);
            running -= 1;
            q->t_done = Clock::now();
            q->info = info;
            if (q->cancel) {
                q->status = RANKY_E_CANCELLED;
                cancelled += 1;
            } else {
                q->status = rs;
                if (rs == RANKY_OK) {
                    completed += 1;
                    nnz_done += (double)q->r.A.nnz;
                    lat_us.push_back(std::chrono::duration<double, std::micro>(q->t_done - q->t_submit).count());
                    last_done = q->t_done;
                } else {
                    failed += 1;
                }
            }
            q->state = kDone;
            cv_done.notify_all();
            cv_work.notify_all();
        }
    }
    if (stream) hipStreamDestroy(stream);
    if (ctx) ranky_ctx_destroy(ctx);
}

extern "C" {

ranky_status ranky_serve_create(const ranky_serve_cfg *cfg, ranky_server **out) {
    if (!cfg || !out || !cfg->arena || cfg->arena_bytes == 0 || cfg->max_slots < 1 || cfg->max_queue < 1)
        return RANKY_E_INVALID;
    if (reinterpret_cast<uintptr_t>(cfg->arena) % 256) return RANKY_E_INVALID;   // carved workspaces keep it
    if (cfg->opts.block_start) return RANKY_E_INVALID;   // requests differ in N: no shared boundaries
    auto *s = new ranky_server();
    s->cfg = *cfg;
    s->arena.reset(cfg->arena_bytes);
    for (int i = 0; i < cfg->max_slots; ++i) s->workers.emplace_back(&ranky_server::worker, s, i);
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
    auto q = std::make_unique<Req>();
    q->r = r;
    q->csc_bytes = align256(sizeof(int32_t) * (size_t)(r.N + 1)) + align256(sizeof(int32_t) * (size_t)r.A.nnz) +
                   align256(value_bytes(r.A.dtype) * (size_t)r.A.nnz);
    q->ws_bytes = ws;
    q->footprint = q->csc_bytes + ws;
    std::memset(&q->info, 0, sizeof(q->info));
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stopping) return RANKY_E_INVALID;
    if (q->footprint > srv->arena.size()) {
        srv->rejected += 1;
        return RANKY_E_NOMEM;
    }
    if ((int64_t)srv->queue.size() >= srv->cfg.max_queue) {
        srv->rejected += 1;
        return RANKY_E_BUSY;
    }
    q->id = srv->next_id++;
    q->t_submit = Clock::now();
    if (!srv->any_submit) {
        srv->any_submit = true;
        srv->first_submit = q->t_submit;
    }
    *ticket = q->id;
    srv->queue.push_back(q.get());
    srv->reqs.emplace(q->id, std::move(q));
    srv->submitted += 1;
    srv->cv_work.notify_all();
    return RANKY_OK;
}

ranky_status ranky_serve_poll(ranky_server *srv, uint64_t ticket, ranky_info *info) {
    if (!srv) return RANKY_E_INVALID;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return RANKY_E_INVALID;
    if (it->second->state != kDone) return RANKY_PENDING;
    if (info) *info = it->second->info;
    return it->second->status;
}

ranky_status ranky_serve_wait(ranky_server *srv, uint64_t ticket, int64_t timeout_us, ranky_info *info) {
    if (!srv) return RANKY_E_INVALID;
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return RANKY_E_INVALID;
    Req *q = it->second.get();
    auto done = [&] { return q->state == kDone; };
    if (timeout_us < 0) srv->cv_done.wait(lk, done);
    else srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done);
    if (q->state != kDone) return RANKY_PENDING;
    if (info) *info = q->info;
    return q->status;
}

ranky_status ranky_serve_cancel(ranky_server *srv, uint64_t ticket) {
    if (!srv) return RANKY_E_INVALID;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return RANKY_E_INVALID;
    Req *q = it->second.get();
    if (q->state == kDone) return RANKY_OK;
    q->cancel = true;
    if (q->state == kQueued) {
        auto pos = std::find(srv->queue.begin(), srv->queue.end(), q);
        if (pos != srv->queue.end()) srv->queue.erase(pos);
        q->state = kDone;
        q->status = RANKY_E_CANCELLED;
        q->t_done = Clock::now();
        srv->cancelled += 1;
        srv->cv_done.notify_all();
        srv->cv_work.notify_all();
    }
    return RANKY_OK;
}

ranky_status ranky_serve_stats(ranky_server *srv, ranky_serve_summary *out) {
    if (!srv || !out) return RANKY_E_INVALID;
    std::lock_guard<std::mutex> lk(srv->mu);
    std::memset(out, 0, sizeof(*out));
    std::vector<double> l = srv->lat_us;
    std::sort(l.begin(), l.end());
    if (!l.empty()) {
        auto pct = [&](double p) {  // nearest-rank percentile
            size_t idx = (size_t)std::ceil(p * (double)l.size());
            if (idx < 1) idx = 1;
            return l[std::min(idx, l.size()) - 1];
        };
        out->p50_us = pct(0.50);
        out->p99_us = pct(0.99);
        double sum = 0.0;
        for (double v : l) sum += v;
        out->mean_us = sum / (double)l.size();
        out->max_us = l.back();
        out->span_s = std::chrono::duration<double>(srv->last_done - srv->first_submit).count();
        if (out->span_s > 0) {
            out->req_per_s = (double)srv->completed / out->span_s;
            out->nnz_per_s = srv->nnz_done / out->span_s;
        }
    }
    out->submitted = srv->submitted;
    out->admitted = srv->admitted;
    out->completed = srv->completed;
    out->failed = srv->failed;
    out->cancelled = srv->cancelled;
    out->rejected = srv->rejected;
    out->queued_now = (int64_t)srv->queue.size();
    out->running_now = srv->running;
    out->peak_running = srv->peak_running;
    out->arena_peak_bytes = srv->arena.peak();
    return RANKY_OK;
}

ranky_status ranky_serve_destroy(ranky_server *srv) {
    if (!srv) return RANKY_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stopping = true;
        srv->cv_work.notify_all();
    }
    for (auto &t : srv->workers) t.join();
    const ranky_status st = srv->worker_error;
    delete srv;
    return st;
}

}  // extern "C"
