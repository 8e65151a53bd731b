// serve_core.hpp -- the request scheduler behind ranky_serve_*, independent of the device.
//
// Requests queue FIFO.  A worker slot admits the head of the queue as soon as its
// footprint fits in a first-fit arena (offsets into the caller's device buffer); the
// slot's executor then computes the request and the footprint is released.  Requests
// arriving while others run are admitted as slots and memory free up.  The executor is
// a template parameter so that the scheduling logic builds and runs on the host alone
// (a fake executor under the thread and address sanitizers); serve.cpp binds it to the
// HIP path.  Nothing here touches HIP.
#pragma once

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

namespace ranky_serve {

using Clock = std::chrono::steady_clock;

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

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
    size_t used() const { return used_; }

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
    std::vector<int32_t> blk;   // the request's own copy of the per-block counts info points to
};

// Exec must provide
//   ranky_status run(const Req &q, ranky_info *info)
// which computes request q in its arena range [q.off, q.off + q.footprint) on the calling
// worker thread and fills *info.  One Exec per slot, used by that slot's thread only.
template <class Exec>
class Scheduler {
public:
    Scheduler(size_t arena_bytes, int32_t max_queue) : max_queue_(max_queue) { arena_.reset(arena_bytes); }
    ~Scheduler() { stop(); }

    // Takes ownership of one executor per slot and starts the slot threads.
    void start(std::vector<std::unique_ptr<Exec>> execs) {
        execs_ = std::move(execs);
        for (size_t i = 0; i < execs_.size(); ++i) workers_.emplace_back(&Scheduler::worker, this, (int)i);
    }

    size_t arena_size() const { return arena_.size(); }

    // E_NOMEM: the footprint can never fit; E_BUSY: the queue is full; E_INVALID: stopping.
    ranky_status submit(const ranky_request &r, size_t csc_bytes, size_t ws_bytes, uint64_t *ticket) {
        auto q = std::make_unique<Req>();
        q->r = r;
        q->csc_bytes = csc_bytes;
        q->ws_bytes = ws_bytes;
        q->footprint = csc_bytes + ws_bytes;
        std::memset(&q->info, 0, sizeof(q->info));
        std::lock_guard<std::mutex> lk(mu_);
        if (stopping_) return RANKY_E_INVALID;
        if (align256(q->footprint) > arena_.size()) {
            rejected_ += 1;
            return RANKY_E_NOMEM;
        }
        if ((int64_t)queue_.size() >= max_queue_) {
            rejected_ += 1;
            return RANKY_E_BUSY;
        }
        q->id = next_id_++;
        q->t_submit = Clock::now();
        if (!any_submit_) {
            any_submit_ = true;
            first_submit_ = q->t_submit;
        }
        *ticket = q->id;
        queue_.push_back(q.get());
        reqs_.emplace(q->id, std::move(q));
        submitted_ += 1;
        cv_work_.notify_all();
        return RANKY_OK;
    }

    ranky_status poll(uint64_t ticket, ranky_info *info) {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = reqs_.find(ticket);
        if (it == reqs_.end()) return RANKY_E_INVALID;
        if (it->second->state != kDone) return RANKY_PENDING;
        if (info) *info = it->second->info;
        return it->second->status;
    }

    ranky_status wait(uint64_t ticket, int64_t timeout_us, ranky_info *info) {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = reqs_.find(ticket);
        if (it == reqs_.end()) return RANKY_E_INVALID;
        Req *q = it->second.get();
        auto done = [&] { return q->state == kDone; };
        if (timeout_us < 0) cv_done_.wait(lk, done);
        else cv_done_.wait_for(lk, std::chrono::microseconds(timeout_us), done);
        if (q->state != kDone) return RANKY_PENDING;
        if (info) *info = q->info;
        return q->status;
    }

    ranky_status cancel(uint64_t ticket) {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = reqs_.find(ticket);
        if (it == reqs_.end()) return RANKY_E_INVALID;
        Req *q = it->second.get();
        if (q->state == kDone) return RANKY_OK;
        q->cancel = true;
        if (q->state == kQueued) {
            auto pos = std::find(queue_.begin(), queue_.end(), q);
            if (pos != queue_.end()) queue_.erase(pos);
            q->state = kDone;
            q->status = RANKY_E_CANCELLED;
            q->t_done = Clock::now();
            cancelled_ += 1;
            cv_done_.notify_all();
            cv_work_.notify_all();
        }
        return RANKY_OK;
    }

    void stats(ranky_serve_summary *out) {
        std::lock_guard<std::mutex> lk(mu_);
        std::memset(out, 0, sizeof(*out));
        std::vector<double> l = lat_us_;
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
            out->span_s = std::chrono::duration<double>(last_done_ - first_submit_).count();
            if (out->span_s > 0) {
                out->req_per_s = (double)completed_ / out->span_s;
                out->nnz_per_s = nnz_done_ / out->span_s;
            }
        }
        out->submitted = submitted_;
        out->admitted = admitted_;
        out->completed = completed_;
        out->failed = failed_;
        out->cancelled = cancelled_;
        out->rejected = rejected_;
        out->queued_now = (int64_t)queue_.size();
        out->running_now = running_;
        out->peak_running = peak_running_;
        out->arena_peak_bytes = arena_.peak();
    }

    // Stops admission of new submissions, drains queued and running requests, joins the
    // slot threads.  Idempotent.
    void stop() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stopping_ = true;
            cv_work_.notify_all();
        }
        for (auto &t : workers_)
            if (t.joinable()) t.join();
        workers_.clear();
    }

    // Arena bytes in use (0 once every admitted request has completed).
    size_t arena_used() {
        std::lock_guard<std::mutex> lk(mu_);
        return arena_.used();
    }

private:
    void worker(int slot) {
        Exec &ex = *execs_[slot];
        for (;;) {
            Req *q = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_work_.wait(lk, [&] {
                    if (queue_.empty()) return stopping_;
                    Req *h = queue_.front();
                    size_t off = 0;
                    if (h->cancel || arena_.alloc(h->footprint, &off)) {
                        if (!h->cancel) h->off = off;
                        return true;
                    }
                    return false;
                });
                if (queue_.empty()) break;  // stopping and drained
                q = queue_.front();
                queue_.pop_front();
                if (q->cancel) {
                    q->state = kDone;
                    q->status = RANKY_E_CANCELLED;
                    q->t_done = Clock::now();
                    cancelled_ += 1;
                    cv_done_.notify_all();
                    cv_work_.notify_all();
                    continue;
                }
                q->state = kRunning;
                admitted_ += 1;
                running_ += 1;
                peak_running_ = std::max(peak_running_, running_);
                cv_work_.notify_all();  // the next head may fit as well
            }
            ranky_info info;
            std::memset(&info, 0, sizeof(info));
            const ranky_status rs = ex.run(*q, &info);
            // the per-block counts live in the slot's context until its next request: keep a copy
            std::vector<int32_t> blk;
            if (info.lonely_per_block && info.n_blocks > 0) {
                blk.assign(info.lonely_per_block, info.lonely_per_block + info.n_blocks);
                if (info.single_per_block) blk.insert(blk.end(), info.single_per_block, info.single_per_block + info.n_blocks);
            }
            {
                std::lock_guard<std::mutex> lk(mu_);
                arena_.release(q->off, q->footprint);
                running_ -= 1;
                q->t_done = Clock::now();
                q->blk = std::move(blk);
                q->info = info;
                q->info.lonely_per_block = q->blk.empty() ? nullptr : q->blk.data();
                q->info.single_per_block =
                    q->blk.size() >= 2 * (size_t)info.n_blocks && info.n_blocks > 0 ? q->blk.data() + info.n_blocks : nullptr;
                if (q->cancel) {
                    q->status = RANKY_E_CANCELLED;
                    cancelled_ += 1;
                } else {
                    q->status = rs;
                    if (rs == RANKY_OK) {
                        completed_ += 1;
                        nnz_done_ += (double)q->r.A.nnz;
                        lat_us_.push_back(std::chrono::duration<double, std::micro>(q->t_done - q->t_submit).count());
                        last_done_ = q->t_done;
                    } else {
                        failed_ += 1;
                    }
                }
                q->state = kDone;
                cv_done_.notify_all();
                cv_work_.notify_all();
            }
        }
    }

    Arena arena_;
    int32_t max_queue_;
    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::deque<Req *> queue_;
    std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs_;
    std::vector<std::unique_ptr<Exec>> execs_;
    std::vector<std::thread> workers_;
    bool stopping_ = false;
    uint64_t next_id_ = 1;
    int64_t submitted_ = 0, admitted_ = 0, completed_ = 0, failed_ = 0, cancelled_ = 0, rejected_ = 0;
    int64_t running_ = 0, peak_running_ = 0;
    double nnz_done_ = 0.0;
    std::vector<double> lat_us_;
    bool any_submit_ = false;
    Clock::time_point first_submit_, last_done_;
};

}  // namespace ranky_serve
