// Host-only check of the serving scheduler (csrc/serve_core.hpp) with a fake executor:
// several submitter threads, random footprints, cancellations, a small arena.  Built twice by
// tests/test_serve_cpu.py, under ThreadSanitizer and under AddressSanitizer + UBSan.
//
// Checked: every admitted request's arena range [off, off + footprint) lies inside the arena
// and overlaps no other running request's range; no more requests run at once than there are
// slots; every ticket ends in exactly one final state; the arena is empty at the end; the
// counters add up; and each request's per-block counts come back as its own copy.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <random>
#include <set>
#include <thread>
#include <utility>
#include <vector>

#include "serve_core.hpp"

namespace {

constexpr size_t kArena = 1 << 20;
constexpr int kSlots = 4;

std::mutex g_mu;
std::set<std::pair<size_t, size_t>> g_live;   // running [off, end) ranges
std::atomic<int> g_running{0}, g_max_running{0}, g_errors{0};
std::vector<unsigned char> g_arena(kArena);

void error(const char *what) {
    std::fprintf(stderr, "FAIL: %s\n", what);
    g_errors.fetch_add(1);
}

struct FakeExec {
    int slot;
    std::vector<int32_t> counts;   // the slot's "context memory" for the per-block counts
    explicit FakeExec(int s) : slot(s) {}
    ranky_status run(const ranky_serve::Req &q, ranky_info *info) {
        const size_t end = q.off + ranky_serve::align256(q.footprint);
        if (end > kArena) error("range outside the arena");
        {
            std::lock_guard<std::mutex> lk(g_mu);
            for (const auto &r : g_live)
                if (q.off < r.second && r.first < end) error("overlapping arena ranges");
            g_live.insert({q.off, end});
        }
        const int now = g_running.fetch_add(1) + 1;
        int prev = g_max_running.load();
        while (now > prev && !g_max_running.compare_exchange_weak(prev, now)) {
        }
        // touch every byte of the range (ASan: in bounds; TSan: no other writer)
        for (size_t b = q.off; b < std::min(end, kArena); ++b) g_arena[b] = (unsigned char)(q.id & 0xff);
        std::this_thread::sleep_for(std::chrono::microseconds(50 + (q.id * 7919) % 400));
        for (size_t b = q.off; b < std::min(end, kArena); ++b)
            if (g_arena[b] != (unsigned char)(q.id & 0xff)) {
                error("arena bytes changed under a running request");
                break;
            }
        g_running.fetch_sub(1);
        {
            std::lock_guard<std::mutex> lk(g_mu);
            g_live.erase({q.off, end});
        }
        const int D = 1 + (int)(q.id % 5);
        counts.assign(2 * D, 0);
        for (int b = 0; b < D; ++b) {
            counts[b] = (int32_t)(q.id + b);
            counts[D + b] = (int32_t)(2 * q.id + b);
        }
        info->n_blocks = D;
        info->lonely_per_block = counts.data();
        info->single_per_block = counts.data() + D;
        info->rank = (int32_t)q.id;
        return q.id % 11 == 0 ? RANKY_E_NOT_CONVERGED : RANKY_OK;
    }
};

}  // namespace

int main() {
    using Sched = ranky_serve::Scheduler<FakeExec>;
    std::vector<std::unique_ptr<FakeExec>> execs;
    for (int i = 0; i < kSlots; ++i) execs.emplace_back(new FakeExec(i));
    Sched sched(kArena, 64);
    sched.start(std::move(execs));

    std::mutex tmu;
    std::vector<uint64_t> tickets;
    std::atomic<int> busy{0}, nomem{0};
    auto submitter = [&](int seed) {
        std::mt19937 rng(seed);
        for (int i = 0; i < 400; ++i) {
            ranky_request r;
            std::memset(&r, 0, sizeof(r));
            r.A.nnz = 1000 + (rng() % 5000);
            r.M = 8;
            r.N = 16;
            r.k = 4;
            const size_t csc = 256 * (1 + rng() % 64);
            const size_t ws = (rng() % 100 == 0) ? 2 * kArena : 256 * (1 + rng() % 1024);   // a few never fit
            uint64_t t = 0;
            const ranky_status st = sched.submit(r, csc, ws, &t);
            if (st == RANKY_OK) {
                std::lock_guard<std::mutex> lk(tmu);
                tickets.push_back(t);
                if (rng() % 13 == 0) sched.cancel(t);
            } else if (st == RANKY_E_BUSY) {
                busy.fetch_add(1);
                std::this_thread::sleep_for(std::chrono::microseconds(200));
            } else if (st == RANKY_E_NOMEM) {
                nomem.fetch_add(1);
            } else {
                error("unexpected submit status");
            }
        }
    };
    std::vector<std::thread> subs;
    for (int s = 0; s < 3; ++s) subs.emplace_back(submitter, 1234 + s);
    for (auto &t : subs) t.join();

    int ok = 0, cancelled = 0, failed = 0;
    for (uint64_t t : tickets) {
        ranky_info info;
        std::memset(&info, 0, sizeof(info));
        const ranky_status st = sched.wait(t, -1, &info);
        if (st == RANKY_OK) {
            ++ok;
            if (info.rank != (int32_t)t) error("info of another request");
            if (!info.lonely_per_block || !info.single_per_block) error("missing per-block counts");
            else
                for (int b = 0; b < info.n_blocks; ++b)
                    if (info.lonely_per_block[b] != (int32_t)(t + b) || info.single_per_block[b] != (int32_t)(2 * t + b))
                        error("per-block counts of another request");
        } else if (st == RANKY_E_CANCELLED) {
            ++cancelled;
        } else if (st == RANKY_E_NOT_CONVERGED) {
            ++failed;
        } else {
            error("unexpected final status");
        }
        if (sched.poll(t, nullptr) != st) error("poll disagrees with wait");
    }
    ranky_serve_summary s;
    sched.stats(&s);
    sched.stop();
    if (s.completed != ok || s.cancelled != cancelled || s.failed != failed) error("counters disagree");
    if (s.submitted != (int64_t)tickets.size()) error("submitted count");
    if (ok + cancelled + failed != (int)tickets.size()) error("a ticket without a final state");
    if (s.peak_running > kSlots || g_max_running.load() > kSlots) error("more running than slots");
    if (sched.arena_used() != 0) error("arena not empty at the end");
    if (s.rejected != busy.load() + nomem.load()) error("rejected count");
    std::printf("requests %zu ok %d cancelled %d failed %d busy %d nomem %d peak %lld p50 %.0f us errors %d\n",
                tickets.size(), ok, cancelled, failed, busy.load(), nomem.load(), (long long)s.peak_running, s.p50_us,
                g_errors.load());
    return g_errors.load() == 0 ? 0 : 1;
}
