// host_pool.h -- persistent helper threads for host-side loops of the
// serving path (packing a round's requests, settling its results).
#pragma once

#include <algorithm>
#include <condition_variable>
#include <cstdint>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace hetm {

// Persistent helper threads of the serving loop: run(n, grain, f) cuts
// [0, n) into up to (helpers + 1) slices of at least `grain` items and runs
// f(lo, hi) on each, slice 0 on the calling thread.  Threads that cannot be
// started are simply not there (fewer slices).
struct Pool {
    static constexpr unsigned kMaxThreads = 12;
    std::vector<std::thread> th;
    std::mutex m;
    std::condition_variable cv_go, cv_done;
    const std::function<void(uint64_t, uint64_t)> *fn = nullptr;
    uint64_t n = 0, per = 0, gen = 0;
    unsigned parts = 0, pending = 0;
    bool stop = false;

    void start() {
        try {
            for (unsigned k = 0; k + 1 < kMaxThreads; ++k) th.emplace_back([this, k] { helper(k); });
        } catch (...) {
        }
    }
    void finish() {
        {
            std::lock_guard<std::mutex> l(m);
            stop = true;
        }
        cv_go.notify_all();
        for (auto &x : th) x.join();
        th.clear();
    }
    void helper(unsigned k) {   // takes slice k + 1
        uint64_t seen = 0;
        for (;;) {
            std::unique_lock<std::mutex> l(m);
            cv_go.wait(l, [&] { return stop || gen != seen; });
            if (stop) return;
            seen = gen;
            const auto *f = fn;
            const uint64_t lo = std::min(n, (uint64_t)(k + 1) * per), hi = std::min(n, lo + per);
            const bool mine = k + 1 < parts && lo < hi;
            l.unlock();
            if (mine) (*f)(lo, hi);
            l.lock();
            if (--pending == 0) cv_done.notify_one();
        }
    }
    void run(uint64_t count, uint64_t grain, const std::function<void(uint64_t, uint64_t)> &f) {
        const unsigned p = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(th.size() + 1, count / grain));
        if (p == 1) {
            f(0, count);
            return;
        }
        {
            std::lock_guard<std::mutex> l(m);
            fn = &f;
            n = count;
            per = (count + p - 1) / p;
            parts = p;
            pending = (unsigned)th.size();
            ++gen;
        }
        cv_go.notify_all();
        f(0, std::min(count, per));
        std::unique_lock<std::mutex> l(m);
        cv_done.wait(l, [&] { return pending == 0; });
    }
};

}  // namespace hetm
