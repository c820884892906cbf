// merge_host.cpp -- the host worker that scatters staged dirty granules
// into the host replica (double-buffered merge).
#include "merge_host.h"

#include <emmintrin.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "hetm.h"

namespace hetm {

namespace {

struct Job {
    hipEvent_t ready;
    const uint32_t *ids;
    const uint8_t *data;
    uint64_t n;
    uint8_t *host;
    uint64_t gbytes;
    uint64_t total;
    uint64_t seq;
};

// Granules [lo, hi) of the job.  A granule of whole 16-byte lines goes out
// with streaming stores: it overwrites its destination lines entirely, so
// reading them first would only double the host memory traffic.
void scatter_range(const Job &j, uint64_t lo, uint64_t hi) {
    const bool stream = j.gbytes % 16 == 0 && ((uintptr_t)j.host % 16) == 0;
    for (uint64_t i = lo; i < hi; ++i) {
        const uint64_t off = (uint64_t)j.ids[i] * j.gbytes;
        if (off >= j.total) continue;
        const uint64_t len = std::min(j.gbytes, j.total - off);
        const uint8_t *s = j.data + i * j.gbytes;
        uint8_t *d = j.host + off;
        if (stream && len == j.gbytes) {
            for (uint64_t k = 0; k < len; k += 16)
                _mm_stream_si128((__m128i *)(d + k), _mm_loadu_si128((const __m128i *)(s + k)));
        } else {
            memcpy(d, s, len);
        }
    }
    _mm_sfence();
}

// Persistent helpers of the merge worker: a job is cut into `parts` equal
// slices of granules, slice 0 for the worker itself and slice k for helper
// k - 1.  One thread per 2 MiB of granules, at most kMaxParts: a random
// 64-byte scatter into host memory runs at ~6 GB/s per thread.
constexpr unsigned kMaxParts = 8;

struct ScatterPool {
    std::vector<std::thread> th;
    std::mutex m;
    std::condition_variable cv_go, cv_done;
    const Job *job = nullptr;
    unsigned parts = 0, pending = 0;
    uint64_t gen = 0;
    bool stop = false;

    static void slice(const Job &j, unsigned parts, unsigned k) {
        const uint64_t per = (j.n + parts - 1) / parts;
        const uint64_t lo = std::min(j.n, (uint64_t)k * per), hi = std::min(j.n, lo + per);
        scatter_range(j, lo, hi);
    }
    void helper(unsigned k) {   // takes slice k + 1
        uint64_t seen = 0;
        for (;;) {
            std::unique_lock<std::mutex> l(m);
            cv_go.wait(l, [&] { return stop || gen != seen; });
            if (stop) return;
            seen = gen;
            const Job *j = job;
            const unsigned p = parts;
            l.unlock();
            if (k + 1 < p) slice(*j, p, k + 1);
            l.lock();
            if (--pending == 0) cv_done.notify_one();
        }
    }
    // as many helpers as start (none if the system refuses threads)
    void start() {
        try {
            for (unsigned k = 0; k + 1 < kMaxParts; ++k) th.emplace_back([this, k] { helper(k); });
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
    }
    void scatter(const Job &j) {
        const uint64_t bytes = j.n * j.gbytes;
        const unsigned p = (unsigned)std::max<uint64_t>(
            1, std::min<uint64_t>(std::min<uint64_t>(kMaxParts, th.size() + 1), bytes >> 21));
        if (p == 1 || th.empty()) {
            scatter_range(j, 0, j.n);
            return;
        }
        {
            std::lock_guard<std::mutex> l(m);
            job = &j;
            parts = p;
            pending = (unsigned)th.size();
            ++gen;
        }
        cv_go.notify_all();
        slice(j, p, 0);
        std::unique_lock<std::mutex> l(m);
        cv_done.wait(l, [&] { return pending == 0; });
    }
};

}  // namespace

struct MergeWorker {
    std::mutex m;
    std::condition_variable cv_job, cv_done;
    std::deque<Job> q;
    uint64_t issued = 0, done = 0;
    int err = HETM_OK;
    double us_scatter = 0, us_wait = 0;
    bool stop = false;
    std::thread th;
    ScatterPool pool;

    void run() {
        for (;;) {
            Job j;
            {
                std::unique_lock<std::mutex> l(m);
                cv_job.wait(l, [&] { return stop || !q.empty(); });
                if (q.empty()) return;
                j = q.front();
            }
            const int e = !j.ready || hipEventSynchronize(j.ready) == hipSuccess ? HETM_OK : HETM_EDEVICE;
            const auto t0 = std::chrono::steady_clock::now();
            if (e == HETM_OK) pool.scatter(j);
            const double us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
            {
                std::lock_guard<std::mutex> l(m);
                us_scatter += us;
                q.pop_front();
                if (e != HETM_OK && err == HETM_OK) err = e;
                done = j.seq;
            }
            cv_done.notify_all();
        }
    }
};

MergeWorker *merge_worker_create() {
    MergeWorker *w = nullptr;
    try {
        w = new MergeWorker;
        w->pool.start();
        w->th = std::thread([w] { w->run(); });
        return w;
    } catch (...) {
        if (w) {
            w->pool.finish();
            delete w;
        }
        return nullptr;
    }
}

void merge_worker_destroy(MergeWorker *w) {
    if (!w) return;
    {
        std::lock_guard<std::mutex> l(w->m);
        w->stop = true;
    }
    w->cv_job.notify_all();
    w->th.join();
    w->pool.finish();
    delete w;
}

uint64_t merge_submit(MergeWorker *w, hipEvent_t ready, const uint32_t *ids, const uint8_t *data, uint64_t n,
                      uint8_t *host, uint64_t gbytes, uint64_t total_bytes) {
    uint64_t seq;
    {
        std::lock_guard<std::mutex> l(w->m);
        try {
            w->q.push_back(Job{ready, ids, data, n, host, gbytes, total_bytes, w->issued + 1});
        } catch (...) {
            return 0;
        }
        seq = ++w->issued;
    }
    w->cv_job.notify_one();
    return seq;
}

int merge_wait(MergeWorker *w, uint64_t seq) {
    std::unique_lock<std::mutex> l(w->m);
    if (w->done >= seq) return w->err;
    const auto t0 = std::chrono::steady_clock::now();
    w->cv_done.wait(l, [&] { return w->done >= seq; });
    w->us_wait += std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
    return w->err;
}

void merge_times(MergeWorker *w, double *us_scatter, double *us_wait) {
    std::lock_guard<std::mutex> l(w->m);
    *us_scatter = w->us_scatter;
    *us_wait = w->us_wait;
}

uint64_t merge_done(MergeWorker *w) {
    std::lock_guard<std::mutex> l(w->m);
    return w->done;
}

}  // namespace hetm
