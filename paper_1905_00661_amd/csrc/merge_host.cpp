// merge_host.cpp -- the host worker that scatters DMA-staged dirty granules
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

void scatter(const Job &j) {
    // one thread per 4 MiB of granules, at most 4 (the caller's threads need
    // the host's memory bandwidth too)
    const uint64_t bytes = j.n * j.gbytes;
    const unsigned t = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(4, bytes >> 22));
    if (t == 1) {
        scatter_range(j, 0, j.n);
        return;
    }
    std::vector<std::thread> th;
    const uint64_t per = (j.n + t - 1) / t;
    for (unsigned k = 1; k < t; ++k) {
        const uint64_t lo = std::min(j.n, k * per), hi = std::min(j.n, lo + per);
        th.emplace_back(scatter_range, std::cref(j), lo, hi);
    }
    scatter_range(j, 0, std::min(j.n, per));
    for (auto &x : th) x.join();
}

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

    void run() {
        for (;;) {
            Job j;
            {
                std::unique_lock<std::mutex> l(m);
                cv_job.wait(l, [&] { return stop || !q.empty(); });
                if (q.empty()) return;
                j = q.front();
            }
            const int e = hipEventSynchronize(j.ready) == hipSuccess ? HETM_OK : HETM_EDEVICE;
            const auto t0 = std::chrono::steady_clock::now();
            if (e == HETM_OK) scatter(j);
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
    auto *w = new MergeWorker;
    w->th = std::thread([w] { w->run(); });
    return w;
}

void merge_worker_destroy(MergeWorker *w) {
    if (!w) return;
    {
        std::lock_guard<std::mutex> l(w->m);
        w->stop = true;
    }
    w->cv_job.notify_all();
    w->th.join();
    delete w;
}

uint64_t merge_submit(MergeWorker *w, hipEvent_t ready, const uint32_t *ids, const uint8_t *data, uint64_t n,
                      uint8_t *host, uint64_t gbytes, uint64_t total_bytes) {
    uint64_t seq;
    {
        std::lock_guard<std::mutex> l(w->m);
        seq = ++w->issued;
        w->q.push_back(Job{ready, ids, data, n, host, gbytes, total_bytes, seq});
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
