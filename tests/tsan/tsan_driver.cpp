// Drives the library's threaded host code -- the host TM's worker threads
// and the merge worker with its scatter pool -- for a build with
// ThreadSanitizer, without a GPU: merge jobs are host-only (no event to wait
// for), so the HIP runtime is never entered.  Exits 0 when every check
// holds; any data race is reported by the sanitizer itself.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <random>
#include <thread>
#include <vector>

#include "hetm.h"
#include "host_pool.h"
#include "merge_host.h"

// The worker only synchronizes on events of jobs that carry one; this build
// submits none, and a call here would mean otherwise.
hipError_t hipEventSynchronize(hipEvent_t) {
    fprintf(stderr, "hipEventSynchronize called by a host-only job\n");
    abort();
}

#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            exit(1);                                               \
        }                                                          \
    } while (0)

// Bank transfers on 8 threads over a small, skewed account set (heavy lock
// contention), three rounds; every round is checked against a serial replay
// in commit-timestamp order.
static void host_tm_transfers() {
    const uint64_t n_acc = 1 << 12, n = 1 << 15;
    std::vector<int64_t> bal(n_acc, 1000);
    hetm_host_tm *tm = nullptr;
    CHECK(hetm_host_tm_create(bal.data(), n_acc, 8, 4, 0, &tm) == HETM_OK);
    std::mt19937_64 g(7);
    for (int round = 0; round < 3; ++round) {
        std::vector<uint32_t> src(n), dst(n), amt(n);
        for (uint64_t i = 0; i < n; ++i) {
            // a quarter of the transfers touch the 16 hottest accounts
            src[i] = (uint32_t)((g() & 3) ? g() % n_acc : g() % 16);
            dst[i] = (uint32_t)((g() & 3) ? g() % n_acc : g() % 16);
            amt[i] = (uint32_t)(g() % 300);
        }
        const std::vector<int64_t> before = bal;
        const uint64_t clock0 = hetm_host_tm_clock(tm);
        std::vector<uint64_t> ts(n);
        std::vector<hetm_log_entry8> log(2 * n);
        uint64_t n_log = 0;
        CHECK(hetm_host_run_transfers(tm, src.data(), dst.data(), amt.data(), n, 8, ts.data(), log.data(), log.size(),
                                      &n_log) == HETM_OK);
        CHECK(std::accumulate(bal.begin(), bal.end(), (int64_t)0) == (int64_t)(1000 * n_acc));
        std::vector<uint64_t> order(n);
        std::iota(order.begin(), order.end(), 0);
        std::sort(order.begin(), order.end(), [&](uint64_t a, uint64_t b) { return ts[a] < ts[b]; });
        for (uint64_t k = 0; k < n; ++k) {
            CHECK(ts[order[k]] > clock0 && ts[order[k]] <= hetm_host_tm_clock(tm));
            if (k) CHECK(ts[order[k]] != ts[order[k - 1]]);
        }
        std::vector<int64_t> serial = before;
        uint64_t applied = 0;
        for (uint64_t k : order) {
            if (src[k] != dst[k] && serial[src[k]] >= (int64_t)amt[k]) {
                serial[src[k]] -= amt[k];
                serial[dst[k]] += amt[k];
                ++applied;
            }
        }
        CHECK(serial == bal);
        CHECK(n_log == 2 * applied);
    }
    CHECK(hetm_host_tm_free(tm) == HETM_OK);
}

// Cache PUTs on 8 threads into a small cache (many collisions per set).
static void host_tm_cache_puts() {
    const uint64_t n_words = 128 * 64, n = 1 << 14;
    std::vector<uint32_t> cache(n_words, 0);
    hetm_host_tm *tm = nullptr;
    CHECK(hetm_host_tm_create(cache.data(), n_words, 4, 1, 100, &tm) == HETM_OK);
    std::mt19937_64 g(11);
    std::vector<uint64_t> keys(n), ts(n);
    for (auto &k : keys) k = 1 + g() % 5000;
    std::vector<hetm_log_entry4> log(12 * n);
    uint64_t n_log = 0;
    CHECK(hetm_host_run_cache_puts(tm, keys.data(), n, 8, ts.data(), log.data(), log.size(), &n_log) == HETM_OK);
    CHECK(n_log == 12 * n);
    std::vector<uint64_t> s = ts;
    std::sort(s.begin(), s.end());
    CHECK(std::adjacent_find(s.begin(), s.end()) == s.end());
    CHECK(s.front() > 100 && s.back() == hetm_host_tm_clock(tm));
    CHECK(hetm_host_tm_free(tm) == HETM_OK);
}

// The merge worker: 24 host-only jobs of 2^17 to 2^18 granules of 64 bytes
// (8 to 16 MiB, so the scatter pool splits them across its helpers) into
// a 64 MiB replica, waited on in turn, while a second thread polls the
// worker's counters.  The replica ends as the jobs applied in order.
static void merge_worker() {
    const uint64_t gbytes = 64, n_gran = 1 << 20, total = n_gran * gbytes;
    std::vector<uint8_t> host(total, 0), expect(total, 0);
    hetm::MergeWorker *w = hetm::merge_worker_create();
    CHECK(w != nullptr);
    std::atomic<bool> stop{false};
    std::thread poller([&] {
        uint64_t last = 0;
        while (!stop.load()) {
            const uint64_t d = hetm::merge_done(w);
            CHECK(d >= last);
            last = d;
            double a, b;
            hetm::merge_times(w, &a, &b);
        }
    });
    std::mt19937_64 g(3);
    struct Buf {
        std::vector<uint32_t> ids;
        std::vector<uint8_t> data;
        uint64_t seq = 0;
    } bufs[2];
    std::vector<uint32_t> pool(n_gran + 64);
    std::iota(pool.begin(), pool.end(), 0u);
    for (int job = 0; job < 24; ++job) {
        Buf &b = bufs[job & 1];
        if (b.seq) CHECK(hetm::merge_wait(w, b.seq) == HETM_OK);   // the buffer is free again
        const uint64_t n = (1 << 17) + g() % (1 << 17);
        b.ids.resize(n);
        b.data.resize(n * gbytes);
        // distinct ids within a job, as a compaction of dirty granules gives;
        // some past the end, which the worker clips
        std::shuffle(pool.begin(), pool.end(), g);
        for (uint64_t i = 0; i < n; ++i) {
            b.ids[i] = pool[i];
            memset(&b.data[i * gbytes], (int)((job * 31 + i) & 0xFF), gbytes);
        }
        // the serial effect: jobs in submission order
        for (uint64_t i = 0; i < n; ++i)
            if (b.ids[i] < n_gran) memcpy(&expect[(uint64_t)b.ids[i] * gbytes], &b.data[i * gbytes], gbytes);
        b.seq = hetm::merge_submit(w, nullptr, b.ids.data(), b.data.data(), n, host.data(), gbytes, total);
        CHECK(b.seq == (uint64_t)job + 1);
    }
    CHECK(hetm::merge_wait(w, 24) == HETM_OK);
    stop.store(true);
    poller.join();
    hetm::merge_worker_destroy(w);
    CHECK(host == expect);
}

// The serving path's helper pool: 2000 runs of random sizes and grains, each
// index visited exactly once, slices written by whichever thread owns them.
static void serve_pool() {
    hetm::Pool pool;
    pool.start();
    std::mt19937_64 g(5);
    std::vector<uint32_t> hits(1 << 14);
    for (int r = 0; r < 2000; ++r) {
        const uint64_t n = g() % (hits.size() + 1), grain = 1 + g() % 4096;
        std::fill(hits.begin(), hits.end(), 0u);
        pool.run(n, grain, [&](uint64_t lo, uint64_t hi) {
            for (uint64_t i = lo; i < hi; ++i) ++hits[i];
        });
        for (uint64_t i = 0; i < hits.size(); ++i) CHECK(hits[i] == (i < n ? 1u : 0u));
    }
    pool.finish();
}

int main() {
    serve_pool();
    host_tm_transfers();
    host_tm_cache_puts();
    merge_worker();
    printf("tsan driver: all checks passed\n");
    return 0;
}
