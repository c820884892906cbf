// host_tm.cpp -- the host side of a SHeTM round as plain C++ threads: worker
// threads run transactions on the host replica and, at commit, append the
// <word, value, timestamp> of every word they updated to a thread-local log
// (§IV-B, CPU instrumentation).  The round's log is the concatenation of the
// thread logs, in no particular order (§IV-C.2 applies it by timestamp).
//
// Concurrency control is two-phase locking over per-stripe spinlocks taken
// in ascending stripe order; the commit timestamp comes from one global
// clock incremented while the transaction holds its locks, so timestamps
// totally order the updates of every word, as the paper requires of a guest
// TM.  Every transaction (also one that writes nothing) gets a timestamp, so
// the host side can be replayed serially in timestamp order.
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "hetm.h"

struct hetm_host_tm {
    void *H = nullptr;
    uint64_t n_words = 0;
    uint32_t word_bytes = 4;
    uint32_t stripe_shift = 0;
    std::atomic<uint8_t> *locks = nullptr;
    uint64_t n_locks = 0;
    std::atomic<uint64_t> clock{0};
};

namespace {

struct Guard {
    std::atomic<uint8_t> *l[2];
    int n = 0;
    void lock(std::atomic<uint8_t> *p) {
        for (;;) {
            uint8_t z = 0;
            if (p->compare_exchange_weak(z, 1, std::memory_order_acquire)) break;
            while (p->load(std::memory_order_relaxed)) std::this_thread::yield();
        }
        l[n++] = p;
    }
    ~Guard() {
        for (int i = n - 1; i >= 0; --i) l[i]->store(0, std::memory_order_release);
    }
};

template <typename Fn>
void parallel_for(uint64_t n, uint32_t threads, Fn fn) {
    if (threads <= 1 || n < 2) {
        fn(0, 0, n);
        return;
    }
    std::vector<std::thread> ts;
    ts.reserve(threads);
    const uint64_t per = (n + threads - 1) / threads;
    for (uint32_t t = 0; t < threads; ++t) {
        const uint64_t lo = t * per, hi = std::min(n, lo + per);
        if (lo >= hi) break;
        try {
            ts.emplace_back(fn, t, lo, hi);
        } catch (...) {
            fn(t, lo, hi);   // no thread to spare: this slice runs here
        }
    }
    for (auto &t : ts) t.join();
}

uint64_t mix64(uint64_t z) {   // splitmix64 finalizer
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

}  // namespace

extern "C" {

int hetm_host_tm_create(void *host_replica, uint64_t n_words, uint32_t word_bytes, uint32_t lock_stripe_words,
                        uint64_t ts_start, hetm_host_tm **out) {
    if (!host_replica || !out || n_words == 0 || (word_bytes != 4 && word_bytes != 8) || lock_stripe_words == 0 ||
        (lock_stripe_words & (lock_stripe_words - 1)))
        return HETM_EINVAL;
    hetm_host_tm *t = new (std::nothrow) hetm_host_tm();
    if (!t) return HETM_ENOMEM;
    t->H = host_replica;
    t->n_words = n_words;
    t->word_bytes = word_bytes;
    while ((1u << t->stripe_shift) < lock_stripe_words) ++t->stripe_shift;
    t->n_locks = ((n_words - 1) >> t->stripe_shift) + 1;
    t->locks = new (std::nothrow) std::atomic<uint8_t>[t->n_locks];
    if (!t->locks) {
        delete t;
        return HETM_ENOMEM;
    }
    for (uint64_t i = 0; i < t->n_locks; ++i) t->locks[i].store(0, std::memory_order_relaxed);
    t->clock.store(ts_start);
    *out = t;
    return HETM_OK;
}

int hetm_host_tm_free(hetm_host_tm *t) {
    if (!t) return HETM_EINVAL;
    delete[] t->locks;
    delete t;
    return HETM_OK;
}

uint64_t hetm_host_tm_clock(hetm_host_tm *t) { return t ? t->clock.load() : 0; }

int hetm_host_run_transfers(hetm_host_tm *t, const uint32_t *src, const uint32_t *dst, const uint32_t *amt,
                            uint64_t n, uint32_t n_threads, uint64_t *ts_out, hetm_log_entry8 *log_out,
                            uint64_t log_capacity, uint64_t *n_log_out) {
    if (!t || t->word_bytes != 8 || (n && (!src || !dst || !amt || !ts_out)) || !n_log_out) return HETM_EINVAL;
    for (uint64_t i = 0; i < n; ++i)
        if (src[i] >= t->n_words || dst[i] >= t->n_words) return HETM_EINVAL;
    int64_t *H = (int64_t *)t->H;
    if (n_threads == 0) n_threads = 1;
    // each slice's log reserved up front (two entries per transfer at most),
    // so the worker threads never allocate
    std::vector<std::vector<hetm_log_entry8>> logs;
    try {
        logs.resize(n_threads);
        for (auto &lg : logs) lg.reserve(2 * ((n + n_threads - 1) / n_threads));
    } catch (...) {
        return HETM_ENOMEM;
    }
    parallel_for(n, n_threads, [&](uint32_t tid, uint64_t lo, uint64_t hi) {
        auto &lg = logs[tid];
        for (uint64_t i = lo; i < hi; ++i) {
            const uint32_t s = src[i], d = dst[i];
            const uint64_t ls = s >> t->stripe_shift, ld = d >> t->stripe_shift;
            Guard g;
            g.lock(&t->locks[std::min(ls, ld)]);
            if (ls != ld) g.lock(&t->locks[std::max(ls, ld)]);
            const int64_t bs = H[s], bd = H[d];
            const bool applied = s != d && bs >= (int64_t)amt[i];
            const uint64_t ts = t->clock.fetch_add(1) + 1;
            if (applied) {
                H[s] = bs - (int64_t)amt[i];
                H[d] = bd + (int64_t)amt[i];
                lg.push_back({s, 0u, (uint64_t)H[s], ts});
                lg.push_back({d, 0u, (uint64_t)H[d], ts});
            }
            ts_out[i] = ts;
        }
    });
    uint64_t m = 0;
    for (auto &lg : logs) m += lg.size();
    *n_log_out = m;
    if (m > log_capacity || (m && !log_out)) return HETM_ECAPACITY;
    for (auto &lg : logs) {
        if (!lg.empty()) memcpy(log_out, lg.data(), lg.size() * sizeof(hetm_log_entry8));
        log_out += lg.size();
    }
    return HETM_OK;
}

// PUTs into the set-associative cache layout of the CACHE program (one
// 128-word record per set) with stamp = (uint32_t)ts; each PUT logs the 12
// words it writes (key 2, value 8, way stamp, set PUT stamp).  The lock
// covering the set's first word guards the whole set.
int hetm_host_run_cache_puts(hetm_host_tm *t, const uint64_t *keys, uint64_t n, uint32_t n_threads,
                             uint64_t *ts_out, hetm_log_entry4 *log_out, uint64_t log_capacity,
                             uint64_t *n_log_out) {
    if (!t || t->word_bytes != 4 || (n && (!keys || !ts_out)) || !n_log_out) return HETM_EINVAL;
    const uint64_t nsets = t->n_words / 128;
    if (t->n_words % 128 || nsets < 2 || (nsets & (nsets - 1))) return HETM_EINVAL;
    for (uint64_t i = 0; i < n; ++i)
        if (keys[i] == 0) return HETM_EINVAL;
    uint32_t *H = (uint32_t *)t->H;
    if (n_threads == 0) n_threads = 1;
    // each slice's log reserved up front (twelve entries per PUT), so the
    // worker threads never allocate
    std::vector<std::vector<hetm_log_entry4>> logs;
    try {
        logs.resize(n_threads);
        for (auto &lg : logs) lg.reserve(12 * ((n + n_threads - 1) / n_threads));
    } catch (...) {
        return HETM_ENOMEM;
    }
    parallel_for(n, n_threads, [&](uint32_t tid, uint64_t lo, uint64_t hi) {
        auto &lg = logs[tid];
        for (uint64_t i = lo; i < hi; ++i) {
            const uint64_t key = keys[i];
            const uint64_t set = (mix64(key) & (nsets - 1) & ~1ull) | (key & 1ull);
            const uint64_t base = set * 128;
            Guard g;
            g.lock(&t->locks[base >> t->stripe_shift]);
            const uint64_t ts = t->clock.fetch_add(1) + 1;
            const uint32_t stamp = (uint32_t)ts;
            uint32_t *rec = H + base;
            int hit = -1;
            for (int w = 0; w < 8 && hit < 0; ++w)
                if (((uint64_t)rec[2 * w] | ((uint64_t)rec[2 * w + 1] << 32)) == key) hit = w;
            uint32_t victim = 0;
            for (uint32_t w = 1; w < 8; ++w)
                if (rec[16 + w] < rec[16 + victim]) victim = w;
            if (hit >= 0) victim = (uint32_t)hit;
            uint32_t v[8], chk = (uint32_t)mix64(key);
            for (uint32_t k = 0; k < 7; ++k) {
                v[k] = (uint32_t)mix64(key ^ ((uint64_t)stamp << 32) ^ k);
                chk ^= v[k];
            }
            v[7] = chk;
            const uint32_t words[12] = {2 * victim, 2 * victim + 1, 32 + 8 * victim, 33 + 8 * victim,
                                        34 + 8 * victim, 35 + 8 * victim, 36 + 8 * victim, 37 + 8 * victim,
                                        38 + 8 * victim, 39 + 8 * victim, 16 + victim, 24};
            rec[2 * victim] = (uint32_t)key;
            rec[2 * victim + 1] = (uint32_t)(key >> 32);
            for (uint32_t k = 0; k < 8; ++k) rec[32 + 8 * victim + k] = v[k];
            rec[16 + victim] = stamp;
            rec[24] = stamp;
            for (uint32_t k = 0; k < 12; ++k) lg.push_back({(uint32_t)(base + words[k]), rec[words[k]], ts});
            ts_out[i] = ts;
        }
    });
    uint64_t m = 0;
    for (auto &lg : logs) m += lg.size();
    *n_log_out = m;
    if (m > log_capacity || (m && !log_out)) return HETM_ECAPACITY;
    for (auto &lg : logs) {
        if (!lg.empty()) memcpy(log_out, lg.data(), lg.size() * sizeof(hetm_log_entry4));
        log_out += lg.size();
    }
    return HETM_OK;
}

}  // extern "C"
