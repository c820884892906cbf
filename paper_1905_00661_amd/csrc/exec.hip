// exec.hip -- execution phase (§IV-C.1): the GPU's local TM running a batch of
// transactions against the GPU replica of the STMR, with the read-set and
// write-set granule bitmaps of §IV-B updated by every committed transaction.
//
// Design (gfx950, wave64):
//  * One transaction per lane.  A wave pulls work from a device queue with
//    one atomic per refill, so finished or committed lanes take the next
//    transaction while conflicting lanes retry (persistent kernel).
//  * Lock table: one u64 per stripe of S words, bit 63 = lock, bits 0..62 =
//    version.  Reads are a batched seqlock: load every read stripe's lock
//    word, one acquire fence, load every value, so the number of fences per
//    attempt does not grow with the transaction's length.  The read set is
//    remembered as the sum of the versions seen (versions only grow, and a
//    round commits fewer than 2^32 times, so equal sums mean equal versions).
//  * Commit: try-lock each distinct write stripe with a 64-bit CAS (a lane
//    never waits on a lock, so lanes of one wave cannot deadlock), take a
//    commit ticket (one atomic per wave, lanes ranked by mbcnt), re-load the
//    read stripes' lock words and compare with the first pass, write the
//    LDS-staged write buffer, release with version+1.  A lock acquired before
//    the ticket and a validation after it make ascending tickets a valid
//    serial order for update and read-only transactions alike.
//  * Bitmaps are set only by the committed attempt: the read-set bitmap gets
//    every word read or written (writes included, so WS is within RS and the
//    validation also excludes write-write conflicts, §IV-C.2).
//  * Two layouts of the replica.  Split: a value array plus a lock table of
//    one word per stripe of S words.  Slot (u32 words, S = 1): each word's
//    value, version and lock share one u64 (bits 0..31 value, 32..62
//    version, 63 lock), so one load returns a value together with the
//    version it belongs to, one store publishes a commit, and a read touches
//    one cache line instead of two.
#include "hetm_dev.h"

namespace hetm {

namespace {

// Replica layouts (see above).  lock(w) is the lock word covering word w,
// stripe(w) its identity, load(w) a device-coherent read of the value.
template <typename Word>
struct Split {
    gmem<Word> *vals;
    gmem<uint64_t> *locks;
    uint32_t sh;
    static constexpr bool kFused = false;
    __device__ gmem<uint64_t> *lock(uint32_t w) const { return &locks[w >> sh]; }
    __device__ uint32_t stripe(uint32_t w) const { return w >> sh; }
    __device__ Word load(uint32_t w) const { return ld_agent(&vals[w]); }
};

struct Slot {
    gmem<uint64_t> *slots;
    static constexpr bool kFused = true;
    __device__ gmem<uint64_t> *lock(uint32_t w) const { return &slots[w]; }
    __device__ uint32_t stripe(uint32_t w) const { return w; }
    __device__ uint32_t load(uint32_t w) const { return (uint32_t)ld_agent(&slots[w]); }
    static __device__ uint32_t version(uint64_t slot) { return (uint32_t)(slot >> 32) & 0x7FFFFFFFu; }
    // an unlocked slot: version above, value below
    static __device__ uint64_t make(uint32_t ver, uint32_t value) {
        return ((uint64_t)(ver & 0x7FFFFFFFu) << 32) | value;
    }
};

// Per-lane write buffer staged in LDS, [slot][lane] so that the 64 lanes of a
// wave touch 64 consecutive dwords per slot (no bank conflicts).
template <typename Word, int MAXW>
struct WriteBuf {
    uint32_t (*addr)[kWave];
    Word (*val)[kWave];
    uint32_t lane;
    uint32_t n;
    uint32_t locked;   // entries whose lock word this lane holds
    // slot layout, undo log: entries whose word had a version from before the
    // round (at most base_ver) when locked, and their values then
    uint32_t first = 0;
    uint32_t base_ver = 0xFFFFFFFFu;
    uint32_t prev[MAXW];

    __device__ void put(uint32_t w, Word v) {
        addr[n][lane] = w;
        val[n][lane] = v;
        ++n;
    }
    __device__ uint32_t at(uint32_t k) const { return addr[k][lane]; }

    // Try-lock every distinct lock word in ascending stripe order (so two
    // lanes wanting the same stripes collide on the first one instead of each
    // holding one of them in lockstep); on failure release what was taken.
    template <typename Lay>
    __device__ bool lock_all(const Lay &lay) {
        locked = 0;
        first = 0;
        int64_t last = -1;
        for (;;) {
            uint32_t kmin = n;
            uint32_t smin = 0;
            for (uint32_t k = 0; k < n; ++k) {
                const uint32_t s = lay.stripe(at(k));
                if ((int64_t)s > last && (kmin == n || s < smin)) {
                    kmin = k;
                    smin = s;
                }
            }
            if (kmin == n) return true;
            gmem<uint64_t> *p = lay.lock(at(kmin));
            uint64_t cur = ld_agent(p);
            if ((cur & kLockBit) || !cas_agent(p, cur, cur | kLockBit)) {
                abort(lay);
                return false;
            }
            locked |= 1u << kmin;
            if constexpr (Lay::kFused) {
#pragma unroll
                for (int k = 0; k < MAXW; ++k)
                    if ((uint32_t)k == kmin) prev[k] = (uint32_t)cur;
                if (Slot::version(cur) <= base_ver) first |= 1u << kmin;
            }
            last = smin;
        }
    }
    template <typename Lay>
    __device__ bool mine(const Lay &lay, uint32_t s) const {
        for (uint32_t k = 0; k < n; ++k)
            if (((locked >> k) & 1u) && lay.stripe(at(k)) == s) return true;
        return false;
    }
    // unlock with the version unchanged
    template <typename Lay>
    __device__ void abort(const Lay &lay) {
        for (uint32_t k = 0; k < n; ++k)
            if ((locked >> k) & 1u)
                __hip_atomic_fetch_and(lay.lock(at(k)), ~kLockBit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        locked = 0;
    }
    // Publish the buffered writes.  Split: store every value, then release
    // each held stripe with version + 1.  Slot: one store per held word
    // writes value, version + 1 and the cleared lock together (duplicate
    // entries of a word carry the same value, so the held one suffices).
    __device__ void commit(const Split<Word> &lay) {
        for (uint32_t k = 0; k < n; ++k) st_agent(&lay.vals[at(k)], val[k][lane]);
        hw_order();
        for (uint32_t k = 0; k < n; ++k)
            if ((locked >> k) & 1u)
                __hip_atomic_fetch_add(lay.lock(at(k)), 1ull - kLockBit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        locked = 0;
    }
    // Slot: one store per held word writes the value, the writer's version
    // and the cleared lock together (duplicate entries of a word carry the
    // same value, so the held one suffices)
    __device__ void commit(const Slot &lay, uint32_t ver) {
        for (uint32_t k = 0; k < n; ++k)
            if ((locked >> k) & 1u) st_agent(lay.lock(at(k)), Slot::make(ver, (uint32_t)val[k][lane]));
        locked = 0;
    }
    __device__ void mark_writes(gmem<uint8_t> *rs, gmem<uint32_t> *ws, const Div32 &G) {
        for (uint32_t k = 0; k < n; ++k) {
            uint32_t g = div32(at(k), G);
            rs_mark(rs, g);
            bitmap_set(ws, g);
        }
    }
};

// Revalidation of one read word after the ticket: returns its lock word
// without the lock bit, or sets ok = false if another transaction holds it.
template <typename Lay, typename WB>
__device__ __forceinline__ uint64_t reread(const Lay &lay, uint32_t w, const WB &wb, bool &ok) {
    uint64_t l = ld_agent(lay.lock(w));
    if (l & kLockBit) {
        if (!wb.mine(lay, lay.stripe(w))) ok = false;
        l &= ~kLockBit;
    }
    return l;
}

// Per-lane bookkeeping of the persistent loop.
struct LaneState {
    uint32_t txn = kNoTxn;
    uint32_t attempts = 0;
    uint32_t wait = 0;      // loop iterations to sit out after a local abort
    uint64_t commits = 0;
    uint64_t retries = 0;
};

// Contention manager: after its k-th local abort a transaction sits out a
// pseudo-random number of iterations below min(2^k, 256).  Lanes of one wave
// run in lockstep, so two transactions that each write what the other read
// would otherwise abort each other identically forever; the random wait
// breaks the symmetry.
__device__ __forceinline__ uint32_t backoff(uint32_t txn, uint32_t attempts) {
    uint32_t h = txn * 0x9E3779B1u ^ attempts * 0x85EBCA77u;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    const uint32_t window = attempts >= 8 ? 256u : (1u << attempts);
    return h & (window - 1);
}

// Whether this lane runs an attempt in this iteration (it has a transaction
// and is not backing off).
__device__ __forceinline__ bool lane_turn(LaneState &ls, uint32_t n) {
    if (ls.txn >= n) return false;
    if (ls.wait) {
        --ls.wait;
        return false;
    }
    return true;
}

// Lane g of the grid starts with transaction g; later work comes from the
// device queue, which hands out transactions n_lanes, n_lanes+1, ...
__device__ __forceinline__ LaneState first_txn(uint32_t n) {
    LaneState ls;
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    ls.txn = g < n ? g : kDoneTxn;
    return ls;
}

// Refill lanes without work from the device queue; returns false when the
// whole wave is out of work.  Reached by all 64 lanes.
__device__ __forceinline__ bool refill(LaneState &ls, HotCounters *hot, uint32_t n) {
    const bool need = ls.txn == kNoTxn;
    if (__ballot(need)) {
        const uint32_t got = wave_fetch_add(&hot->queue_head.v, need);
        if (need) {
            const uint64_t t = (uint64_t)gridDim.x * blockDim.x + got;
            ls.txn = t < n ? (uint32_t)t : kDoneTxn;
            ls.attempts = 0;
        }
    }
    return __ballot(ls.txn < n) != 0;
}

// OPLIST work split.  A wave whose lanes mix read-only transactions and
// updates runs every attempt at the pace of its update lanes (try-locks,
// the clock draw, revalidation) while the read-only lanes wait; at one
// update in ten, nearly every wave of 64 holds several.  So k_partition
// splits the batch into a read-only list (the front of `order`) and an
// update list (its back), and each wave draws from one list until that
// runs dry, then from the other.  Serializability does not depend on which
// transactions run together.
struct KindQueues {
    const gmem<uint32_t> *order;
    uint32_t n, n_ro, n_upd;
    bool upd;   // wave-uniform: the list this wave draws from
};

__device__ __forceinline__ KindQueues kind_queues(const DevArgs *a) {
    KindQueues q;
    q.order = glob(a->order);
    q.n = a->n_txns;
    q.n_ro = ld_agent(&a->hot->n_ro.v);
    q.n_upd = ld_agent(&a->hot->n_upd.v);
    // Update waves get a share of the grid 2.5x the update share of the
    // batch, at least one if there are updates; the first wave of every
    // workgroup comes first, which spreads them over the compute units.
    // Measured on 2^20 transactions with one update in ten: 683 us at 0.5x,
    // 653 at 1x and 1.5x, 600 at 2.5x, 608 at 4x, 621 at 6x and beyond
    // (where updates all run first): an update attempt takes longer, and
    // updates finishing early leave the read-only tail free of writers.
    const uint32_t waves = gridDim.x * kExecWaves;
    const uint32_t rank = (threadIdx.x / kWave) * gridDim.x + blockIdx.x;
    uint32_t upd_waves = 0;
    if (q.n_upd) {
        const uint64_t w = (5ull * q.n_upd * waves + 2ull * q.n - 1) / (2ull * q.n);
        upd_waves = (uint32_t)(w < 1 ? 1 : (w > waves ? waves : w));
    }
    q.upd = rank < upd_waves;
    return q;
}

// Refill lanes without work from the wave's list, switching the wave to the
// other list for good once its own is used up; returns false when the whole
// wave is out of work.  Reached by all 64 lanes.
__device__ __forceinline__ bool refill(LaneState &ls, KindQueues &q, HotCounters *hot) {
    bool need = ls.txn == kNoTxn;
    for (int pass = 0; pass < 2 && __ballot(need); ++pass) {
        const bool upd = q.upd;
        const uint32_t lim = upd ? q.n_upd : q.n_ro;
        const uint32_t got = wave_fetch_add(upd ? &hot->queue_upd.v : &hot->queue_head.v, need);
        if (need && got < lim) {
            ls.txn = upd ? q.order[q.n - 1 - got] : q.order[got];
            ls.attempts = 0;
            need = false;
        }
        if (__ballot(need)) q.upd = !upd;
    }
    if (need) ls.txn = kDoneTxn;   // both lists used up
    return __ballot(ls.txn < q.n) != 0;
}

// After an attempt: account, then free the lane on commit, retry cap, or a
// malformed transaction (already latched as HETM_EINVAL, never executed).
__device__ __forceinline__ void settle(LaneState &ls, bool act, bool malformed, bool ok, uint32_t ticket,
                                       uint32_t *tickets, DevCounters *cnt, uint32_t retry_cap) {
    if (malformed) {
        ls.txn = kNoTxn;
    } else if (ok) {
        tickets[ls.txn] = ticket;
        ls.commits++;
        ls.txn = kNoTxn;
    } else if (act) {
        ls.retries++;
        if (++ls.attempts >= retry_cap) {
            latch_error(cnt, HETM_ERETRY, ls.txn);
            ls.txn = kNoTxn;
        } else {
            ls.wait = backoff(ls.txn, ls.attempts);
        }
    }
}

__device__ __forceinline__ void flush_counts(const LaneState &ls, DevCounters *cnt) {
    unsigned long long c = ls.commits, r = ls.retries;
    for (int o = 32; o > 0; o >>= 1) {
        c += __shfl_xor(c, o);
        r += __shfl_xor(r, o);
    }
    if (lane_id() == 0) {
        if (c) __hip_atomic_fetch_add(&cnt->committed, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (r) __hip_atomic_fetch_add(&cnt->retries, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Early validation doomed this round (§IV-D): the CPU wins, so the rest of
// the batch is not worth executing.  The round is marked conflicted here, so
// the skipped transactions can never be reported as committed even if the
// chunk that doomed it is left out of the final validation.  Checked at the
// top of the loop, where a lane holds no lock; the flag is wave-uniform.
__device__ __forceinline__ bool doomed(DevCounters *cnt, uint32_t epoch) {
    const uint32_t d = __builtin_amdgcn_readfirstlane(ld_agent(&cnt->doomed));
    if (d != epoch) return false;
    if (lane_id() == 0) st_agent(&cnt->conflict, 1u);
    return true;
}
// The same with the flag loaded earlier (one iteration's latency hidden).
__device__ __forceinline__ bool doomed(DevCounters *cnt, uint32_t epoch, uint32_t loaded) {
    if (__builtin_amdgcn_readfirstlane(loaded) != epoch) return false;
    if (lane_id() == 0) st_agent(&cnt->conflict, 1u);
    return true;
}

template <typename Lay>
__device__ __forceinline__ Lay make_layout(const DevArgs *a);
template <>
__device__ __forceinline__ Slot make_layout<Slot>(const DevArgs *a) {
    return Slot{glob((uint64_t *)a->stmr)};
}
template <>
__device__ __forceinline__ Split<uint32_t> make_layout<Split<uint32_t>>(const DevArgs *a) {
    return Split<uint32_t>{glob((uint32_t *)a->stmr), glob(a->locks), a->stripe_shift};
}
template <>
__device__ __forceinline__ Split<uint64_t> make_layout<Split<uint64_t>>(const DevArgs *a) {
    return Split<uint64_t>{glob((uint64_t *)a->stmr), glob(a->locks), a->stripe_shift};
}

// ------------------------------------------------------------------ OPLIST
// Transaction i reads idx[off[i] .. off[i+1]) in order, then writes each of
// its first nw[i] words with (value read + tid[i]) mod 2^32.
// An attempt loads its word list from HBM once, into LDS ([op][lane] per
// wave, max_ops x 64 dwords, dynamic), and every later pass -- lock words,
// values, revalidation, bitmaps -- reads it from there.
// Memory accesses of a pass go out in chunks of kChunk independent loads
// before any result is used, so a lane keeps kChunk requests in flight
// instead of waiting out each one in turn.  Lanes past their transaction's
// length load a word already in the chunk (a cache hit) instead of
// branching, which keeps the loads in one straight-line block.
constexpr uint32_t kChunk = 8;
static_assert(kChunk == 8, "the vector result stores cover a chunk of 8");
typedef uint32_t U32x4 __attribute__((ext_vector_type(4)));

template <typename Lay>
__global__ __launch_bounds__(kExecWaves *kWave) void k_exec_oplist(const DevArgs *__restrict__ a) {
    __shared__ uint32_t s_addr[kExecWaves][kOplistMaxWrites][kWave];
    __shared__ uint32_t s_val[kExecWaves][kOplistMaxWrites][kWave];
    extern __shared__ uint32_t s_dyn[];
    const uint32_t wv = threadIdx.x / kWave;
    const Lay lay = make_layout<Lay>(a);
    gmem<uint8_t> *rs = glob(a->rs);
    gmem<uint32_t> *ws = glob(a->ws);
    DevCounters *cnt = a->cnt;
    const uint32_t n = a->n_txns, max_ops = a->max_ops;
    const Div32 G = a->gdiv;
    const uint64_t N = a->n_words;
    const gmem<uint32_t> *off = glob(a->off), *idx = glob(a->idx), *tid = glob(a->tid);
    const gmem<uint8_t> *nw = glob(a->nw);
    gmem<uint32_t> *res = glob((uint32_t *)a->results);
    const bool res_aligned = ((uintptr_t)a->results & 15u) == 0;
    const bool idx_aligned = ((uintptr_t)a->idx & 15u) == 0;
    WriteBuf<uint32_t, kOplistMaxWrites> wb{s_addr[wv], s_val[wv], lane_id(), 0, 0};
    uint32_t *ix = s_dyn + wv * max_ops * kWave + lane_id();     // ix[j * kWave]: word j of this lane's txn
    const uint32_t epoch = a->epoch;
    const uint32_t clock_base = ld_agent(&cnt->clock_base);
    LaneState ls;                               // every lane starts without a transaction
    KindQueues q = kind_queues(a);
    uint32_t doom = ld_agent(&cnt->doomed);   // the doom flag, loaded one iteration ahead of its check

    while (refill(ls, q, a->hot)) {
        const bool act = lane_turn(ls, n);
        if (doomed(cnt, epoch, doom)) break;
        doom = ld_agent(&cnt->doomed);     // in flight across this iteration, checked at the next
        if (!__ballot(act)) {          // every lane is backing off
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        // Slot layout: the attempt's clock snapshot is issued first, so its
        // latency (the clock line is contended) overlaps the loads of the
        // transaction's descriptor and word list
        const uint32_t rv_load = Lay::kFused ? ld_agent(&a->hot->clock.v) : 0u;
        uint32_t o = 0, L = 0, nwr = 0, tv = 0;
        bool malformed = false;
        if (act) {
            o = off[ls.txn];
            uint32_t e = off[ls.txn + 1];
            nwr = nw[ls.txn];
            tv = tid[ls.txn];
            L = e - o;
            malformed = e < o || L > max_ops || nwr > L || nwr > kOplistMaxWrites;
            if (malformed) L = 0;
            // the word list, into LDS (a chunk of eight 16-byte aligned
            // indices with two 16-byte loads)
            for (uint32_t j0 = 0; j0 < L; j0 += kChunk) {
                uint32_t w[kChunk];
                if (idx_aligned && j0 + kChunk <= L && ((o + j0) & 3u) == 0) {
                    const gmem<U32x4> *q = (const gmem<U32x4> *)(idx + o + j0);
                    const U32x4 q0 = q[0], q1 = q[1];
                    w[0] = q0.x; w[1] = q0.y; w[2] = q0.z; w[3] = q0.w;
                    w[4] = q1.x; w[5] = q1.y; w[6] = q1.z; w[7] = q1.w;
                } else {
#pragma unroll
                    for (uint32_t k = 0; k < kChunk; ++k) w[k] = idx[o + (j0 + k < L ? j0 + k : j0)];
                }
#pragma unroll
                for (uint32_t k = 0; k < kChunk; ++k)
                    if (j0 + k < L) {
                        ix[(j0 + k) * kWave] = w[k];
                        malformed |= w[k] >= N;
                    }
            }
            if (malformed) {
                latch_error(cnt, HETM_EINVAL, ls.txn);
                L = 0;
            }
        }
        bool ok = act && !malformed;
        wb.n = 0;
        uint32_t ticket;
        if constexpr (Lay::kFused) {
            // Slot layout, TL2-style: the wave takes one snapshot rv of the
            // version clock; a read is valid if its slot is unlocked and no
            // newer than rv, so one load per read returns a consistent
            // value.  A read-only transaction commits at rv with no lock,
            // ticket or second pass; an update locks its writes, draws its
            // write version wv from the clock and re-checks its reads only
            // if another writer drew in between (wv != rv).
            const uint32_t rv = __builtin_amdgcn_readfirstlane(rv_load);
            hw_order();   // the snapshot load has completed before any slot load issues
            uint64_t seen[kOplistMaxWrites];   // the written words' slots as this pass read them
            static_assert(kOplistMaxWrites <= kChunk, "the write entries are all in the first chunk");
            for (uint32_t j0 = 0; j0 < L; j0 += kChunk) {
                uint32_t w[kChunk];
                uint64_t l[kChunk];
#pragma unroll
                for (uint32_t k = 0; k < kChunk; ++k) w[k] = ix[(j0 + k < L ? j0 + k : j0) * kWave];
#pragma unroll
                for (uint32_t k = 0; k < kChunk; ++k) l[k] = ld_agent(lay.lock(w[k]));
                if (j0 == 0) {
#pragma unroll
                    for (uint32_t k = 0; k < kOplistMaxWrites; ++k) seen[k] = l[k];
                }
                // a whole chunk of results 16-byte aligned goes out in two 16-byte stores
                const bool vec = res_aligned && j0 + kChunk <= L && ((o + j0) & 3u) == 0;
#pragma unroll
                for (uint32_t k = 0; k < kChunk; ++k) {
                    const uint32_t j = j0 + k;
                    if (j < L) {
                        ok &= !(l[k] & kLockBit) && Slot::version(l[k]) <= rv;
                        const uint32_t v = (uint32_t)l[k];
                        if (!vec) res[o + j] = v;
                        if (j < nwr) wb.put(w[k], v + tv);
                    }
                }
                if (vec) {
                    gmem<U32x4> *r4 = (gmem<U32x4> *)(res + o + j0);
                    r4[0] = U32x4{(uint32_t)l[0], (uint32_t)l[1], (uint32_t)l[2], (uint32_t)l[3]};
                    r4[1] = U32x4{(uint32_t)l[4], (uint32_t)l[5], (uint32_t)l[6], (uint32_t)l[7]};
                }
            }
            const bool upd = nwr != 0;
            // Try-lock every distinct written word at once: a CAS from the
            // slot as the first pass read it (unlocked, version <= rv) to
            // the same slot with the lock bit.  Success means the word is
            // unchanged since the read; any failure aborts the attempt and
            // puts back exactly the slots taken.  No lane waits for a lock,
            // so the order of the CASes does not matter.  (With updates in
            // waves of their own this measured 589 us against 602 us for
            // locking one word at a time in ascending order, load then CAS.)
            if (ok && upd) {
                bool want[kOplistMaxWrites], got[kOplistMaxWrites];
#pragma unroll
                for (uint32_t k = 0; k < kOplistMaxWrites; ++k) {
                    bool dup = false;
#pragma unroll
                    for (uint32_t k2 = 0; k2 < k; ++k2) dup |= k2 < nwr && wb.at(k2) == wb.at(k);
                    want[k] = k < nwr && !dup;
                }
#pragma unroll
                for (uint32_t k = 0; k < kOplistMaxWrites; ++k)
                    got[k] = want[k] && cas_agent(lay.lock(wb.at(k)), seen[k], seen[k] | kLockBit);
                uint32_t held = 0;
#pragma unroll
                for (uint32_t k = 0; k < kOplistMaxWrites; ++k) {
                    if (got[k]) held |= 1u << k;
                    ok &= got[k] || !want[k];
                }
                wb.locked = held;
                if (!ok) {
#pragma unroll
                    for (uint32_t k = 0; k < kOplistMaxWrites; ++k)
                        if (got[k]) st_agent(lay.lock(wb.at(k)), seen[k]);
                    wb.locked = 0;
                }
            }
            hw_order();
            const uint32_t wv = wave_fetch_add(&a->hot->clock.v, ok && upd);
            hw_order();
            if (ok && upd && wv != rv) {
                for (uint32_t j0 = 0; j0 < L; j0 += kChunk) {
                    uint32_t w[kChunk];
                    uint64_t l[kChunk];
#pragma unroll
                    for (uint32_t k = 0; k < kChunk; ++k) w[k] = ix[(j0 + k < L ? j0 + k : j0) * kWave];
#pragma unroll
                    for (uint32_t k = 0; k < kChunk; ++k) l[k] = ld_agent(lay.lock(w[k]));
#pragma unroll
                    for (uint32_t k = 0; k < kChunk; ++k)
                        if (j0 + k < L && (((l[k] & kLockBit) && !wb.mine(lay, w[k])) || Slot::version(l[k]) > rv))
                            ok = false;
                }
            }
            if (ok && upd && wv >= kClockLimit) {
                latch_error(cnt, HETM_ECAPACITY, ls.txn);
                ok = false;
            }
            // the round's first write of a word (its slot older than the
            // round) goes to the undo log with the value it replaces
            uint32_t umask = 0, uw[kOplistMaxWrites], uo[kOplistMaxWrites];
#pragma unroll
            for (uint32_t k = 0; k < kOplistMaxWrites; ++k) {
                uw[k] = wb.at(k < nwr ? k : 0);
                uo[k] = (uint32_t)seen[k];
                if (ok && upd && ((wb.locked >> k) & 1u) && Slot::version(seen[k]) <= clock_base) umask |= 1u << k;
            }
            if (ok && upd)
                wb.commit(lay, wv + 1);
            else if (wb.locked)
                wb.abort(lay);
            if (a->undo_cap) undo_record(a, umask, uw, uo);
            ticket = upd ? 2u * (wv - clock_base) + 1u : 2u * (rv - clock_base);
        } else {
            // Split layout: first pass over the read stripes, then the values
            uint64_t sum1 = 0;
            for (uint32_t j0 = 0; j0 < L; j0 += kChunk) {
                uint64_t l[kChunk];
#pragma unroll
                for (uint32_t k = 0; k < kChunk; ++k) l[k] = ld_agent(lay.lock(ix[(j0 + k < L ? j0 + k : j0) * kWave]));
#pragma unroll
                for (uint32_t k = 0; k < kChunk; ++k)
                    if (j0 + k < L) {
                        ok &= !(l[k] & kLockBit);
                        sum1 += l[k];
                    }
            }
            hw_order();
            if (ok) {
                for (uint32_t j0 = 0; j0 < L; j0 += kChunk) {
                    uint32_t w[kChunk], v[kChunk];
#pragma unroll
                    for (uint32_t k = 0; k < kChunk; ++k) w[k] = ix[(j0 + k < L ? j0 + k : j0) * kWave];
#pragma unroll
                    for (uint32_t k = 0; k < kChunk; ++k) v[k] = lay.load(w[k]);
#pragma unroll
                    for (uint32_t k = 0; k < kChunk; ++k) {
                        const uint32_t j = j0 + k;
                        if (j < L) {
                            res[o + j] = v[k];
                            if (j < nwr) wb.put(w[k], v[k] + tv);
                        }
                    }
                }
                if (nwr) ok = wb.lock_all(lay);
            }
            hw_order();
            ticket = wave_fetch_add(&a->hot->ticket.v, ok);
            hw_order();
            if (ok) {
                // revalidation: reload every read stripe's lock word
                uint64_t sum2 = 0;
                for (uint32_t j0 = 0; j0 < L; j0 += kChunk) {
                    uint32_t w[kChunk];
                    uint64_t l[kChunk];
#pragma unroll
                    for (uint32_t k = 0; k < kChunk; ++k) w[k] = ix[(j0 + k < L ? j0 + k : j0) * kWave];
#pragma unroll
                    for (uint32_t k = 0; k < kChunk; ++k) l[k] = ld_agent(lay.lock(w[k]));
#pragma unroll
                    for (uint32_t k = 0; k < kChunk; ++k)
                        if (j0 + k < L) {
                            if (l[k] & kLockBit) {
                                if (!wb.mine(lay, lay.stripe(w[k]))) ok = false;
                                l[k] &= ~kLockBit;
                            }
                            sum2 += l[k];
                        }
                }
                ok &= sum2 == sum1;
            }
            if (ok)
                wb.commit(lay);
            else if (wb.locked)
                wb.abort(lay);
        }
        if (ok) {
            for (uint32_t j = nwr; j < L; ++j) rs_mark(rs, div32(ix[j * kWave], G));
            wb.mark_writes(rs, ws, G);
        }
        settle(ls, act, malformed, ok, ticket, a->tickets, cnt, a->retry_cap);
    }
    flush_counts(ls, cnt);
}

// CACHE layout constants (see the CACHE kernel below) and the set a key maps to.
constexpr uint32_t kSetWords = 128, kStampBase = 16, kSetStamp = 24, kValBase = 32;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {   // splitmix64 finalizer
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint32_t cache_set(uint64_t key, uint64_t nsets) {
    return (uint32_t)((mix64(key) & (nsets - 1) & ~1ull) | (key & 1ull));
}

// ---------------------------------------------------------------- TRANSFER
// Reads balances of src and dst (int64 words); if src != dst and the source
// balance covers amt, moves amt.  Results: [bs | bd | applied] (3 x n int64).
//
// Skewed account popularity (the bank workload draws accounts Zipf(0.9))
// makes a few accounts part of a large share of the batch.  Run as one
// transaction per lane, every commit on such an account hands its lock to
// the next lane through device memory, and the lanes in between abort and
// retry.  So before the transaction kernel a sample of the batch names the
// hot accounts, each transfer touching one becomes part of that account's
// chain (the hotter account's, if both are hot), and the kernel runs each
// chain on one wave: the wave holds the hot account's balance in a register
// and applies up to 64 transfers per step under the locks of both sides,
// in lane order, with consecutive commit tickets.  The other transfers form
// the cold list and run one per lane as before.  Which transfers run
// together has no bearing on serializability: every transfer still commits
// under the locks of both of its accounts with its ticket taken inside.

constexpr uint32_t kTxSample = 1u << 16;          // transfers sampled per batch
constexpr uint32_t kTxHotMin = 4;                 // sample appearances that make an account hot
constexpr uint32_t kTxMapSlots = 2 * kTxMaxHot;   // LDS map of the hot accounts
constexpr uint32_t kTxTile = 4096;                // transfers per classify / scatter block and tile
constexpr uint32_t kTxThreads = 256;
constexpr uint32_t kNoChain = 0xFFFFFFFFu;
constexpr uint32_t kNoAccount = 0xFFFFFFFFu;      // free map slot (accounts are below 2^32 - 1)

__device__ __forceinline__ uint32_t tx_hash(uint32_t w) { return w * 0x9E3779B1u; }

// count one appearance of account w in the sample table (key = w + 1 in the
// high half, count in the low half); a crowded neighbourhood leaves w cold
__device__ __forceinline__ void tx_count(uint64_t *tab, uint32_t w) {
    const uint64_t key = (uint64_t)(w + 1) << 32;
    uint32_t s = tx_hash(w) >> (32 - kTxTabBits);
    for (uint32_t i = 0; i < 64; ++i, s = (s + 1) & (kTxTabSlots - 1)) {
        uint64_t cur = ld_agent(&tab[s]);
        if (cur == 0) {
            uint64_t exp = 0;
            if (__hip_atomic_compare_exchange_strong(&tab[s], &exp, key | 1ull, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT))
                return;
            cur = exp;
        }
        if ((cur & ~0xFFFFFFFFull) == key) {
            __hip_atomic_fetch_add(&tab[s], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
    }
}

// The objects a transaction touches, as the hot-object pre-pass sees them:
// a transfer's two accounts, a cache operation's set.  Returns 0 for a
// malformed transaction (the transaction kernel reports it).
template <uint32_t P>
__device__ __forceinline__ uint32_t tx_objects(const DevArgs *a, uint32_t t, uint32_t &o0, uint32_t &o1) {
    if constexpr (P == HETM_PROG_TRANSFER) {
        o0 = a->src[t];
        o1 = a->dst[t];
        if (o0 >= a->n_words || o1 >= a->n_words) return 0;
        return o0 == o1 ? 1 : 2;
    } else {
        const uint64_t key = a->key[t];
        if (key == 0 || a->op[t] > 1) return 0;
        o0 = o1 = cache_set(key, a->n_words / kSetWords);
        return 1;
    }
}

// every (n / S)-th transaction of the batch, S = min(n, kTxSample)
template <uint32_t P>
__global__ __launch_bounds__(kTxThreads) void k_tx_sample(const DevArgs *__restrict__ a) {
    const uint32_t n = a->n_txns;
    const uint32_t S = n < kTxSample ? n : kTxSample;
    const uint32_t step = S ? n / S : 1;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < S; i += gridDim.x * blockDim.x) {
        uint32_t o0, o1;
        const uint32_t k = tx_objects<P>(a, i * step, o0, o1);
        if (k >= 1) tx_count(a->tx_tab, o0);
        if (k == 2) tx_count(a->tx_tab, o1);
    }
}

// one thread per table slot: accounts seen kTxHotMin times or more become
// chains; every slot is cleared for the next batch
__global__ __launch_bounds__(kTxThreads) void k_tx_pick(const DevArgs *__restrict__ a) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t v = a->tx_tab[i];
    bool hot = false;
    uint64_t e = 0;
    if (v) {
        a->tx_tab[i] = 0;
        hot = (uint32_t)v >= kTxHotMin;
        e = ((uint64_t)(uint32_t)v << 32) | ((v >> 32) - 1);
    }
    const uint32_t pos = wave_fetch_add(&a->hot->n_ro.v, hot);
    if (hot && pos < kTxMaxHot) a->tx_hot[pos] = e;
}

struct HotMap {
    uint32_t acc[kTxMapSlots];
    uint16_t idx[kTxMapSlots];
};

__device__ __forceinline__ uint32_t tx_n_hot(const DevArgs *a) {
    const uint32_t h = ld_agent(&a->hot->n_ro.v);
    return h < kTxMaxHot ? h : kTxMaxHot;
}

__device__ void load_hot_map(const DevArgs *a, HotMap &m, uint32_t n_hot) {
    for (uint32_t i = threadIdx.x; i < kTxMapSlots; i += blockDim.x) m.acc[i] = kNoAccount;
    __syncthreads();
    for (uint32_t h = threadIdx.x; h < n_hot; h += blockDim.x) {
        const uint32_t w = (uint32_t)a->tx_hot[h];
        uint32_t s = tx_hash(w) & (kTxMapSlots - 1);
        while (atomicCAS(&m.acc[s], kNoAccount, w) != kNoAccount) s = (s + 1) & (kTxMapSlots - 1);
        m.idx[s] = (uint16_t)h;
    }
    __syncthreads();
}

__device__ __forceinline__ uint32_t hot_index(const HotMap &m, uint32_t w) {
    uint32_t s = tx_hash(w) & (kTxMapSlots - 1);
    for (;;) {
        const uint32_t k = m.acc[s];
        if (k == w) return m.idx[s];
        if (k == kNoAccount) return kNoChain;
        s = (s + 1) & (kTxMapSlots - 1);
    }
}

// the chain a transaction belongs to: its hot object's, the hotter one's (by
// sample count, then object) if both are hot, none if neither is
template <uint32_t P>
__device__ __forceinline__ uint32_t chain_of(const DevArgs *a, const HotMap &m, uint32_t t) {
    uint32_t o0, o1;
    const uint32_t k = tx_objects<P>(a, t, o0, o1);
    if (k == 0) return kNoChain;
    const uint32_t hs = hot_index(m, o0), hd = k == 1 ? hs : hot_index(m, o1);
    if (hs == kNoChain) return hd;
    if (hd == kNoChain || hd == hs) return hs;
    return a->tx_hot[hs] > a->tx_hot[hd] ? hs : hd;
}

// classify: cold transactions go to the back of `order`; chain members are
// counted per chain
template <uint32_t P>
__global__ __launch_bounds__(kTxThreads) void k_tx_classify(const DevArgs *__restrict__ a) {
    __shared__ HotMap m;
    __shared__ uint32_t hist[kTxMaxHot];
    const uint32_t n = a->n_txns, n_hot = tx_n_hot(a);
    for (uint32_t h = threadIdx.x; h < kTxMaxHot; h += blockDim.x) hist[h] = 0;
    load_hot_map(a, m, n_hot);
    uint32_t *order = a->order;
    for (uint64_t t0 = (uint64_t)blockIdx.x * kTxTile; t0 < n; t0 += (uint64_t)gridDim.x * kTxTile) {
        for (uint32_t k = threadIdx.x; k < kTxTile; k += kTxThreads) {   // uniform trip count
            const uint64_t t = t0 + k;
            uint32_t c = kNoChain;
            if (t < n) c = chain_of<P>(a, m, (uint32_t)t);
            const bool cold = t < n && c == kNoChain;
            const uint32_t pos = wave_fetch_add(&a->hot->n_upd.v, cold);
            if (cold) order[n - 1 - pos] = (uint32_t)t;
            else if (t < n) atomicAdd(&hist[c], 1u);
        }
    }
    __syncthreads();
    uint32_t *count = a->tx_chain;
    for (uint32_t h = threadIdx.x; h < n_hot; h += blockDim.x)
        if (hist[h]) __hip_atomic_fetch_add(&count[h], hist[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// one block: each chain's first position in `order` and its cursor, and the
// chains sorted by length, longest first; the counts are cleared
__global__ __launch_bounds__(1024) void k_tx_plan(const DevArgs *__restrict__ a) {
    __shared__ unsigned long long key[kTxMaxHot];
    __shared__ uint32_t sh[1024 / kWave];
    const uint32_t n_hot = tx_n_hot(a);
    uint32_t *count = a->tx_chain, *start = count + kTxMaxHot, *cursor = start + kTxMaxHot + 1,
             *corder = cursor + kTxMaxHot;
    constexpr uint32_t kPer = kTxMaxHot / 1024;
    uint32_t c[kPer], sum = 0;
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) {
        const uint32_t h = threadIdx.x * kPer + j;
        c[j] = h < n_hot ? ld_agent(&count[h]) : 0u;
        sum += c[j];
        key[h] = h < n_hot ? ((unsigned long long)c[j] << 32) | h : 0ull;
    }
    // exclusive prefix of the per-thread sums
    const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
    uint32_t inc = sum;
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t t = __shfl_up(inc, o);
        if ((int)lane >= o) inc += t;
    }
    if (lane == kWave - 1) sh[wv] = inc;
    __syncthreads();
    uint32_t run = inc - sum;
    for (uint32_t i = 0; i < wv; ++i) run += sh[i];
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) {
        const uint32_t h = threadIdx.x * kPer + j;
        if (h < n_hot) {
            start[h] = run;
            cursor[h] = run;
            count[h] = 0;
        }
        run += c[j];
    }
    if (threadIdx.x == 1023) start[n_hot] = run;
    __syncthreads();
    // bitonic sort, descending
    for (uint32_t k = 2; k <= kTxMaxHot; k <<= 1)
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < kTxMaxHot; i += 1024) {
                const uint32_t l = i ^ j;
                if (l > i) {
                    const bool desc = (i & k) == 0;
                    const unsigned long long x = key[i], y = key[l];
                    if (desc ? x < y : x > y) {
                        key[i] = y;
                        key[l] = x;
                    }
                }
            }
            __syncthreads();
        }
    for (uint32_t i = threadIdx.x; i < n_hot; i += 1024) corder[i] = (uint32_t)key[i];
}

// scatter: chain members into their chain's range of `order`, one atomic per
// chain and tile reserving the tile's share
template <uint32_t P>
__global__ __launch_bounds__(kTxThreads) void k_tx_scatter(const DevArgs *__restrict__ a) {
    __shared__ HotMap m;
    __shared__ uint32_t pos[kTxMaxHot];
    const uint32_t n = a->n_txns, n_hot = tx_n_hot(a);
    if (n_hot == 0) return;
    load_hot_map(a, m, n_hot);
    uint32_t *order = a->order, *cursor = a->tx_chain + 2 * kTxMaxHot + 1;
    for (uint64_t t0 = (uint64_t)blockIdx.x * kTxTile; t0 < n; t0 += (uint64_t)gridDim.x * kTxTile) {
        for (uint32_t h = threadIdx.x; h < n_hot; h += kTxThreads) pos[h] = 0;
        __syncthreads();
        constexpr uint32_t kPer = kTxTile / kTxThreads;
        uint32_t c[kPer];
#pragma unroll
        for (uint32_t j = 0; j < kPer; ++j) {
            const uint64_t t = t0 + j * kTxThreads + threadIdx.x;
            c[j] = t < n ? chain_of<P>(a, m, (uint32_t)t) : kNoChain;
            if (c[j] != kNoChain) atomicAdd(&pos[c[j]], 1u);
        }
        __syncthreads();
        for (uint32_t h = threadIdx.x; h < n_hot; h += kTxThreads)
            if (pos[h]) pos[h] = __hip_atomic_fetch_add(&cursor[h], pos[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
#pragma unroll
        for (uint32_t j = 0; j < kPer; ++j)
            if (c[j] != kNoChain) order[atomicAdd(&pos[c[j]], 1u)] = (uint32_t)(t0 + j * kTxThreads + threadIdx.x);
        __syncthreads();
    }
}

__device__ __forceinline__ uint32_t readlane(uint32_t v, uint32_t k) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)k);
}
__device__ __forceinline__ int64_t readlane64(int64_t v, uint32_t k) {
    const uint64_t u = (uint64_t)v;
    return (int64_t)(((uint64_t)readlane((uint32_t)(u >> 32), k) << 32) | readlane((uint32_t)u, k));
}
// lane k's copy of v becomes x (x and k wave-uniform)
__device__ __forceinline__ uint32_t writelane(uint32_t v, uint32_t x, uint32_t k) { return lane_id() == k ? x : v; }
__device__ __forceinline__ int64_t writelane64(int64_t v, int64_t x, uint32_t k) { return lane_id() == k ? x : v; }

// One wave applies the chain of hot account X: list[0 .. m) are transfer ids
// that touch X.  Each step, lanes without a transfer take the chain's next
// ones; lane 0 locks X's stripe, the first lane of every other stripe the
// step touches locks it (a lane whose stripe is held elsewhere sits the step
// out and keeps its transfer); the step's transfers are applied in lane
// order with X's balance in a scalar register and the other accounts'
// balances in the registers of the first lane naming them, take consecutive
// tickets, store, mark the bitmaps and release (version + 1 for a stripe
// that was written).  Every lock is a try-lock and released within the
// step, so no wave waits while holding one.
__device__ void run_chain(const DevArgs *a, const Split<uint64_t> &lay, uint32_t X, const uint32_t *list, uint32_t m,
                          LaneState &ls, uint32_t *sflag, uint32_t epoch) {
    DevCounters *cnt = a->cnt;
    const uint32_t n = a->n_txns;
    const uint64_t N = a->n_words;
    const Div32 G = a->gdiv;
    gmem<uint8_t> *rs = glob(a->rs);
    gmem<uint32_t> *ws = glob(a->ws);
    int64_t *res = (int64_t *)a->results;
    const uint32_t lane = lane_id();
    const uint32_t xst = lay.stripe(X);
    uint32_t next = 0, t = kNoTxn, tries = 0;
    for (;;) {
        const bool need = t == kNoTxn;
        const uint64_t nm = __ballot(need);
        if (need && next + lanes_below(nm) < m) t = list[next + lanes_below(nm)];
        next = min(m, next + (uint32_t)__popcll(nm));
        const bool have = t != kNoTxn;
        if (!__ballot(have)) break;
        if (doomed(cnt, epoch)) break;
        uint32_t s = 0, d = 0, am = 0;
        if (have) {
            s = a->src[t];
            d = a->dst[t];
            am = a->amt[t];
        }
        if (have && (s >= N || d >= N)) {      // malformed: reported, never executed
            latch_error(cnt, HETM_EINVAL, t);
            t = kNoTxn;
            continue;
        }
        const bool live = t != kNoTxn;
        const uint32_t y = s == X ? d : s;     // the other account (X itself for a transfer X -> X)
        const uint32_t yst = lay.stripe(y);
        // the first live lane naming the same account (its balance) and the
        // same stripe (its lock)
        uint32_t vslot = lane, lslot = lane;
        const uint64_t lm = __ballot(live);
        for (uint32_t k = 0; k < kWave; ++k) {
            if (!((lm >> k) & 1u)) continue;
            const uint32_t yk = readlane(y, k);
            if (k < lane && vslot == lane && yk == y) vslot = k;
            if (k < lane && lslot == lane && lay.stripe(yk) == yst) lslot = k;
        }
        // lock X's stripe, then every other stripe once
        uint32_t xl = 0;
        if (lane == 0) {
            gmem<uint64_t> *p = lay.lock(X);
            const uint64_t cur = ld_agent(p);
            xl = !(cur & kLockBit) && cas_agent(p, cur, cur | kLockBit);
        }
        if (!readlane(xl, 0)) {                // another chain holds it (X as its other side): retry
            if (live) {
                ls.retries++;
                if (++tries >= a->retry_cap) {
                    latch_error(cnt, HETM_ERETRY, t);
                    t = kNoTxn;
                }
            }
            __builtin_amdgcn_s_sleep(4);
            continue;
        }
        uint32_t mine = 0;                     // this lane holds the lock of stripe yst
        if (live && lslot == lane && yst != xst) {
            gmem<uint64_t> *p = lay.lock(y);
            const uint64_t cur = ld_agent(p);
            mine = !(cur & kLockBit) && cas_agent(p, cur, cur | kLockBit);
        }
        const bool part = live && (yst == xst || __shfl((int)mine, (int)lslot) != 0);
        hw_order();                            // locks held before any balance is read
        int64_t xv = 0, yv = 0;
        if (lane == 0) xv = (int64_t)lay.load(X);
        if (part && vslot == lane && y != X) yv = (int64_t)lay.load(y);
        hw_order();
        int64_t bx = readlane64(xv, 0);
        int64_t r_bs = 0, r_bd = 0;
        uint32_t r_ap = 0, ywr = 0, xwr = 0;
        const uint64_t pm = __ballot(part);
        for (uint32_t k = 0; k < kWave; ++k) {     // the step's transfers in lane order
            if (!((pm >> k) & 1u)) continue;
            const uint32_t sk = readlane(s, k), dk = readlane(d, k), ak = readlane(am, k), vk = readlane(vslot, k);
            int64_t bs, bd;
            uint32_t ap = 0;
            if (sk == dk) {                        // X -> X: reads only
                bs = bd = bx;
            } else {
                int64_t by = readlane64(yv, vk);
                if (sk == X) {
                    bs = bx;
                    bd = by;
                    ap = bx >= (int64_t)ak;
                    if (ap) {
                        bx -= ak;
                        by += ak;
                    }
                } else {
                    bs = by;
                    bd = bx;
                    ap = by >= (int64_t)ak;
                    if (ap) {
                        by -= ak;
                        bx += ak;
                    }
                }
                if (ap) {
                    yv = writelane64(yv, by, vk);
                    ywr = writelane(ywr, 1u, vk);
                    xwr = 1;
                }
            }
            r_bs = writelane64(r_bs, bs, k);
            r_bd = writelane64(r_bd, bd, k);
            r_ap = writelane(r_ap, ap, k);
        }
        // tickets: the step's transfers in lane order
        uint32_t base = 0;
        if (lane == 0 && pm) base = __hip_atomic_fetch_add(&a->hot->ticket.v, (uint32_t)__popcll(pm), __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
        base = readlane(base, 0);
        if (part && vslot == lane && ywr) st_agent(&lay.vals[y], (uint64_t)yv);
        if (lane == 0 && xwr) st_agent(&lay.vals[X], (uint64_t)bx);
        if (part) {
            res[t] = r_bs;
            res[n + t] = r_bd;
            res[2 * (uint64_t)n + t] = r_ap;
            a->tickets[t] = base + lanes_below(pm);
        }
        // which lock-holding lanes' stripes were written
        sflag[lane] = 0;
        if (part && r_ap && yst != xst) sflag[lslot] = 1;
        hw_order();                            // balances stored before any stripe is released
        if (lane == 0)
            __hip_atomic_fetch_add(lay.lock(X), xwr ? 1ull - kLockBit : 0ull - kLockBit, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        if (mine)
            __hip_atomic_fetch_add(lay.lock(y), sflag[lane] ? 1ull - kLockBit : 0ull - kLockBit, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        if (part) {
            const uint32_t gs = div32(s, G), gd = div32(d, G);
            rs_mark(rs, gs);
            rs_mark(rs, gd);
            if (r_ap) {
                bitmap_set(ws, gs);
                bitmap_set(ws, gd);
            }
            ls.commits++;
            t = kNoTxn;
            tries = 0;
        } else if (live) {
            ls.retries++;
            if (++tries >= a->retry_cap) {
                latch_error(cnt, HETM_ERETRY, t);
                t = kNoTxn;
            }
        }
    }
}

// Refill lanes without work from the cold list (the back of `order`);
// returns false when the whole wave is out of work.  Reached by all 64 lanes.
__device__ __forceinline__ bool refill_cold(LaneState &ls, const DevArgs *a, uint32_t n, uint32_t n_cold) {
    const bool need = ls.txn == kNoTxn;
    if (__ballot(need)) {
        const uint32_t got = wave_fetch_add(&a->hot->queue_head.v, need);
        if (need) {
            ls.txn = got < n_cold ? a->order[n - 1 - got] : kDoneTxn;
            ls.attempts = 0;
        }
    }
    return __ballot(ls.txn < n) != 0;
}

__global__ __launch_bounds__(kExecWaves *kWave) void k_exec_transfer(const DevArgs *__restrict__ a) {
    __shared__ uint32_t s_addr[kExecWaves][2][kWave];
    __shared__ uint64_t s_val[kExecWaves][2][kWave];
    __shared__ uint32_t s_flag[kExecWaves][kWave];
    const uint32_t wv = threadIdx.x / kWave;
    const Split<uint64_t> lay = make_layout<Split<uint64_t>>(a);
    gmem<uint8_t> *rs = glob(a->rs);
    gmem<uint32_t> *ws = glob(a->ws);
    DevCounters *cnt = a->cnt;
    const uint32_t n = a->n_txns;
    const Div32 G = a->gdiv;
    const uint64_t N = a->n_words;
    int64_t *res = (int64_t *)a->results;
    WriteBuf<uint64_t, 2> wb{s_addr[wv], s_val[wv], lane_id(), 0, 0};
    const uint32_t epoch = a->epoch;
    LaneState ls;

    // the hot accounts' chains, longest first, one wave each
    const uint32_t n_hot = ld_agent(&a->hot->n_ro.v) < kTxMaxHot ? ld_agent(&a->hot->n_ro.v) : kTxMaxHot;
    const uint32_t *start = a->tx_chain + kTxMaxHot, *corder = a->tx_chain + 3 * kTxMaxHot + 1;
    for (;;) {
        uint32_t c = 0;
        if (lane_id() == 0) c = __hip_atomic_fetch_add(&a->hot->queue_upd.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        c = readlane(c, 0);
        if (c >= n_hot) break;
        const uint32_t h = corder[c];
        const uint32_t lo = start[h], hi = start[h + 1];
        run_chain(a, lay, (uint32_t)a->tx_hot[h], a->order + lo, hi - lo, ls, s_flag[wv], epoch);
        if (doomed(cnt, epoch)) break;
    }

    // the cold list, one transfer per lane
    const uint32_t n_cold = ld_agent(&a->hot->n_upd.v);
    while (refill_cold(ls, a, n, n_cold)) {
        const bool act = lane_turn(ls, n);
        if (doomed(cnt, epoch)) break;
        if (!__ballot(act)) {          // every lane is backing off
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        bool ok = act;
        uint32_t s = 0, d = 0, am = 0;
        if (act) {
            s = a->src[ls.txn];
            d = a->dst[ls.txn];
            am = a->amt[ls.txn];
            if (s >= N || d >= N) {
                latch_error(cnt, HETM_EINVAL, ls.txn);
                ok = false;
            }
        }
        uint64_t sum1 = 0;
        if (ok) {
            uint64_t l1 = ld_agent(lay.lock(s));
            uint64_t l2 = ld_agent(lay.lock(d));
            ok = !((l1 | l2) & kLockBit);
            sum1 = l1 + l2;
        }
        hw_order();
        wb.n = 0;
        if (ok) {
            int64_t bs = (int64_t)lay.load(s);
            int64_t bd = (int64_t)lay.load(d);
            bool applied = s != d && bs >= (int64_t)am;
            res[ls.txn] = bs;
            res[n + ls.txn] = bd;
            res[2 * (uint64_t)n + ls.txn] = applied;
            if (applied) {
                wb.put(s, (uint64_t)(bs - (int64_t)am));
                wb.put(d, (uint64_t)(bd + (int64_t)am));
                ok = wb.lock_all(lay);
            }
        }
        hw_order();
        uint32_t ticket = wave_fetch_add(&a->hot->ticket.v, ok);
        hw_order();
        if (ok) {
            uint64_t sum2 = reread(lay, s, wb, ok);
            sum2 += reread(lay, d, wb, ok);
            ok &= sum2 == sum1;
        }
        if (ok)
            wb.commit(lay);
        else if (wb.locked)
            wb.abort(lay);
        if (ok) {
            rs_mark(rs, div32(s, G));
            rs_mark(rs, div32(d, G));
            wb.mark_writes(rs, ws, G);
        }
        settle(ls, act, act && (s >= N || d >= N), ok, ticket, a->tickets, cnt, a->retry_cap);
    }
    flush_counts(ls, cnt);
}

// ------------------------------------------------------------------- CACHE
// 8-way set-associative cache in 32-bit words, one 128-word record per set:
// keys at 0..15 (u64 per way, low word first), LRU stamps at 16..23, set PUT
// stamp at 24, values at 32 + 8*way.  GET reads the set stamp and the keys;
// on a hit it reads the value and writes the way's stamp := tid.  PUT also
// reads the stamps, picks the way holding the key or else the smallest
// stamp (lowest way on ties) and writes key, value, stamp and set stamp.

// j-th word of the header read list: 8 keys (16 words), set stamp, 8 stamps
__device__ __forceinline__ uint32_t header_word(uint32_t j) {
    return j < 16 ? j : (j == 16 ? kSetStamp : kStampBase + (j - 17));
}

// One wave applies the chain of hot set X: list[0 .. m) are the cache
// operations on it.  Only this chain touches the set (an operation reads and
// writes its own set only, and every operation on X is in X's chain), so the
// wave takes no lock: it loads the set once into its registers -- lane L
// holds words 2L and 2L + 1 -- applies the operations in steps of up to 64,
// each in lane order with the same steps as the one-lane program, and stores
// the words it wrote when the chain is done.  Tickets are drawn per step:
// slot layout, one version-clock value per operation (its written words get
// that value + 1 as their version, as a commit would); lock table, the
// ticket counter.
template <typename Lay>
__device__ void run_cache_chain(const DevArgs *a, const Lay &lay, uint32_t X, const uint32_t *list, uint32_t m,
                                LaneState &ls, uint32_t epoch, uint32_t clock_base) {
    DevCounters *cnt = a->cnt;
    const Div32 G = a->gdiv;
    gmem<uint8_t> *rs = glob(a->rs);
    gmem<uint32_t> *ws = glob(a->ws);
    uint32_t *res = (uint32_t *)a->results;
    const uint32_t lane = lane_id();
    const uint32_t base = X * kSetWords;
    // the set: value, version and written flag of this lane's two words,
    // and their slots as found (the undo log records the round's first writes)
    uint64_t f0 = 0, f1 = 0;
    uint32_t w0, w1;
    if constexpr (Lay::kFused) {
        f0 = ld_agent(lay.lock(base + 2 * lane));
        f1 = ld_agent(lay.lock(base + 2 * lane + 1));
        w0 = (uint32_t)f0;
        w1 = (uint32_t)f1;
    } else {
        w0 = lay.load(base + 2 * lane);
        w1 = lay.load(base + 2 * lane + 1);
    }
    uint32_t v0 = 0, v1 = 0, d0 = 0, d1 = 0;
    uint32_t next = 0, t = kNoTxn;
    for (;;) {
        const bool need = t == kNoTxn;
        const uint64_t nm = __ballot(need);
        if (need && next + lanes_below(nm) < m) t = list[next + lanes_below(nm)];
        next = min(m, next + (uint32_t)__popcll(nm));
        const bool have = t != kNoTxn;
        if (!__ballot(have)) break;
        if (doomed(cnt, epoch)) break;
        uint64_t key = 0;
        uint32_t put = 0, tv = 0;
        if (have) {
            key = a->key[t];
            put = a->op[t];
            tv = a->tid[t];
        }
        const uint64_t pm = __ballot(have);
        // tickets, one per operation in lane order
        uint32_t first = 0;
        if (lane == 0)
            first = __hip_atomic_fetch_add(Lay::kFused ? &a->hot->clock.v : &a->hot->ticket.v, (uint32_t)__popcll(pm),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        first = readlane(first, 0);
        const uint32_t draw = first + lanes_below(pm);
        uint32_t r[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        uint32_t way = 0;       // GET: the hit way (8 = miss); PUT: the victim
        for (uint32_t k = 0; k < kWave; ++k) {
            if (!((pm >> k) & 1u)) continue;
            const uint64_t kk = ((uint64_t)readlane((uint32_t)(key >> 32), k) << 32) | readlane((uint32_t)key, k);
            const uint32_t pk = readlane(put, k), tk = readlane(tv, k);
            const uint32_t ver = readlane(draw, k) + 1;
            // lanes 0..7 hold the keys of ways 0..7
            const uint64_t hm = __ballot(lane < 8 && (((uint64_t)w1 << 32) | w0) == kk);
            const int hit = hm ? (int)__ffsll((unsigned long long)hm) - 1 : -1;
            uint32_t st = 0, rv[8] = {0, 0, 0, 0, 0, 0, 0, 0}, wy = 8;
            if (!pk) {
                if (hit >= 0) {
                    st = 0x100u | (uint32_t)hit;
#pragma unroll
                    for (uint32_t i = 0; i < 8; ++i) {      // word 32 + 8 hit + i: lane 16 + 4 hit + i/2
                        const uint32_t L = 16 + 4 * hit + i / 2;
                        rv[i] = (i & 1) ? readlane(w1, L) : readlane(w0, L);
                    }
                    // stamp of the way: word 16 + hit, lane 8 + hit/2
                    const uint32_t L = 8 + hit / 2;
                    if (hit & 1) {
                        w1 = writelane(w1, tk, L), v1 = writelane(v1, ver, L), d1 = writelane(d1, 1u, L);
                    } else {
                        w0 = writelane(w0, tk, L), v0 = writelane(v0, ver, L), d0 = writelane(d0, 1u, L);
                    }
                    wy = (uint32_t)hit;
                }
            } else {
                uint32_t victim = 0, vmin = readlane(w0, 8);
#pragma unroll
                for (uint32_t w = 1; w < 8; ++w) {
                    const uint32_t sw = (w & 1) ? readlane(w1, 8 + w / 2) : readlane(w0, 8 + w / 2);
                    if (sw < vmin) {
                        vmin = sw;
                        victim = w;
                    }
                }
                if (hit >= 0) victim = (uint32_t)hit;
                st = 0x200u | (hit >= 0 ? 0x100u : 0u) | victim;
                uint32_t chk = (uint32_t)mix64(kk);
#pragma unroll
                for (uint32_t i = 0; i < 7; ++i) {
                    rv[i] = (uint32_t)mix64(kk ^ ((uint64_t)tk << 32) ^ i);
                    chk ^= rv[i];
                }
                rv[7] = chk;
                // key: words 2v, 2v+1 (lane v); values: words 32 + 8v + i (lane 16 + 4v + i/2);
                // stamp: word 16 + v; set stamp: word 24 (lane 12, low word)
                w0 = writelane(w0, (uint32_t)kk, victim), v0 = writelane(v0, ver, victim), d0 = writelane(d0, 1u, victim);
                w1 = writelane(w1, (uint32_t)(kk >> 32), victim), v1 = writelane(v1, ver, victim),
                d1 = writelane(d1, 1u, victim);
#pragma unroll
                for (uint32_t i = 0; i < 8; i += 2) {
                    const uint32_t L = 16 + 4 * victim + i / 2;
                    w0 = writelane(w0, rv[i], L), v0 = writelane(v0, ver, L), d0 = writelane(d0, 1u, L);
                    w1 = writelane(w1, rv[i + 1], L), v1 = writelane(v1, ver, L), d1 = writelane(d1, 1u, L);
                }
                const uint32_t L = 8 + victim / 2;
                if (victim & 1) {
                    w1 = writelane(w1, tk, L), v1 = writelane(v1, ver, L), d1 = writelane(d1, 1u, L);
                } else {
                    w0 = writelane(w0, tk, L), v0 = writelane(v0, ver, L), d0 = writelane(d0, 1u, L);
                }
                w0 = writelane(w0, tk, 12), v0 = writelane(v0, ver, 12), d0 = writelane(d0, 1u, 12);
                wy = victim;
            }
            r[0] = writelane(r[0], st, k);
#pragma unroll
            for (uint32_t i = 0; i < 8; ++i) r[1 + i] = writelane(r[1 + i], rv[i], k);
            way = writelane(way, wy, k);
        }
        if (have) {
            uint32_t *o = res + 9ull * t;
#pragma unroll
            for (uint32_t i = 0; i < 9; ++i) o[i] = r[i];
            const bool upd = put || way < 8;
            a->tickets[t] = Lay::kFused ? 2u * (draw - clock_base) + 1u : draw;
            if (Lay::kFused && draw + 1 >= kClockLimit) latch_error(cnt, HETM_ECAPACITY, t);
            // the bitmaps: what the one-lane program marks for this operation
            const uint32_t nh = put ? 25u : 17u;
            for (uint32_t j = 0; j < nh; ++j) rs_mark(rs, div32(base + header_word(j), G));
            if (!put && way < 8)
                for (uint32_t i = 0; i < 8; ++i) rs_mark(rs, div32(base + kValBase + 8 * way + i, G));
            if (upd) {
                if (put) {
                    const uint32_t vb = base + kValBase + 8 * way;
                    uint32_t wl[12] = {base + 2 * way, base + 2 * way + 1, vb, vb + 1, vb + 2, vb + 3, vb + 4, vb + 5,
                                       vb + 6, vb + 7, base + kStampBase + way, base + kSetStamp};
                    for (uint32_t j = 0; j < 12; ++j) {
                        rs_mark(rs, div32(wl[j], G));
                        bitmap_set(ws, div32(wl[j], G));
                    }
                } else {
                    const uint32_t g = div32(base + kStampBase + way, G);
                    rs_mark(rs, g);
                    bitmap_set(ws, g);
                }
            }
            ls.commits++;
            t = kNoTxn;
        }
    }
    // the words the chain wrote
    if constexpr (Lay::kFused) {
        if (d0) st_agent(lay.lock(base + 2 * lane), Slot::make(v0, w0));
        if (d1) st_agent(lay.lock(base + 2 * lane + 1), Slot::make(v1, w1));
        const uint32_t umask = (d0 && Slot::version(f0) <= clock_base ? 1u : 0u) |
                               (d1 && Slot::version(f1) <= clock_base ? 2u : 0u);
        const uint32_t uw[2] = {base + 2 * lane, base + 2 * lane + 1}, uo[2] = {(uint32_t)f0, (uint32_t)f1};
        if (a->undo_cap) undo_record(a, umask, uw, uo);
    } else {
        if (d0) st_agent(&lay.vals[base + 2 * lane], w0);
        if (d1) st_agent(&lay.vals[base + 2 * lane + 1], w1);
    }
}

template <typename Lay>
__global__ __launch_bounds__(kExecWaves *kWave) void k_exec_cache(const DevArgs *__restrict__ a) {
    __shared__ uint32_t s_addr[kExecWaves][kCacheMaxWrites][kWave];
    __shared__ uint32_t s_val[kExecWaves][kCacheMaxWrites][kWave];
    const uint32_t wv = threadIdx.x / kWave;
    const Lay lay = make_layout<Lay>(a);
    gmem<uint8_t> *rs = glob(a->rs);
    gmem<uint32_t> *ws = glob(a->ws);
    DevCounters *cnt = a->cnt;
    const uint32_t n = a->n_txns;
    const Div32 G = a->gdiv;
    const uint64_t nsets = a->n_words / kSetWords;
    uint32_t *res = (uint32_t *)a->results;
    WriteBuf<uint32_t, kCacheMaxWrites> wb{s_addr[wv], s_val[wv], lane_id(), 0, 0};
    const uint32_t epoch = a->epoch;
    const uint32_t clock_base = ld_agent(&cnt->clock_base);
    wb.base_ver = clock_base;
    LaneState ls;

    // the hot sets' chains, longest first, one wave each
    const uint32_t n_hot = ld_agent(&a->hot->n_ro.v) < kTxMaxHot ? ld_agent(&a->hot->n_ro.v) : kTxMaxHot;
    const uint32_t *start = a->tx_chain + kTxMaxHot, *corder = a->tx_chain + 3 * kTxMaxHot + 1;
    for (;;) {
        uint32_t c = 0;
        if (lane_id() == 0) c = __hip_atomic_fetch_add(&a->hot->queue_upd.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        c = readlane(c, 0);
        if (c >= n_hot) break;
        const uint32_t h = corder[c];
        const uint32_t lo = start[h], hi = start[h + 1];
        run_cache_chain(a, lay, (uint32_t)a->tx_hot[h], a->order + lo, hi - lo, ls, epoch, clock_base);
        if (doomed(cnt, epoch)) break;
    }

    // the cold list, one operation per lane
    const uint32_t n_cold = ld_agent(&a->hot->n_upd.v);
    while (refill_cold(ls, a, n, n_cold)) {
        const bool act = lane_turn(ls, n);
        if (doomed(cnt, epoch)) break;
        if (!__ballot(act)) {          // every lane is backing off
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        const uint32_t rv_load = Lay::kFused ? ld_agent(&a->hot->clock.v) : 0u;   // as in the OPLIST kernel
        bool ok = act;
        uint64_t key = 0;
        uint32_t put = 0, tv = 0, base = 0, nh = 0;
        if (act) {
            key = a->key[ls.txn];
            put = a->op[ls.txn];
            tv = a->tid[ls.txn];
            if (key == 0 || put > 1) {
                latch_error(cnt, HETM_EINVAL, ls.txn);
                ok = false;
            }
            base = cache_set(key, nsets) * kSetWords;
            nh = put ? 25u : 17u;
        }
        uint32_t hdr[25], gv[8];
        int hit = -1;
        bool get_hit = false;
        uint64_t sum1 = 0;
        uint32_t rv = 0;
        if constexpr (Lay::kFused) {
            // slot layout, TL2-style (as in the OPLIST kernel): one snapshot,
            // each slot load gives value and version together
            rv = __builtin_amdgcn_readfirstlane(rv_load);
            hw_order();   // the snapshot load has completed before any slot load issues
#pragma unroll
            for (uint32_t j = 0; j < 25; ++j) {
                const bool in = ok && j < nh;
                const uint64_t l = in ? ld_agent(lay.lock(base + header_word(j))) : 0;
                if (in) ok &= !(l & kLockBit) && Slot::version(l) <= rv;
                hdr[j] = (uint32_t)l;
            }
#pragma unroll
            for (int w = 7; w >= 0; --w)
                if (ok && ((uint64_t)hdr[2 * w] | ((uint64_t)hdr[2 * w + 1] << 32)) == key) hit = w;
            get_hit = ok && !put && hit >= 0;
#pragma unroll
            for (uint32_t i = 0; i < 8; ++i) {
                const uint64_t l = get_hit ? ld_agent(lay.lock(base + kValBase + 8 * hit + i)) : 0;
                if (get_hit) ok &= !(l & kLockBit) && Slot::version(l) <= rv;
                gv[i] = (uint32_t)l;
            }
        } else {
            if (ok)
                for (uint32_t j = 0; j < nh; ++j) {
                    uint64_t l = ld_agent(lay.lock(base + header_word(j)));
                    ok &= !(l & kLockBit);
                    sum1 += l;
                }
            hw_order();
#pragma unroll
            for (uint32_t j = 0; j < 25; ++j) hdr[j] = (ok && j < nh) ? lay.load(base + header_word(j)) : 0u;
#pragma unroll
            for (int w = 7; w >= 0; --w)
                if (ok && ((uint64_t)hdr[2 * w] | ((uint64_t)hdr[2 * w + 1] << 32)) == key) hit = w;
            // GET hit: second read phase over the way's value words
            get_hit = ok && !put && hit >= 0;
            if (get_hit)
                for (uint32_t i = 0; i < 8; ++i) {
                    uint64_t l = ld_agent(lay.lock(base + kValBase + 8 * hit + i));
                    ok &= !(l & kLockBit);
                    sum1 += l;
                }
            hw_order();
#pragma unroll
            for (uint32_t i = 0; i < 8; ++i) gv[i] = (ok && get_hit) ? lay.load(base + kValBase + 8 * hit + i) : 0u;
        }
        wb.n = 0;
        uint32_t *r = res + 9ull * (act ? ls.txn : 0);
        if (ok && !put) {
            if (hit >= 0) {
                r[0] = 0x100u | (uint32_t)hit;
                for (uint32_t i = 0; i < 8; ++i) r[1 + i] = gv[i];
                wb.put(base + kStampBase + hit, tv);
            } else {
                for (uint32_t i = 0; i < 9; ++i) r[i] = 0u;
            }
        } else if (ok) {
            uint32_t victim = 0, vmin = hdr[17];
#pragma unroll
            for (uint32_t w = 1; w < 8; ++w)
                if (hdr[17 + w] < vmin) {
                    vmin = hdr[17 + w];
                    victim = w;
                }
            if (hit >= 0) victim = (uint32_t)hit;
            uint32_t chk = (uint32_t)mix64(key);
            uint32_t vb = base + kValBase + 8 * victim;
            r[0] = 0x200u | (hit >= 0 ? 0x100u : 0u) | victim;
            wb.put(base + 2 * victim, (uint32_t)key);
            wb.put(base + 2 * victim + 1, (uint32_t)(key >> 32));
            for (uint32_t i = 0; i < 7; ++i) {
                uint32_t v = (uint32_t)mix64(key ^ ((uint64_t)tv << 32) ^ i);
                chk ^= v;
                wb.put(vb + i, v);
                r[1 + i] = v;
            }
            wb.put(vb + 7, chk);
            r[8] = chk;
            wb.put(base + kStampBase + victim, tv);
            wb.put(base + kSetStamp, tv);
        }
        if (ok && wb.n) ok = wb.lock_all(lay);
        hw_order();
        uint32_t ticket;
        if constexpr (Lay::kFused) {
            const bool upd = wb.n != 0;
            const uint32_t wver = wave_fetch_add(&a->hot->clock.v, ok && upd);
            hw_order();
            if (ok && upd && wver != rv) {
                for (uint32_t j = 0; j < nh; ++j) {
                    const uint32_t w = base + header_word(j);
                    const uint64_t l = ld_agent(lay.lock(w));
                    if (((l & kLockBit) && !wb.mine(lay, w)) || Slot::version(l) > rv) ok = false;
                }
                if (get_hit)
                    for (uint32_t i = 0; i < 8; ++i) {
                        const uint32_t w = base + kValBase + 8 * hit + i;
                        const uint64_t l = ld_agent(lay.lock(w));
                        if (((l & kLockBit) && !wb.mine(lay, w)) || Slot::version(l) > rv) ok = false;
                    }
            }
            if (ok && upd && wver >= kClockLimit) {
                latch_error(cnt, HETM_ECAPACITY, ls.txn);
                ok = false;
            }
            // the round's first writes of words go to the undo log
            const uint32_t umask = ok && upd ? wb.first & wb.locked : 0u;
            uint32_t uw[kCacheMaxWrites];
#pragma unroll
            for (uint32_t k = 0; k < kCacheMaxWrites; ++k) uw[k] = wb.at(k < wb.n ? k : 0);
            if (ok && upd)
                wb.commit(lay, wver + 1);
            else if (wb.locked)
                wb.abort(lay);
            if (a->undo_cap) undo_record(a, umask, uw, wb.prev);
            ticket = upd ? 2u * (wver - clock_base) + 1u : 2u * (rv - clock_base);
        } else {
            ticket = wave_fetch_add(&a->hot->ticket.v, ok);
            hw_order();
            if (ok) {
                uint64_t sum2 = 0;
                for (uint32_t j = 0; j < nh && ok; ++j) sum2 += reread(lay, base + header_word(j), wb, ok);
                if (get_hit)
                    for (uint32_t i = 0; i < 8 && ok; ++i) sum2 += reread(lay, base + kValBase + 8 * hit + i, wb, ok);
                ok &= sum2 == sum1;
            }
            if (ok)
                wb.commit(lay);
            else if (wb.locked)
                wb.abort(lay);
        }
        if (ok) {
            for (uint32_t j = 0; j < nh; ++j) rs_mark(rs, div32(base + header_word(j), G));
            if (get_hit)
                for (uint32_t i = 0; i < 8; ++i) rs_mark(rs, div32(base + kValBase + 8 * hit + i, G));
            wb.mark_writes(rs, ws, G);
        }
        settle(ls, act, act && (key == 0 || put > 1), ok, ticket, a->tickets, cnt, a->retry_cap);
    }
    flush_counts(ls, cnt);
}

// The OPLIST kind split: transaction i is an update iff nw[i] != 0.  A
// block takes tiles of kPartPerThread x kPartBlock consecutive transactions
// (grid-stride, so one launch shape serves every batch size): each thread
// classifies kPartPerThread of them, a block scan places them in LDS, one
// atomic per list and tile reserves the tile's range, and the block stores
// both ranges with consecutive threads on consecutive entries; both lists
// hold ascending ids within a tile.  The blocks stay at four waves: with
// queued rounds the split starts beside the previous round's merge copy
// (a copy kernel on every compute unit), and 16-wave blocks made those
// rounds slower.
constexpr uint32_t kPartPerThread = 16;
constexpr uint32_t kPartBlock = 256;
constexpr uint64_t kPartTile = (uint64_t)kPartPerThread * kPartBlock;
constexpr uint32_t kPartMaxBlocks = 1024;

__global__ __launch_bounds__(kPartBlock) void k_partition(const DevArgs *__restrict__ a) {
    __shared__ uint32_t s_sum[kPartBlock / kWave];
    __shared__ uint32_t s_base[2];
    __shared__ uint32_t s_ids[kPartTile];   // read-only ids from the front, update ids from the back
    const uint32_t n = a->n_txns;
    const gmem<uint8_t> *nw = glob(a->nw);
    gmem<uint32_t> *order = glob(a->order);
    const uint32_t lane = lane_id(), wave = threadIdx.x / kWave;
    for (uint64_t tile = blockIdx.x; tile * kPartTile < n; tile += gridDim.x) {
        const uint64_t first = tile * kPartTile + (uint64_t)threadIdx.x * kPartPerThread;
        uint32_t kinds = 0, n_ro = 0, n_upd = 0;
#pragma unroll
        for (uint32_t k = 0; k < kPartPerThread; ++k) {
            if (first + k < n) {
                const uint32_t u = nw[first + k] != 0;
                kinds |= u << k;
                n_upd += u;
                n_ro += 1u - u;
            }
        }
        // block-exclusive prefix of both counts at once (each <= 4096 per tile)
        const uint32_t v = n_ro << 16 | n_upd;
        uint32_t inc = v;
        for (uint32_t o = 1; o < kWave; o <<= 1) {
            const uint32_t t = __shfl_up(inc, o);
            if (lane >= o) inc += t;
        }
        if (lane == kWave - 1) s_sum[wave] = inc;
        __syncthreads();
        uint32_t before = 0, total = 0;
        for (uint32_t w = 0; w < kPartBlock / kWave; ++w) {
            if (w < wave) before += s_sum[w];
            total += s_sum[w];
        }
        if (threadIdx.x == 0) {
            s_base[0] = (total >> 16) ? __hip_atomic_fetch_add(&a->hot->n_ro.v, total >> 16, __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_AGENT) : 0u;
            s_base[1] = (total & 0xFFFFu) ? __hip_atomic_fetch_add(&a->hot->n_upd.v, total & 0xFFFFu,
                                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
        }
        const uint32_t excl = before + inc - v;
        uint32_t pr = excl >> 16, pu = excl & 0xFFFFu;   // within the tile
#pragma unroll
        for (uint32_t k = 0; k < kPartPerThread; ++k) {
            if (first + k < n) {
                if ((kinds >> k) & 1u)
                    s_ids[kPartTile - 1 - pu++] = (uint32_t)(first + k);
                else
                    s_ids[pr++] = (uint32_t)(first + k);
            }
        }
        __syncthreads();
        const uint32_t tot_ro = total >> 16, tot_upd = total & 0xFFFFu, base_ro = s_base[0], base_upd = s_base[1];
        for (uint32_t k = threadIdx.x; k < tot_ro; k += kPartBlock) order[base_ro + k] = s_ids[k];
        for (uint32_t k = threadIdx.x; k < tot_upd; k += kPartBlock)
            order[n - 1 - (base_upd + k)] = s_ids[kPartTile - 1 - k];
        __syncthreads();   // s_sum, s_base and s_ids are reused by the next tile
    }
}

}  // namespace


hipError_t exec_prepare(uint32_t max_ops) {
    const int lds = (int)oplist_lds_bytes(max_ops);
    hipError_t e = hipFuncSetAttribute((const void *)k_exec_oplist<Slot>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void *)k_exec_oplist<Split<uint32_t>>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               lds);
}

void launch_exec(uint32_t program, const DevArgs *a, uint32_t workgroups, uint32_t max_ops, bool slot,
                 uint64_t batch_capacity, hipStream_t s, hipEvent_t exec_started) {
    // the argument upload before these kernels has reset the batch's cursors
    dim3 grid(workgroups), block(kExecWaves * kWave);
    const uint32_t lds = oplist_lds_bytes(max_ops);
    if (program == HETM_PROG_OPLIST) {
        const uint64_t tiles = (batch_capacity + kPartTile - 1) / kPartTile;
        hipLaunchKernelGGL(k_partition, dim3((uint32_t)(tiles < kPartMaxBlocks ? tiles : kPartMaxBlocks)),
                           dim3(kPartBlock), 0, s, a);
    } else {
        // hot objects from a sample, then their chains and the cold list
        const uint64_t tiles = (batch_capacity + kTxTile - 1) / kTxTile;
        const uint32_t tgrid = (uint32_t)(tiles < 512 ? tiles : 512);
        if (program == HETM_PROG_TRANSFER) {
            hipLaunchKernelGGL(k_tx_sample<HETM_PROG_TRANSFER>, dim3(256), dim3(kTxThreads), 0, s, a);
            hipLaunchKernelGGL(k_tx_pick, dim3(kTxTabSlots / kTxThreads), dim3(kTxThreads), 0, s, a);
            hipLaunchKernelGGL(k_tx_classify<HETM_PROG_TRANSFER>, dim3(tgrid), dim3(kTxThreads), 0, s, a);
            hipLaunchKernelGGL(k_tx_plan, dim3(1), dim3(1024), 0, s, a);
            hipLaunchKernelGGL(k_tx_scatter<HETM_PROG_TRANSFER>, dim3(tgrid), dim3(kTxThreads), 0, s, a);
        } else {
            hipLaunchKernelGGL(k_tx_sample<HETM_PROG_CACHE>, dim3(256), dim3(kTxThreads), 0, s, a);
            hipLaunchKernelGGL(k_tx_pick, dim3(kTxTabSlots / kTxThreads), dim3(kTxThreads), 0, s, a);
            hipLaunchKernelGGL(k_tx_classify<HETM_PROG_CACHE>, dim3(tgrid), dim3(kTxThreads), 0, s, a);
            hipLaunchKernelGGL(k_tx_plan, dim3(1), dim3(1024), 0, s, a);
            hipLaunchKernelGGL(k_tx_scatter<HETM_PROG_CACHE>, dim3(tgrid), dim3(kTxThreads), 0, s, a);
        }
    }
    if (exec_started) (void)hipEventRecord(exec_started, s);
    if (program == HETM_PROG_OPLIST) {
        if (slot)
            hipLaunchKernelGGL(k_exec_oplist<Slot>, grid, block, lds, s, a);
        else
            hipLaunchKernelGGL(k_exec_oplist<Split<uint32_t>>, grid, block, lds, s, a);
    } else if (program == HETM_PROG_TRANSFER) {
        hipLaunchKernelGGL(k_exec_transfer, grid, block, 0, s, a);
    } else if (slot) {
        hipLaunchKernelGGL(k_exec_cache<Slot>, grid, block, 0, s, a);
    } else {
        hipLaunchKernelGGL(k_exec_cache<Split<uint32_t>>, grid, block, 0, s, a);
    }
}

}  // namespace hetm
