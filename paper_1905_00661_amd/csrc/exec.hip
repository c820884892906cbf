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
            if (ok && upd)
                wb.commit(lay, wv + 1);
            else if (wb.locked)
                wb.abort(lay);
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

// ---------------------------------------------------------------- TRANSFER
// Reads balances of src and dst (int64 words); if src != dst and the source
// balance covers amt, moves amt.  Results: [bs | bd | applied] (3 x n int64).
__global__ __launch_bounds__(kExecWaves *kWave) void k_exec_transfer(const DevArgs *__restrict__ a) {
    __shared__ uint32_t s_addr[kExecWaves][2][kWave];
    __shared__ uint64_t s_val[kExecWaves][2][kWave];
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
    LaneState ls = first_txn(n);

    while (refill(ls, a->hot, n)) {
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
constexpr uint32_t kSetWords = 128, kStampBase = 16, kSetStamp = 24, kValBase = 32;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {   // splitmix64 finalizer
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// j-th word of the header read list: 8 keys (16 words), set stamp, 8 stamps
__device__ __forceinline__ uint32_t header_word(uint32_t j) {
    return j < 16 ? j : (j == 16 ? kSetStamp : kStampBase + (j - 17));
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
    LaneState ls = first_txn(n);

    while (refill(ls, a->hot, n)) {
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
            base = (uint32_t)(((mix64(key) & (nsets - 1) & ~1ull) | (key & 1ull)) * kSetWords);
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
            if (ok && upd)
                wb.commit(lay, wver + 1);
            else if (wb.locked)
                wb.abort(lay);
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

__global__ void k_begin_batch(const DevArgs *__restrict__ a) {
    if (threadIdx.x == 0) {
        st_agent(&a->hot->queue_head.v, 0u);
        st_agent(&a->hot->queue_upd.v, 0u);
        st_agent(&a->hot->n_ro.v, 0u);
        st_agent(&a->hot->n_upd.v, 0u);
    }
}

// The OPLIST kind split: transaction i is an update iff nw[i] != 0.  A
// block takes tiles of kPartPerThread x kPartBlock consecutive transactions
// (grid-stride, so one launch shape serves every batch size): each thread
// classifies kPartPerThread of them, a block scan places them in LDS, one
// atomic per list and tile reserves the tile's range, and the block stores
// both ranges with consecutive threads on consecutive entries; both lists
// hold ascending ids within a tile.
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
    hipLaunchKernelGGL(k_begin_batch, dim3(1), dim3(64), 0, s, a);
    dim3 grid(workgroups), block(kExecWaves * kWave);
    const uint32_t lds = oplist_lds_bytes(max_ops);
    if (program == HETM_PROG_OPLIST) {
        const uint64_t tiles = (batch_capacity + kPartTile - 1) / kPartTile;
        hipLaunchKernelGGL(k_partition, dim3((uint32_t)(tiles < kPartMaxBlocks ? tiles : kPartMaxBlocks)),
                           dim3(kPartBlock), 0, s, a);
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
