// log_apply.hip -- validation and apply of a host log chunk (§IV-C.2) on
// gfx950, with the chunk bucketed by word so that every word's entries meet
// in one workgroup's LDS and the apply needs no atomics on the timestamps.
//
//  bin      : one coalesced read of the chunk.  Checks each entry's
//             preconditions (word < N, watermark < ts < 2^63), tests it
//             against the read set (one ballot gives 64 flag bits), keeps the
//             chunk's largest and smallest ts, counts its entries per bucket
//             (a multiplicative hash of the word) in an LDS histogram, takes
//             the tile's share of every bucket's region (twice the bucket's
//             mean size) with one atomic per bucket, groups the tile by
//             bucket in LDS and writes each bucket's run with consecutive
//             threads.  A run that does not fit in its region (a log that
//             hammers a few words) goes to a chunk of the spill area linked
//             to its bucket.
//  resolve  : a bucket that spilled is first copied into one range of the
//             spill area.  One workgroup per bucket builds an LDS hash table
//             keyed by word:
//             the largest ts of each word and the one entry carrying it; a
//             second entry at a word's winning ts, or a winning ts equal to
//             the one an earlier chunk of the round applied, is an ordering
//             error.  The winners (one per word) are written back at the
//             bucket's positions.
//  apply    : unless a pass latched an error, every winner stores its value
//             with a plain store.  A chunk that fails any check therefore
//             applies nothing.
//
// Timestamps (TS) leave the hot path.  Every entry's ts is above the
// watermark, the largest ts of any earlier round, so an entry is fresher than
// anything earlier rounds applied to its word: a round's first chunk needs no
// TS at all.  Only a later chunk of the same round must meet the winners of
// the round's earlier chunks, so before such a chunk the previous chunk's
// winners (still bucketed) write their ts into TS, and the chunk's resolve
// reads TS once per distinct word if its smallest ts does not exceed what the
// round applied so far.  Words last written in earlier rounds keep an older
// TS, at most the watermark, which no later entry can tie or lose to.
#include "hetm_dev.h"


namespace hetm {

uint32_t log_bins_for(uint64_t log_capacity) {
    // about 1024 entries per bucket at capacity, so that a bucket's resolve
    // takes one pass (up to 2048 entries) with a wide margin
    uint64_t want = (log_capacity + 1023) / 1024;
    uint32_t b = 16;
    while (b < want && b < kLogMaxBins) b <<= 1;
    return b;
}

namespace {

constexpr uint32_t kThreads = 256;                       // apply and ts write-back blocks
constexpr uint32_t kTileThreads = 1024;                  // bin blocks
constexpr uint32_t kPerThread = kLogTile / kTileThreads; // 4 entries per thread in bin
constexpr uint32_t kResThreads = 512;                    // resolve blocks
constexpr uint32_t kTableBits = 12;
constexpr uint32_t kTable = 1u << kTableBits;            // LDS hash-table slots per resolve block
constexpr uint32_t kRegs = 4;                            // entries a resolve thread holds per pass
constexpr uint32_t kPassEntries = kResThreads * kRegs;   // entries per resolve pass (table at most half full)
constexpr uint32_t kNoEntry = 0xFFFFFFFFu;
constexpr uint32_t kEmpty = 0xFFFFFFFFu;                 // free table slot (words are below 2^32 - 1)

struct Entry4 {
    uint32_t word;
    uint32_t value;
    uint64_t ts;
};
struct Entry8 {
    uint32_t word;
    uint32_t pad;
    uint64_t value;
    uint64_t ts;
};

__device__ __forceinline__ uint32_t bucket_of(uint32_t w, uint32_t bits) {
    return (uint32_t)(((uint64_t)(w * 0x9E3779B1u) << bits) >> 32);
}
// table slot of a word within its bucket (other bits of another product)
__device__ __forceinline__ uint32_t slot_of(uint32_t w) { return (w * 0xC2B2AE35u) >> (32 - kTableBits); }
// resolve pass of a word when a bucket needs several: 24 bits of another
// product scaled to [0, npass) by a multiply and a shift (no division: the
// compiled remainder by a run-time divisor was off for some values)
__device__ __forceinline__ uint32_t pass_of(uint32_t w, uint32_t npass) {
    return (uint32_t)(((uint64_t)((w * 0x85EBCA6Bu) >> 8) * npass) >> 24);
}

__device__ __forceinline__ void store_bits(uint32_t *dst, uint64_t kb, uint64_t m, uint32_t nwords) {
    uint64_t w = kb >> 5;
    dst[w] = (uint32_t)m;
    if (w + 1 < nwords) dst[w + 1] = (uint32_t)(m >> 32);
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
    for (int o = 32; o > 0; o >>= 1) {
        uint64_t t = __shfl_xor((unsigned long long)v, o);
        v = t > v ? t : v;
    }
    return v;
}

// exclusive prefix sum over a block of NT threads (every thread calls it);
// *total gets the sum
template <uint32_t NT>
__device__ __forceinline__ uint32_t block_scan(uint32_t v, uint32_t *sh, uint32_t *total) {
    const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
    uint32_t inc = v;
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t t = __shfl_up(inc, o);
        if ((int)lane >= o) inc += t;
    }
    if (lane == kWave - 1) sh[wv] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (uint32_t i = 0; i < NT / kWave; ++i) {
        before += i < wv ? sh[i] : 0u;
        all += sh[i];
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

// --------------------------------------------------------------------- bin
template <typename E>
__global__ __launch_bounds__(kTileThreads) void k_log_bin(const DevArgs *__restrict__ a) {
    __shared__ uint32_t hist[kLogMaxBins];   // the tile's count per bucket, then its run's start in stage
    __shared__ uint32_t base[kLogMaxBins];   // the run's start in the bucket's region (past its end: spilled)
    __shared__ uint32_t spill[kLogMaxBins];  // where the run's spilled part starts in the spill area
    __shared__ E stage[kLogTile];            // the tile's entries grouped by bucket
    __shared__ unsigned long long s_mx[kTileThreads / kWave], s_mn[kTileThreads / kWave];
    __shared__ uint32_t s_cf[kTileThreads / kWave];
    __shared__ uint32_t sh[kTileThreads / kWave];
    const uint64_t n = a->n_log;
    const uint64_t t0 = (uint64_t)blockIdx.x * kLogTile;
    if (t0 >= n) return;
    if (blockIdx.x == 0 && threadIdx.x == 0 && a->word_shift) {
        // slot layout: the chunk's writes get a version of their own, above
        // every version the round's transactions wrote (the undo log tells
        // the two apart)
        DevCounters *c0 = a->cnt;
        const uint32_t v = __hip_atomic_fetch_add(&a->hot->clock.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
        if (v >= kClockLimit) latch_error(c0, HETM_ECAPACITY, 0);
        st_agent(&c0->apply_ver, v);
        if (ld_agent(&c0->apply_floor) == 0xFFFFFFFFu) st_agent(&c0->apply_floor, v);
    }
    const uint32_t B = a->log_bins, bbits = a->log_bin_bits;
    for (uint32_t i = threadIdx.x; i < B; i += kTileThreads) hist[i] = 0;
    __syncthreads();
    const E *log = (const E *)a->log;
    const uint64_t N = a->n_words;
    const Div32 G = a->gdiv;
    const uint8_t *rs = a->rs;
    uint32_t *flags = a->flags;
    DevCounters *cnt = a->cnt;
    const uint64_t floor_ts = ld_agent(&cnt->floor_ts);
    const uint32_t nflagw = (uint32_t)((n + 31) / 32);
    const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
    E e[kPerThread];
#pragma unroll
    for (uint32_t j = 0; j < kPerThread; ++j) {
        const uint64_t k = t0 + j * kTileThreads + threadIdx.x;
        e[j] = log[k < n ? k : n - 1];      // in bounds; entries past n are not used
    }
    bool ok[kPerThread];
    uint8_t hit[kPerThread];
    uint64_t mx = 0, mninv = 0;
#pragma unroll
    for (uint32_t j = 0; j < kPerThread; ++j) {
        const uint64_t k = t0 + j * kTileThreads + threadIdx.x;
        ok[j] = false;
        hit[j] = 0;
        if (k < n) {
            if (e[j].word >= N) {
                latch_error(cnt, HETM_EINVAL, (uint32_t)k);
            } else if (e[j].ts <= floor_ts || e[j].ts >= kTsLimit) {
                latch_error(cnt, HETM_EORDER, (uint32_t)k);
            } else {
                ok[j] = true;
                // the read-set loads go out together; the map was written by
                // earlier kernels, so plain loads see it
                hit[j] = rs[div32(e[j].word, G)];
                mx = e[j].ts > mx ? e[j].ts : mx;
                mninv = ~e[j].ts > mninv ? ~e[j].ts : mninv;
            }
        }
    }
    bool conflict = false;
    uint32_t bk[kPerThread], rank[kPerThread];
#pragma unroll
    for (uint32_t j = 0; j < kPerThread; ++j) {
        bk[j] = bucket_of(e[j].word, bbits);
        rank[j] = ok[j] ? atomicAdd(&hist[bk[j]], 1u) : 0u;
        const uint64_t m = __ballot(ok[j] && hit[j] != 0);
        const uint64_t kb = t0 + j * kTileThreads + wv * kWave;
        if (flags && lane == 0 && kb < n) store_bits(flags, kb, m, nflagw);
        conflict |= m != 0;
    }
    __syncthreads();
    // each bucket's run of this tile: its place in the bucket's region (one
    // atomic per bucket the tile touches), a spill chunk linked to the bucket
    // for the part that does not fit, and its start in the tile grouped by
    // bucket (an exclusive scan of the counts); thread t owns buckets
    // [t per, (t + 1) per)
    const uint32_t C = a->log_region;
    const uint32_t per = (B + kTileThreads - 1) / kTileThreads, b0 = threadIdx.x * per;
    uint32_t mine = 0;
    for (uint32_t i = b0; i < b0 + per && i < B; ++i) {
        const uint32_t h = hist[i];
        uint32_t at = 0, sp = kLogNone;
        if (h) {
            at = __hip_atomic_fetch_add(&a->log_cursor[i], h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t fit = at >= C ? 0u : (C - at < h ? C - at : h);
            if (fit < h) {
                const uint32_t rest = h - fit;
                sp = __hip_atomic_fetch_add(&cnt->log_spill, rest, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t d = __hip_atomic_fetch_add(&cnt->log_ndesc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((uint64_t)sp + rest > a->log_spill_cap || d >= a->log_tiles * B) {
                    latch_error(cnt, HETM_ECAPACITY, i);    // the area holds the chunk twice: not reached
                    sp = kLogNone;
                } else {
                    uint32_t *dd = a->log_desc + 3ull * d;
                    dd[0] = sp;
                    dd[1] = rest;
                    dd[2] = __hip_atomic_exchange(&a->log_head[i], d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
        base[i] = at;
        spill[i] = sp;
        mine += h;
    }
    uint32_t placed;
    uint32_t run = block_scan<kTileThreads>(mine, sh, &placed);
    for (uint32_t i = b0; i < b0 + per && i < B; ++i) {
        const uint32_t h = hist[i];
        hist[i] = run;
        run += h;
    }
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < kPerThread; ++j)
        if (ok[j]) stage[hist[bk[j]] + rank[j]] = e[j];
    __syncthreads();
    // every entry into its bucket's region or spill chunk, each run by
    // consecutive threads
    E *out = (E *)a->log_sorted;
    const uint64_t spill_base = (uint64_t)B * C;
    for (uint32_t k = threadIdx.x; k < placed; k += kTileThreads) {
        const E x = stage[k];
        const uint32_t bx = bucket_of(x.word, bbits);
        const uint32_t q = k - hist[bx], at = base[bx], p = at + q;
        if (p < C) {
            out[(uint64_t)bx * C + p] = x;
        } else if (spill[bx] != kLogNone) {
            out[spill_base + spill[bx] + (q - (at >= C ? 0u : C - at))] = x;
        }
    }
    // the chunk's ts range and conflict, staged (a chunk that fails a check
    // must not count) with at most one atomic per block and counter, and only
    // when it raises the value: same-address atomics serialize
    mx = wave_max_u64(mx);
    mninv = wave_max_u64(mninv);
    const uint64_t cf = __ballot(conflict);
    if (lane == 0) {
        s_mx[wv] = mx;
        s_mn[wv] = mninv;
        s_cf[wv] = cf != 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long bm = 0, bn = 0;
        uint32_t bc = 0;
        for (uint32_t i = 0; i < kTileThreads / kWave; ++i) {
            bm = s_mx[i] > bm ? s_mx[i] : bm;
            bn = s_mn[i] > bn ? s_mn[i] : bn;
            bc |= s_cf[i];
        }
        if (bm > ld_agent(&cnt->chunk_max_ts))
            __hip_atomic_fetch_max(&cnt->chunk_max_ts, bm, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (bn > ld_agent(&cnt->chunk_min_inv))
            __hip_atomic_fetch_max(&cnt->chunk_min_inv, bn, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (bc && !ld_agent(&cnt->chunk_conflict))
            __hip_atomic_fetch_or(&cnt->chunk_conflict, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ----------------------------------------------------------------- resolve
// LDS table of one bucket: the word (kEmpty = free), its largest ts (bit 63
// set once a second entry carrying it shows up) and the bucket position of
// the entry carrying it (kNoEntry until one claims it).
// A pass takes up to kPassEntries entries, kRegs per thread in registers; a
// bucket of more entries is resolved in several passes, each over the words
// of one hash class, streaming the bucket twice per pass.
struct Table {
    uint32_t key[kTable];
    unsigned long long maxts[kTable];
    uint32_t idx[kTable];
};

__device__ __forceinline__ uint32_t table_insert(uint32_t *key, uint32_t w) {
    uint32_t s = slot_of(w);
    for (uint32_t i = 0; i < kTable; ++i, s = (s + 1) & (kTable - 1)) {
        const uint32_t old = atomicCAS(&key[s], kEmpty, w);
        if (old == kEmpty || old == w) return s;
    }
    return kTable;
}
__device__ __forceinline__ uint32_t table_find(const uint32_t *key, uint32_t w) {
    uint32_t s = slot_of(w);
    for (uint32_t i = 0; i < kTable; ++i, s = (s + 1) & (kTable - 1)) {
        const uint32_t k = key[s];
        if (k == w) return s;
        if (k == kEmpty) return kTable;
    }
    return kTable;
}

template <typename E>
__device__ __forceinline__ void load_group(const E *in, uint32_t c, uint32_t g0, E (&e)[kRegs], uint32_t (&pos)[kRegs]) {
#pragma unroll
    for (uint32_t r = 0; r < kRegs; ++r) {
        const uint32_t i = g0 + r * kResThreads + threadIdx.x;
        pos[r] = i < c ? i : kNoEntry;
        e[r] = in[i < c ? i : 0];
    }
}

template <typename E>
__global__ __launch_bounds__(kResThreads) void k_log_resolve(const DevArgs *__restrict__ a) {
    __shared__ Table t;
    __shared__ uint32_t s_nwin, s_at;
    DevCounters *cnt = a->cnt;
    const uint32_t b = blockIdx.x;
    if (b >= a->log_bins) return;
    // the bucket's entry count and spill chunks, read and cleared for the
    // next chunk (also when the chunk failed a check)
    const uint32_t c = ld_agent(&a->log_cursor[b]);
    const uint32_t head = ld_agent(&a->log_head[b]);
    __syncthreads();
    if (threadIdx.x == 0) {
        a->log_cursor[b] = 0;
        a->log_head[b] = kLogNone;
    }
    // an empty chunk leaves the bucket starts unwritten (and apply stores nothing)
    if (a->n_log == 0 || ld_agent(&cnt->error)) return;
    const uint32_t C = a->log_region;
    uint32_t s0 = b * C;
    if (head != kLogNone) {
        // the bucket outgrew its region: the region (full) and its spill
        // chunks are copied into one range of the spill area, where its
        // winners go too
        if (threadIdx.x == 0)
            s_at = __hip_atomic_fetch_add(&cnt->log_spill, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const uint32_t at = s_at;
        if ((uint64_t)at + c > a->log_spill_cap) {    // the area holds the chunk twice: not reached
            if (threadIdx.x == 0) {
                latch_error(cnt, HETM_ECAPACITY, b);
                a->log_bwin[b] = 0;
            }
            return;
        }
        const uint32_t sb = a->log_bins * C;
        E *sorted = (E *)a->log_sorted;
        E *dst = sorted + sb + at;
        for (uint32_t i = threadIdx.x; i < C; i += kResThreads) dst[i] = sorted[s0 + i];
        uint32_t off = C;
        for (uint32_t d = head; d != kLogNone;) {
            const uint32_t *dd = a->log_desc + 3ull * d;
            const uint32_t st = dd[0], cn = dd[1];
            for (uint32_t i = threadIdx.x; i < cn; i += kResThreads) dst[off + i] = sorted[sb + st + i];
            off += cn;
            d = dd[2];
        }
        __syncthreads();    // the copy is read back by the whole block
        s0 = sb + at;
    }
    if (threadIdx.x == 0) a->log_bstart[b] = s0;     // for apply and the ts write-back
    if (c == 0) {
        if (threadIdx.x == 0) a->log_bwin[b] = 0;
        return;
    }
    // a chunk whose smallest ts does not exceed what earlier chunks of the
    // round applied must meet their winners, which TS holds
    const bool slow = ~ld_agent(&cnt->chunk_min_inv) <= ld_agent(&cnt->max_ts);
    const E *in = (const E *)a->log_sorted + s0;
    E *win = (E *)a->log_win + s0;
    const uint64_t *ts = a->ts;
    const uint32_t npass = (c + kPassEntries - 1) / kPassEntries;
    if (threadIdx.x == 0) s_nwin = 0;
    E e[kRegs];
    uint32_t pos[kRegs], sl[kRegs];
    for (uint32_t p = 0; p < npass; ++p) {
        for (uint32_t s = threadIdx.x; s < kTable; s += kResThreads) {
            t.key[s] = kEmpty;
            t.maxts[s] = 0;
            t.idx[s] = kNoEntry;
        }
        __syncthreads();
        // each word's largest ts
        for (uint32_t g0 = 0; g0 < c; g0 += kPassEntries) {
            load_group(in, c, g0, e, pos);
#pragma unroll
            for (uint32_t r = 0; r < kRegs; ++r) {
                if (pos[r] != kNoEntry && npass > 1 && pass_of(e[r].word, npass) != p) pos[r] = kNoEntry;
                sl[r] = pos[r] != kNoEntry ? table_insert(t.key, e[r].word) : kTable;
                if (pos[r] != kNoEntry && sl[r] == kTable) latch_error(cnt, HETM_ECAPACITY, e[r].word);
                if (sl[r] < kTable) atomicMax(&t.maxts[sl[r]], (unsigned long long)e[r].ts);
            }
        }
        __syncthreads();
        // the entry carrying it claims the slot; a second one is a tie
        for (uint32_t g0 = 0; g0 < c; g0 += kPassEntries) {
            if (npass > 1) {       // one pass keeps its entries and slots in registers
                load_group(in, c, g0, e, pos);
#pragma unroll
                for (uint32_t r = 0; r < kRegs; ++r) {
                    if (pos[r] != kNoEntry && pass_of(e[r].word, npass) != p) pos[r] = kNoEntry;
                    sl[r] = pos[r] != kNoEntry ? table_find(t.key, e[r].word) : kTable;
                }
            }
#pragma unroll
            for (uint32_t r = 0; r < kRegs; ++r) {
                if (sl[r] >= kTable || e[r].ts != t.maxts[sl[r]]) continue;
                if (atomicCAS(&t.idx[sl[r]], kNoEntry, pos[r]) != kNoEntry)
                    atomicOr(&t.maxts[sl[r]], (unsigned long long)kTsLimit);   // a tie (ts are below 2^63)
            }
        }
        __syncthreads();
        // the winners
        for (uint32_t s = threadIdx.x; s < kTable; s += kResThreads) {
            const uint32_t w = t.key[s];
            if (w == kEmpty) continue;
            const uint64_t m = t.maxts[s] & (kTsLimit - 1);
            if (slow) {
                const uint64_t old = ts[w];
                if (old > m) continue;            // an earlier chunk's entry is fresher (ties below it pass)
                if (old == m) {                   // ties the winner of an earlier chunk
                    latch_error(cnt, HETM_EORDER, w);
                    continue;
                }
            }
            if (t.maxts[s] & kTsLimit) {          // two entries carry the word's winning ts
                latch_error(cnt, HETM_EORDER, w);
                continue;
            }
            win[atomicAdd(&s_nwin, 1u)] = in[t.idx[s]];   // the winning entry (the bucket is cache-resident)
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) a->log_bwin[b] = s_nwin;
}

// ------------------------------------------------------------------- apply
// Block b stores bucket b's winners.  Under GPU wins with a conflict the
// host's round is discarded: nothing is stored and the chunk's granules join
// the write set, so the merge copies the GPU's values over the host's writes.
// The last block folds the chunk's outcome and ts range into the round's,
// marks the winners as the round's last applied chunk and clears the chunk's
// counters (no block reads them after its ticket).
template <typename E, typename V>
__global__ __launch_bounds__(kThreads) void k_log_apply(const DevArgs *__restrict__ a) {
    __shared__ uint32_t s_last;
    DevCounters *cnt = a->cnt;
    if (ld_agent(&cnt->error)) return;   // a chunk that failed a check applies nothing
    const bool discard = a->policy == HETM_POLICY_GPU_WINS && ld_agent(&cnt->chunk_conflict) != 0;
    const uint32_t b = blockIdx.x;
    if (b < a->log_bins && a->n_log) {
        const uint32_t s0 = a->log_bstart[b], nw = a->log_bwin[b];
        const E *win = (const E *)a->log_win + s0;
        if (discard) {
            const Div32 G = a->gdiv;
            for (uint32_t i = threadIdx.x; i < nw; i += kThreads) bitmap_set(a->ws, div32(win[i].word, G));
        } else if (a->word_shift) {
            // slot layout: value and the chunk's version in one store
            uint64_t *slots = (uint64_t *)a->stmr;
            const uint64_t ver = (uint64_t)(ld_agent(&cnt->apply_ver) & 0x7FFFFFFFu) << 32;
            for (uint32_t i0 = 0; i0 < nw; i0 += kRegs * kThreads) {
                E e[kRegs];
#pragma unroll
                for (uint32_t r = 0; r < kRegs; ++r) {
                    const uint32_t i = i0 + r * kThreads + threadIdx.x;
                    e[r] = win[i < nw ? i : 0];
                }
#pragma unroll
                for (uint32_t r = 0; r < kRegs; ++r)
                    if (i0 + r * kThreads + threadIdx.x < nw) slots[e[r].word] = ver | (uint32_t)e[r].value;
            }
        } else {
            V *stmr = (V *)a->stmr;
            for (uint32_t i0 = 0; i0 < nw; i0 += kRegs * kThreads) {
                E e[kRegs];
#pragma unroll
                for (uint32_t r = 0; r < kRegs; ++r) {
                    const uint32_t i = i0 + r * kThreads + threadIdx.x;
                    e[r] = win[i < nw ? i : 0];
                }
#pragma unroll
                for (uint32_t r = 0; r < kRegs; ++r)
                    if (i0 + r * kThreads + threadIdx.x < nw) stmr[e[r].word] = (V)e[r].value;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // the last block folds the chunk's outcome in: a count of finished
        // blocks per group, then of finished groups
        const uint32_t g = b % kSubTickets, ng = gridDim.x < kSubTickets ? gridDim.x : kSubTickets;
        const uint32_t in_g = (gridDim.x - g + kSubTickets - 1) / kSubTickets;
        bool last = false;
        if (__hip_atomic_fetch_add(&cnt->log_sub[g], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == in_g - 1)
            last = __hip_atomic_fetch_add(&cnt->log_ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == ng - 1;
        s_last = last;
    }
    __syncthreads();
    if (!s_last || threadIdx.x != 0) return;
    for (uint32_t g = 0; g < kSubTickets; ++g) st_agent(&cnt->log_sub[g], 0u);
    st_agent(&cnt->log_spill, 0u);
    st_agent(&cnt->log_ndesc, 0u);
    if (ld_agent(&cnt->chunk_conflict)) st_agent(&cnt->conflict, 1u);
    const unsigned long long m = ld_agent(&cnt->chunk_max_ts);
    if (!discard && m > ld_agent(&cnt->max_ts)) st_agent(&cnt->max_ts, m);
    if (!discard && a->n_log) st_agent(&cnt->win_pending, 1u);
    st_agent(&cnt->chunk_conflict, 0u);
    st_agent(&cnt->chunk_max_ts, 0ull);
    st_agent(&cnt->chunk_min_inv, 0ull);
    st_agent(&cnt->log_ticket, 0u);
}

// ----------------------------------------------------------- ts write-back
// Before a later chunk of the same round: the last applied chunk's winners
// (bucket starts, counts and entries still in place) write their ts into TS.
template <typename E>
__global__ __launch_bounds__(kThreads) void k_log_ts(const DevArgs *__restrict__ a) {
    DevCounters *cnt = a->cnt;
    if (!ld_agent(&cnt->win_pending)) return;
    const uint32_t b = blockIdx.x;
    if (b < a->log_bins) {
        const uint32_t s0 = a->log_bstart[b], nw = a->log_bwin[b];
        const E *win = (const E *)a->log_win + s0;
        uint64_t *ts = a->ts;
        for (uint32_t i = threadIdx.x; i < nw; i += kThreads) {
            const E e = win[i];
            ts[e.word] = e.ts;
        }
    }
}

// The pending flag goes down once every block has read it.
__global__ void k_log_ts_done(DevCounters *cnt) {
    if (threadIdx.x == 0) st_agent(&cnt->win_pending, 0u);
}

}  // namespace

void launch_validate(const DevArgs *a, uint32_t word_bytes, uint32_t bins, uint32_t tiles, bool later_chunk,
                     DevCounters *cnt, hipStream_t s) {
    if (word_bytes == 4) {
        if (later_chunk) {
            hipLaunchKernelGGL(k_log_ts<Entry4>, dim3(bins), dim3(kThreads), 0, s, a);
            hipLaunchKernelGGL(k_log_ts_done, dim3(1), dim3(64), 0, s, cnt);
        }
        hipLaunchKernelGGL(k_log_bin<Entry4>, dim3(tiles), dim3(kTileThreads), 0, s, a);
        hipLaunchKernelGGL(k_log_resolve<Entry4>, dim3(bins), dim3(kResThreads), 0, s, a);
    } else {
        if (later_chunk) {
            hipLaunchKernelGGL(k_log_ts<Entry8>, dim3(bins), dim3(kThreads), 0, s, a);
            hipLaunchKernelGGL(k_log_ts_done, dim3(1), dim3(64), 0, s, cnt);
        }
        hipLaunchKernelGGL(k_log_bin<Entry8>, dim3(tiles), dim3(kTileThreads), 0, s, a);
        hipLaunchKernelGGL(k_log_resolve<Entry8>, dim3(bins), dim3(kResThreads), 0, s, a);
    }
}

void launch_apply(const DevArgs *a, uint32_t word_bytes, uint32_t bins, hipStream_t s) {
    if (word_bytes == 4)
        hipLaunchKernelGGL((k_log_apply<Entry4, uint32_t>), dim3(bins), dim3(kThreads), 0, s, a);
    else
        hipLaunchKernelGGL((k_log_apply<Entry8, uint64_t>), dim3(bins), dim3(kThreads), 0, s, a);
}

}  // namespace hetm
