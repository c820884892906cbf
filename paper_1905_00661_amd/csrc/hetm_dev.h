// hetm_dev.h -- device-side state, argument blocks and CDNA wavefront helpers
// shared by the libhetm kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hetm.h"

namespace hetm {

constexpr uint64_t kLockBit = 1ull << 63;   // lock-table word: bit 63 lock, 0..62 version
constexpr uint64_t kTsLimit = 1ull << 63;   // host timestamps must stay below
constexpr int kWave = 64;
constexpr int kExecWaves = 4;               // waves per transaction-kernel workgroup
constexpr int kOplistMaxWrites = 8;         // LDS write-buffer slots per lane (OPLIST)
constexpr int kCacheMaxWrites = 12;         // a PUT writes key(2) + value(8) + stamp + set stamp
constexpr uint32_t kNoTxn = 0xFFFFFFFFu;
constexpr uint32_t kDoneTxn = 0xFFFFFFFEu;

// Counters the kernels update during a round (device memory).
// Exact 32-bit division by a runtime constant d >= 1 (Lemire, Kaser and
// Kurz, "Faster remainder by direct computation", 2019): with
// M = floor((2^64 - 1) / d) + 1, n / d = high 64 bits of the 128-bit
// product M * n for every 32-bit n.  d = 1 and powers of two use a shift.
struct Div32 {
    uint64_t magic;
    uint32_t shift;
    uint32_t use_shift;
};
inline Div32 make_div32(uint32_t d) {
    Div32 r{0, 0, 0};
    if ((d & (d - 1)) == 0) {
        r.use_shift = 1;
        while ((1u << r.shift) < d) ++r.shift;
    } else {
        r.magic = UINT64_MAX / d + 1;
    }
    return r;
}
__device__ __forceinline__ uint32_t div32(uint32_t n, const Div32 &d) {
    return d.use_shift ? (n >> d.shift) : (uint32_t)__umul64hi(d.magic, (uint64_t)n);
}

// The two counters every wave hits during execution sit on cache lines of
// their own (same-address atomics serialize at ~90 M/s per line).
struct alignas(256) HotCounter {
    uint32_t v;
    uint32_t pad_[63];
};
struct HotCounters {
    HotCounter ticket;            // next commit ticket (split layout)
    HotCounter queue_head;        // next transaction of the current batch (after the static first pass);
                                  // OPLIST: next entry of the read-only list
    HotCounter clock;             // version clock of the slot layout; persists across rounds
    HotCounter queue_upd;         // OPLIST: next entry of the update list; TRANSFER: next hot-account chain
    HotCounter n_ro;              // OPLIST: length of the read-only list (the partition's cursor);
                                  // TRANSFER: hot accounts found by the sample
    HotCounter n_upd;             // OPLIST: length of the update list (the partition's cursor);
                                  // TRANSFER: length of the cold list
};

// Slot layout: versions are clock values, 31 bits wide.  The host resets
// every version (and the clock) between rounds once the clock passes
// kClockReset; a writer that would still reach kClockLimit latches
// HETM_ECAPACITY instead of committing.
// Blocks that count themselves finished do so in groups: same-address
// atomics serialize (about 20 ns apiece here), so a thousand blocks on one
// counter would cost tens of microseconds; the last block of each group then
// counts the group on the top counter.
constexpr uint32_t kSubTickets = 32;
constexpr uint32_t kClockReset = 1u << 30;
constexpr uint32_t kClockLimit = 0x7FFFFFF0u;

struct DevCounters {
    uint32_t conflict;            // OR of the validation flags of the round
    int32_t error;                // first latched error code (HETM_E*), 0 if none
    uint32_t ticket_snapshot;     // tickets handed out in the round (at finish)
    uint32_t clock_base;          // slot layout: the version clock when the round began
    unsigned long long max_ts;    // largest ts of this round's applied log chunks
    unsigned long long floor_ts;  // watermark: largest ts applied by earlier rounds
    unsigned long long committed; // local commits in this round
    unsigned long long retries;   // local aborts in this round
    unsigned long long chunk_max_ts;  // the current chunk's, folded in when it applies
    unsigned long long chunk_min_inv; // bitwise NOT of the current chunk's smallest ts (0: none yet)
    uint32_t n_dirty;             // write-set granules found by the compaction
    uint32_t n_runs;              // maximal runs of consecutive dirty granules
    uint32_t retry_txn;           // first transaction that hit the retry cap
    uint32_t scan_ticket;         // groups of blocks finished in the compaction count pass
    uint32_t err_index;           // index of the first bad log entry / transaction
    uint32_t chunk_conflict;      // the current chunk's flags, folded in when it applies
    uint32_t doomed;              // epoch of the last round early validation doomed
    uint32_t log_ticket;          // blocks finished in the log apply pass
    uint32_t win_pending;         // the last applied chunk's winners have not written their ts yet
    uint32_t n_undo;              // slot layout: undo records of the round (first writes of a word)
    uint32_t undo_over;           // the undo log ran out of room (a conflict restores from the host)
    uint32_t apply_floor;         // slot layout: version of the round's first applied log chunk
                                  // (0xFFFFFFFF before); every word the log wrote carries a version
                                  // at or above it, every word a transaction wrote one below
    uint32_t apply_ver;           // slot layout: version of the chunk being applied
    uint32_t log_spill;           // entries of the current chunk's spill area in use
    uint32_t log_ndesc;           // spill chunks of the current chunk
    uint32_t log_sub[kSubTickets];    // apply blocks finished, per group of blocks (b mod kSubTickets)
    uint32_t scan_sub[kSubTickets];   // compaction count blocks finished, per group of blocks
    uint32_t hold;                // the last finished round needs the host before another may run
                                  // (a latched error, or a CPU-wins conflict without a whole undo log)
};

// Everything a kernel needs: constant context state plus the arguments of
// the current call.  Lives in device memory; kernels receive its address.
struct DevArgs {
    // ---- context (set once)
    void *stmr;
    uint64_t *locks;
    uint64_t *ts;
    uint8_t *rs;            // read set: one byte per granule (see rs_mark)
    uint32_t *ws;
    // the log chunk bucketed by word (validation + apply):
    uint32_t *log_desc;     // [log_tiles * bins][3] spill chunks: first position, entries, next chunk
    uint32_t *log_bstart;   // [bins] first position of each bucket's entries (and of its winners)
    uint32_t *log_bwin;     // [bins] winning entries (one per word) each bucket resolved
    uint32_t *log_head;     // [bins] first spill chunk of each bucket (kLogNone: none; resolve clears)
    uint32_t *log_cursor;   // [bins] entries of each bucket, region and spill (bin pass; resolve clears)
    void *log_sorted;       // [bins * log_region + 2 * log_capacity] the chunk's entries grouped by bucket:
                            // the regions, then the spill area
    void *log_win;          // same size: each bucket's winners, at the bucket's positions
    uint32_t *blocksums;    // compaction: per-block dirty counts, then offsets
    uint32_t *blockruns;
    uint32_t *ids_scratch;  // ceil(N/G) dirty granule ids
    uint32_t *order;        // OPLIST batch split by kind: read-only ids from the front, update ids from the back;
                            // TRANSFER: the hot accounts' chains from the front, the cold list from the back
    uint64_t *undo;         // slot layout: (old value << 32) | word of each word's first write in the round
    uint32_t undo_cap;      // records the undo log holds (0: no undo log, conflicts restore from the host)
    uint32_t pad3_;
    uint64_t *tx_tab;       // TRANSFER: account counts of the batch sample (kTxTabSlots, cleared after use)
    uint64_t *tx_hot;       // TRANSFER: hot accounts, (sample count << 32) | account, one chain each
    uint32_t *tx_chain;     // TRANSFER: per chain counts, first positions (+ total), cursors, and the chain
                            // order (longest first), kTxMaxHot entries each
    DevCounters *cnt;
    HotCounters *hot;
    Div32 gdiv;             // division by G
    uint64_t n_words;
    uint32_t word_bytes;
    uint32_t word_shift;    // 1 in the slot layout: word w's value is u32 number 2w of the replica
    uint32_t granule;       // G
    uint32_t stripe_shift;  // log2(S)
    uint32_t n_granules;    // ceil(N/G)
    uint32_t n_bm_words;    // ceil(n_granules / 32): words of the write-set bitmap
    uint32_t n_rs_words;    // ceil(n_granules / 4): words of the read-set byte map
    uint32_t retry_cap;
    uint32_t max_ops;
    uint32_t n_scan_blocks;
    uint32_t log_bins;      // buckets of a log chunk, a power of two
    uint32_t log_bin_bits;  // log2(log_bins)
    uint32_t log_tiles;     // bin blocks the launch is sized for (log_capacity / tile)
    uint32_t log_region;    // entries each bucket's region holds
    uint32_t log_spill_cap; // entries of the spill area (twice the chunk capacity)
    // ---- current call
    uint32_t program;
    uint32_t n_txns;
    const uint32_t *off;    // OPLIST
    const uint32_t *idx;
    const uint8_t *nw;
    const uint32_t *tid;    // OPLIST, CACHE
    const uint32_t *src;    // TRANSFER
    const uint32_t *dst;
    const uint32_t *amt;
    const uint64_t *key;    // CACHE
    const uint8_t *op;
    void *results;
    uint32_t *tickets;
    const void *log;        // device-resident log chunk
    uint32_t n_log;
    uint32_t *flags;        // nullable
    void *host;             // merge target (pinned host, device-mapped)
    uint32_t *ids_out;      // nullable
    void *staging;          // async merge: packed dirty granules of this round
    uint32_t *stage_ids;    // async merge: their ids
    uint32_t *stage_count;  // async merge: their number
    uint32_t outcome;       // 0 / 1 / HETM_OUTCOME_DEVICE
    uint32_t epoch;         // the open round's number, as early validation tags a doomed round
    uint32_t policy;        // HETM_POLICY_*: who wins an inter-device conflict
    uint32_t gated;         // queued behind a round the host has not collected: runs empty while that
                            // round holds (cnt->hold); an ungated upload lowers the hold
};

// ------------------------------------------------------------------ atomics
// All transactional data (STMR words, lock words) is accessed with
// agent-scope atomics, which gfx950 serves at the device coherence point
// (the per-XCD L2s are not coherent with each other).

template <typename T>
__device__ __forceinline__ T ld_agent(const T *p) {
    return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_agent(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool cas_agent(uint64_t *p, uint64_t expect, uint64_t desired) {
    return __hip_atomic_compare_exchange_strong(p, &expect, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
}
// Global-memory (address space 1) views.  Pointers read out of the argument
// block are generic, so accesses through them compile to flat instructions,
// which count against the LDS/scalar counter as well and force a wait on
// every LDS access between a load and its use; through a global view the
// same accesses are global instructions that only the vector-memory counter
// tracks, so a batch of them stays in flight.
template <typename T>
using gmem = T __attribute__((address_space(1)));
template <typename T>
__device__ __forceinline__ gmem<T> *glob(T *p) {
    return (gmem<T> *)p;
}
template <typename T>
__device__ __forceinline__ const gmem<T> *glob(const T *p) {
    return (const gmem<T> *)p;
}
template <typename T>
__device__ __forceinline__ T ld_agent(const gmem<T> *p) {
    return __hip_atomic_load(const_cast<gmem<T> *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_agent(gmem<T> *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool cas_agent(gmem<uint64_t> *p, uint64_t expect, uint64_t desired) {
    return __hip_atomic_compare_exchange_strong(p, &expect, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void fence_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
__device__ __forceinline__ void fence_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }

// Orders this wave's device-coherent accesses: every earlier vector memory
// operation has completed before any later one issues.  The transactional
// kernels touch shared data only through agent-scope atomics (sc1 loads,
// stores and RMWs, performed at the device coherence point), so completion
// order is all they need; an agent-scope C++ fence would in addition write
// back (release) or invalidate (acquire) the whole XCD L2 for the sake of
// plain accesses, which measures 6x (acquire) to 30x (release) slower than
// the load it orders.  The signal fences keep the compiler from moving
// memory operations across the wait.
__device__ __forceinline__ void hw_order() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ __forceinline__ void latch_error(DevCounters *c, int32_t code, uint32_t where) {
    int32_t zero = 0;
    if (__hip_atomic_compare_exchange_strong(&c->error, &zero, code, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
        st_agent(&c->err_index, where);
}

// ---------------------------------------------------------------- wavefront
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// number of set bits of m below this lane
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Undo log (slot layout): a committed writer that finds a word with a version
// from before the round (at most the round's clock base) writes it first in
// the round and records its old value; entry k of word[] / old[] is recorded
// if bit k of mask is set.  One atomic per wave reserves the wave's records.
// Past the log's room nothing is recorded and the round falls back to
// restoring from the host replica.  Reached by all 64 lanes.
template <int K>
__device__ __forceinline__ void undo_record(const DevArgs *a, uint32_t mask, const uint32_t (&word)[K],
                                            const uint32_t (&old)[K]) {
    const uint32_t lane = __lane_id();
    const uint32_t count = __popc(mask);
    uint32_t inc = count;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(inc, o);
        if ((int)lane >= o) inc += t;
    }
    const uint32_t total = __shfl(inc, 63);
    if (!total) return;
    uint32_t base = 0;
    if (lane == 63)
        base = __hip_atomic_fetch_add(&a->cnt->n_undo, total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    base = __shfl(base, 63) + inc - count;
    if (base + count > a->undo_cap) {
        if (count) __hip_atomic_store(&a->cnt->undo_over, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    uint32_t at = base;
#pragma unroll
    for (int k = 0; k < K; ++k)
        if ((mask >> k) & 1u) a->undo[at++] = ((uint64_t)old[k] << 32) | word[k];
}

// One atomic add per wavefront: lanes with `want` receive consecutive
// values in lane order.  Must be reached by all 64 lanes.
__device__ __forceinline__ uint32_t wave_fetch_add(uint32_t *ctr, bool want) {
    uint64_t m = __ballot(want);
    uint32_t base = 0;
    if (m) {
        int leader = __ffsll((unsigned long long)m) - 1;
        if ((int)lane_id() == leader)
            base = __hip_atomic_fetch_add(ctr, (uint32_t)__popcll(m), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        base = __shfl(base, leader);
    }
    return base + lanes_below(m);
}

// Sets bit g of an agent-visible bitmap; skips the atomic when the bit is
// already set (bits only go 0 -> 1 within a round).  The test load is
// device-coherent so bits set from other XCDs are seen; bitmap lines stay
// cache-resident, so the test costs far less than the atomic it avoids.
__device__ __forceinline__ void bitmap_set(uint32_t *bm, uint32_t g) {
    uint32_t w = g >> 5, b = 1u << (g & 31);
    uint32_t cur = ld_agent(bm + w);
    if (!(cur & b)) __hip_atomic_fetch_or(bm + w, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The read set is a byte map, so marking a granule is an idempotent plain
// byte store instead of an atomic OR on a shared bitmap word (a committed
// transaction marks every granule it read: millions per round).  The L2s
// merge the stores and write back only the bytes they dirtied, and the
// kernel boundary makes every mark visible to validation; early validation,
// running beside the kernel, sees the marks of finished batches and those of
// the running one as their lines are written back.
__device__ __forceinline__ void rs_mark(uint8_t *rs, uint32_t g) { rs[g] = 1; }
__device__ __forceinline__ void rs_mark(gmem<uint8_t> *rs, uint32_t g) { rs[g] = 1; }
__device__ __forceinline__ void bitmap_set(gmem<uint32_t> *bm, uint32_t g) {
    uint32_t w = g >> 5, b = 1u << (g & 31);
    uint32_t cur = ld_agent(bm + w);
    if (!(cur & b)) __hip_atomic_fetch_or(bm + w, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}


// ------------------------------------------------------------- launchers
// Host-side launch wrappers, defined next to their kernels.  `a` is the
// device address of the DevArgs block every kernel reads its arguments from.
void launch_set_args(const DevArgs &host_copy, DevArgs *dev, hipStream_t s);
const void *set_args_kernel();   // host handle of the argument-upload kernel
void launch_clear_error(DevCounters *cnt, hipStream_t s);
// slot: the context keeps u32 words in the slot layout (value, version and
// lock in one u64 per word) instead of a value array plus a lock table
// OPLIST also launches the kind split, sized for batch_capacity transactions;
// exec_started (nullable, not for capture) is recorded on s just before the
// transaction kernel (PLAIN rounds time the kernel with it)
void launch_exec(uint32_t program, const DevArgs *a, uint32_t workgroups, uint32_t max_ops, bool slot,
                 uint64_t batch_capacity, hipStream_t s, hipEvent_t exec_started = nullptr);
// allows the OPLIST kernel the dynamic LDS a context's max_ops needs
hipError_t exec_prepare(uint32_t max_ops);
// dynamic LDS of the OPLIST transaction kernel: each lane's word list
constexpr uint32_t oplist_lds_bytes(uint32_t max_ops) { return kExecWaves * max_ops * kWave * 4u; }
// Validation and apply of one host log chunk (§IV-C.2): launch_validate
// runs the count, scan, scatter and resolve passes, launch_apply the stores.
// bins and tiles are the context's log_bins and log_tiles; later_chunk: the
// round already applied a chunk, whose winners first write their timestamps.
void launch_validate(const DevArgs *a, uint32_t word_bytes, uint32_t bins, uint32_t tiles, bool later_chunk,
                     DevCounters *cnt, hipStream_t s);
void launch_apply(const DevArgs *a, uint32_t word_bytes, uint32_t bins, hipStream_t s);
// Sizing of the bucketed log for a chunk capacity.
constexpr uint32_t kLogTile = 4096;             // entries per bin block
constexpr uint32_t kLogMaxBins = 4096;
constexpr uint32_t kLogNone = 0xFFFFFFFFu;      // end of a bucket's spill-chunk list
uint32_t log_bins_for(uint64_t log_capacity);
// Entries each bucket's region holds: twice the bucket's mean at capacity,
// plus a margin; what does not fit spills.
inline uint32_t log_region_for(uint64_t log_capacity, uint32_t bins) {
    return (uint32_t)(2 * ((log_capacity + bins - 1) / bins) + 64);
}
inline uint32_t log_tiles_for(uint64_t log_capacity) { return (uint32_t)((log_capacity + kLogTile - 1) / kLogTile); }
void launch_compact(const DevArgs *a, uint32_t n_scan_blocks, hipStream_t s);
void launch_copy(const DevArgs *a, uint64_t n_words, uint32_t granule, uint32_t word_bytes, bool slot, hipStream_t s);
void launch_finish(const DevArgs *a, DevCounters *snap, uint32_t n_rs_words, hipStream_t s);
void launch_early_validate(const void *log, uint64_t n, uint32_t word_bytes, const uint8_t *rs, Div32 gdiv,
                           uint64_t n_words, uint32_t epoch, DevCounters *cnt, hipStream_t s);
void launch_gather(const DevArgs *a, uint64_t n_words, uint32_t granule, uint32_t word_bytes, bool slot,
                   hipStream_t s);
void launch_restore(void *stmr, const void *host, const uint32_t *ids, const uint32_t *count, uint64_t n_words,
                    uint32_t granule, uint32_t word_bytes, bool slot, hipStream_t s);
// the device-side rollback of a conflicting round from the undo log; nothing
// for a context without one
void launch_undo(const DevArgs *a, uint32_t undo_cap, hipStream_t s);
void launch_to_slots(const uint32_t *src, uint64_t *slots, uint64_t n, hipStream_t s);
void launch_version_reset(uint64_t *slots, uint64_t n, HotCounters *hot, DevCounters *cnt, hipStream_t s);
void launch_from_slots(const uint64_t *slots, uint32_t *dst, uint64_t n, hipStream_t s);

constexpr uint32_t kScanWordsPerBlock = 2048;   // bitmap words per compaction block
constexpr uint32_t kTxMaxHot = 4096;            // TRANSFER: most hot-account chains per batch
constexpr uint32_t kTxTabBits = 18;
constexpr uint32_t kTxTabSlots = 1u << kTxTabBits;   // TRANSFER: sample count table
constexpr uint32_t kTxChainWords = 4 * kTxMaxHot + 1;
constexpr uint32_t kScanThreads = 256;

}  // namespace hetm
