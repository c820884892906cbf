// round.hip -- early validation, merge and reset of one SHeTM round
// (§IV-C.3, §IV-D) for gfx950.  Validation and apply of the host log are in
// log_apply.hip.
//
//  compact  : popcount + prefix sum over the write-set bitmap (per-block
//             counts, the last block scans the block sums, then each block
//             emits ascending dirty granule ids); runs of consecutive ids are
//             counted from run-start bits.
//  copy     : moves the dirty granules between the GPU replica and the
//             device-mapped pinned host replica, GPU->host on success and
//             host->GPU on conflict; the direction is read on the device.
//  finish   : snapshots the round's counters, clears the bitmaps and raises
//             the timestamp watermark.
#include "hetm_dev.h"

namespace hetm {

namespace {

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

// -------------------------------------------------------- early validation
// Validation only (no apply) of a host log chunk against the read-set bitmap
// as it stands while the batch still executes (§IV-D, early validation).  A
// hit dooms the round: the CPU wins, so the transaction kernel stops at its
// next iteration.  Missing a conflict here is harmless -- the validation at
// the end of the round sees the final bitmap -- so entries failing the
// preconditions are simply skipped (the final validation reports them).
template <typename E>
__global__ __launch_bounds__(256) void k_early_validate(const E *__restrict__ log, uint64_t n, const uint8_t *rs,
                                                        Div32 G, uint64_t N, uint32_t epoch, DevCounters *cnt) {
    bool hit = false;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < n && !hit; k += stride) {
        const E e = log[k];
        if (e.word >= N) continue;
        const uint32_t g = div32(e.word, G);
        hit = ld_agent(&rs[g]) != 0;
    }
    if (__ballot(hit) && lane_id() == 0) st_agent(&cnt->doomed, epoch);
}

// ------------------------------------------------------------------ compact
constexpr uint32_t kWordsPerThread = kScanWordsPerBlock / kScanThreads;   // 8

__device__ __forceinline__ uint32_t block_sum(uint32_t v, uint32_t *sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const uint32_t wv = threadIdx.x / kWave;
    if (lane_id() == 0) sh[wv] = v;
    __syncthreads();
    uint32_t t = 0;
    for (uint32_t i = 0; i < kScanThreads / kWave; ++i) t += sh[i];
    __syncthreads();
    return t;
}

// exclusive prefix of v over the block (256 threads)
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *sh, uint32_t &total) {
    const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
    uint32_t inc = v;
    for (int o = 1; o < kWave; o <<= 1) {
        uint32_t t = __shfl_up(inc, o);
        if ((int)lane >= o) inc += t;
    }
    if (lane == kWave - 1) sh[wv] = inc;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
    for (uint32_t i = 0; i < kScanThreads / kWave; ++i) {
        if (i < wv) before += sh[i];
        total += sh[i];
    }
    __syncthreads();
    return before + inc - v;
}

__global__ __launch_bounds__(kScanThreads) void k_compact_count(const DevArgs *__restrict__ a) {
    __shared__ uint32_t sh[kScanThreads / kWave];
    __shared__ uint32_t s_last;
    const uint32_t *ws = a->ws;
    const uint32_t nbw = a->n_bm_words;
    DevCounters *cnt = a->cnt;
    const uint64_t w0 = (uint64_t)blockIdx.x * kScanWordsPerBlock + threadIdx.x * kWordsPerThread;
    uint32_t c = 0, r = 0;
    uint32_t prev = (w0 > 0 && w0 - 1 < nbw) ? ws[w0 - 1] >> 31 : 0u;
    for (uint32_t i = 0; i < kWordsPerThread; ++i) {
        const uint32_t x = (w0 + i < nbw) ? ws[w0 + i] : 0u;
        c += __popc(x);
        r += __popc(x & ~((x << 1) | prev));     // run starts: set bits whose predecessor is clear
        prev = x >> 31;
    }
    c = block_sum(c, sh);
    r = block_sum(r, sh);
    if (threadIdx.x == 0) {
        // the sums are device-coherent stores: once they have completed,
        // the last block's device-coherent loads (issued after it saw the
        // final ticket) return them
        st_agent(&a->blocksums[blockIdx.x], c);
        st_agent(&a->blockruns[blockIdx.x], r);
        hw_order();
        // finished blocks counted per group, then the groups (the last
        // block of a group counts it after its group's blocks counted)
        const uint32_t g = blockIdx.x % kSubTickets, ng = gridDim.x < kSubTickets ? gridDim.x : kSubTickets;
        const uint32_t in_g = (gridDim.x - g + kSubTickets - 1) / kSubTickets;
        bool last = false;
        if (__hip_atomic_fetch_add(&cnt->scan_sub[g], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == in_g - 1)
            last = __hip_atomic_fetch_add(&cnt->scan_ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == ng - 1;
        s_last = last;
    }
    __syncthreads();
    if (!s_last) return;
    // last block: exclusive scan of the block sums, in place
    const uint32_t nb = gridDim.x;
    const uint32_t per = (nb + kScanThreads - 1) / kScanThreads;
    const uint32_t lo = threadIdx.x * per, hi = min(lo + per, nb);
    uint32_t local = 0, runs = 0;
    for (uint32_t i = lo; i < hi; ++i) {
        local += ld_agent(&a->blocksums[i]);
        runs += ld_agent(&a->blockruns[i]);
    }
    uint32_t total = 0;
    uint32_t run = block_exclusive_scan(local, sh, total);
    runs = block_sum(runs, sh);
    for (uint32_t i = lo; i < hi; ++i) {
        uint32_t v = ld_agent(&a->blocksums[i]);
        st_agent(&a->blocksums[i], run);
        run += v;
    }
    if (threadIdx.x == 0) {
        st_agent(&cnt->n_dirty, total);
        st_agent(&cnt->n_runs, runs);
        st_agent(&cnt->scan_ticket, 0u);
        for (uint32_t g = 0; g < kSubTickets; ++g) st_agent(&cnt->scan_sub[g], 0u);
    }
}

// One block per kScanThreads bitmap words (one word per thread), in one
// round: the block adds up the popcounts of the words before its own within
// its counting block (at most kWordsPerThread - 1 coalesced loads per
// thread) to the counting block's offset, places its ids in LDS with a
// block scan and stores them with consecutive threads on consecutive ids.
// Dirty granules cluster (a hot range fills whole bitmap words); a thread
// storing its own ids one by one made 256 scattered stores in turn, and
// eight rounds per block left the kernel slow beside the apply pass.
__global__ __launch_bounds__(kScanThreads) void k_compact_emit(const DevArgs *__restrict__ a) {
    __shared__ uint32_t sh[kScanThreads / kWave];
    __shared__ uint32_t s_ids[kScanThreads * 32];
    const uint32_t *ws = a->ws;
    const uint32_t nbw = a->n_bm_words;
    uint32_t *ids = a->ids_scratch, *ids_out = a->ids_out;
    const uint32_t cb = blockIdx.x / kWordsPerThread, sub = blockIdx.x % kWordsPerThread;   // counting block, part
    const uint64_t cb0 = (uint64_t)cb * kScanWordsPerBlock;
    const uint64_t w = cb0 + (uint64_t)sub * kScanThreads + threadIdx.x;
    const uint32_t base = ld_agent(&a->blocksums[cb]);   // in flight with the bitmap loads
    const uint32_t x = w < nbw ? ws[w] : 0u;
    uint32_t before = 0;
    for (uint32_t k = 0; k < sub; ++k) {
        const uint64_t v = cb0 + (uint64_t)k * kScanThreads + threadIdx.x;
        before += v < nbw ? __popc(ws[v]) : 0u;
    }
    before = block_sum(before, sh);
    uint32_t v = x, total;
    uint32_t p = block_exclusive_scan(__popc(v), sh, total);
    while (v) {
        s_ids[p++] = (uint32_t)(w * 32 + __ffs(v) - 1);
        v &= v - 1;
    }
    __syncthreads();
    const uint32_t pos = base + before;
    for (uint32_t k = threadIdx.x; k < total; k += kScanThreads) {
        const uint32_t g = s_ids[k];
        ids[pos + k] = g;
        if (ids_out) ids_out[pos + k] = g;
    }
}

// --------------------------------------------------------------------- copy
// Unit u of a list of granules of upg units each: granule i, unit j within
// it (an exact multiply for the quotient rather than the compiled divide).
__device__ __forceinline__ void unit_of(uint64_t u, uint32_t upg, const Div32 &du, uint64_t &i, uint64_t &j) {
    i = u < (1ull << 32) ? div32((uint32_t)u, du) : u / upg;
    j = u - i * upg;
}

// Moves the dirty granules in units of U bytes (16 when granules are whole
// multiples of 16 bytes, else one word); upg = units per granule.  DS = 1:
// the replica is in the slot layout, unit (word) pos sits at u32 index 2 pos.
template <typename U, int DS>
__global__ __launch_bounds__(256) void k_copy(const DevArgs *__restrict__ a, uint32_t upg, Div32 du, uint64_t total_units) {
    DevCounters *cnt = a->cnt;
    if (ld_agent(&cnt->error)) return;
    const uint32_t conflict = a->outcome == HETM_OUTCOME_DEVICE ? ld_agent(&cnt->conflict) : a->outcome;
    const bool restore = conflict && a->policy != HETM_POLICY_GPU_WINS;   // else GPU -> host
    if (restore && a->undo_cap && !ld_agent(&cnt->undo_over)) return;   // k_undo rolled the round back
    const uint64_t D = ld_agent(&cnt->n_dirty);
    const uint32_t *ids = a->ids_scratch;
    U *dev = (U *)a->stmr;
    U *host = (U *)a->host;
    const uint64_t work = D * upg;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; u < work; u += stride) {
        uint64_t i, j;
        unit_of(u, upg, du, i, j);
        const uint64_t pos = (uint64_t)ids[i] * upg + j;
        if (pos >= total_units) continue;
        if (restore)
            dev[pos << DS] = host[pos];
        else
            host[pos] = dev[pos << DS];
    }
}

// ------------------------------------------------------- double-buffered merge
// gather: the round's dirty ids and count are staged always; on success the
// granules themselves are packed into the staging buffer (a conflict leaves
// the restore to the host side, after the previous copy has landed).
// Slot layout with granules of a multiple of 4 words: a lane moves 4 words,
// two 16-byte loads of two slots each and one 16-byte store of their values
// (qpg = granule / 4, a power of two: a granule's quads are qpg_shift bits).
__global__ __launch_bounds__(256) void k_gather_slots(const DevArgs *__restrict__ a, uint32_t qpg_shift,
                                                      uint64_t n_words) {
    DevCounters *cnt = a->cnt;
    if (ld_agent(&cnt->error)) return;
    const uint32_t outcome = ld_agent(&cnt->conflict);
    const uint64_t D = ld_agent(&cnt->n_dirty);
    const uint32_t *ids = a->ids_scratch;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t0 = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    for (uint64_t i = t0; i < D; i += stride) a->stage_ids[i] = ids[i];
    if (t0 == 0) *a->stage_count = (uint32_t)D;
    if (outcome && a->policy != HETM_POLICY_GPU_WINS) return;   // restored from the host instead
    const uint4 *slots = (const uint4 *)a->stmr;   // two slots per 16 bytes
    const uint32_t *words = (const uint32_t *)a->stmr;
    uint4 *stg = (uint4 *)a->staging;
    const uint64_t work = D << qpg_shift;
    const uint64_t qmask = (1ull << qpg_shift) - 1;
    for (uint64_t u = t0; u < work; u += stride) {
        const uint64_t q = ((uint64_t)ids[u >> qpg_shift] << qpg_shift) + (u & qmask);   // quad: words 4q .. 4q+3
        if (4 * q + 3 < n_words) {
            const uint4 s0 = slots[2 * q], s1 = slots[2 * q + 1];
            stg[u] = make_uint4(s0.x, s0.z, s1.x, s1.z);
        } else {
            uint32_t *st = (uint32_t *)(stg + u);
            for (uint32_t k = 0; k < 4; ++k)
                if (4 * q + k < n_words) st[k] = words[2 * (4 * q + k)];
        }
    }
}

template <typename U, int DS>
__global__ __launch_bounds__(256) void k_gather(const DevArgs *__restrict__ a, uint32_t upg, Div32 du, uint64_t total_units) {
    DevCounters *cnt = a->cnt;
    if (ld_agent(&cnt->error)) return;
    const uint32_t outcome = ld_agent(&cnt->conflict);
    const uint64_t D = ld_agent(&cnt->n_dirty);
    const uint32_t *ids = a->ids_scratch;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t0 = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    for (uint64_t i = t0; i < D; i += stride) a->stage_ids[i] = ids[i];
    if (t0 == 0) *a->stage_count = (uint32_t)D;
    if (outcome && a->policy != HETM_POLICY_GPU_WINS) return;   // restored from the host instead
    const U *dev = (const U *)a->stmr;
    U *stg = (U *)a->staging;
    const uint64_t work = D * upg;
    for (uint64_t u = t0; u < work; u += stride) {
        uint64_t i, j;
        unit_of(u, upg, du, i, j);
        const uint64_t pos = (uint64_t)ids[i] * upg + j;
        if (pos < total_units) stg[u] = dev[pos << DS];
    }
}

// Restore after a conflicting double-buffered round (CPU wins): the staged
// dirty granule ids are copied from the host replica back into the GPU
// replica.
template <typename U, int DS>
__global__ __launch_bounds__(256) void k_restore(U *stmr, const U *host, const uint32_t *ids, const uint32_t *count,
                                                 uint32_t upg, Div32 du, uint64_t total_units) {
    const uint64_t D = ld_agent(count);
    const uint64_t work = D * upg;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; u < work; u += stride) {
        uint64_t i, j;
        unit_of(u, upg, du, i, j);
        const uint64_t pos = (uint64_t)ld_agent(&ids[i]) * upg + j;
        if (pos < total_units) stmr[pos << DS] = host[pos];
    }
}

// Fast rollback (slot layout): a conflicting round (CPU wins; a discarded
// round merges as one) puts back the old value of every word the
// round's transactions wrote, from the undo log, except words the host log
// wrote afterwards (their version is at or above the round's first apply
// version), whose host value stands.  The GPU replica then equals the host
// replica (the pre-round state plus the host's writes) with no copy over the
// host link.  Runs only while the log holds every first write of the round.
__global__ __launch_bounds__(256) void k_undo(const DevArgs *__restrict__ a) {
    DevCounters *cnt = a->cnt;
    if (!a->undo_cap || ld_agent(&cnt->undo_over) || ld_agent(&cnt->error)) return;
    const uint32_t conflict = a->outcome == HETM_OUTCOME_DEVICE ? ld_agent(&cnt->conflict) : a->outcome;
    if (!conflict || a->policy == HETM_POLICY_GPU_WINS) return;
    const uint32_t n = min(ld_agent(&cnt->n_undo), a->undo_cap);
    const uint32_t floor = ld_agent(&cnt->apply_floor);
    uint64_t *slots = (uint64_t *)a->stmr;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint64_t rec = a->undo[i];
        const uint32_t w = (uint32_t)rec;
        const uint64_t cur = ld_agent(&slots[w]);
        const uint32_t ver = (uint32_t)(cur >> 32) & 0x7FFFFFFFu;
        if (ver >= floor) continue;
        st_agent(&slots[w], ((uint64_t)ver << 32) | (rec >> 32));
    }
}

// Slot layout: every version back to 0 and the clock with them (between
// rounds, when the clock has run far; no lock is held then).
__global__ __launch_bounds__(256) void k_version_reset(uint64_t *slots, uint64_t n, HotCounters *hot,
                                                       DevCounters *cnt) {
    for (uint64_t w = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; w < n; w += (uint64_t)gridDim.x * blockDim.x)
        slots[w] &= 0xFFFFFFFFull;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st_agent(&hot->clock.v, 0u);
        st_agent(&cnt->clock_base, 0u);
    }
}

// Slot layout <-> plain words (initial image in, state out).
__global__ __launch_bounds__(256) void k_to_slots(const uint32_t *src, uint64_t *slots, uint64_t n) {
    for (uint64_t w = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; w < n; w += (uint64_t)gridDim.x * blockDim.x)
        slots[w] = src[w];
}
__global__ __launch_bounds__(256) void k_from_slots(const uint64_t *slots, uint32_t *dst, uint64_t n) {
    for (uint64_t w = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; w < n; w += (uint64_t)gridDim.x * blockDim.x)
        dst[w] = (uint32_t)slots[w];
}

// ------------------------------------------------------------------- finish
__global__ __launch_bounds__(256) void k_finish(const DevArgs *__restrict__ a, DevCounters *snap) {
    DevCounters *cnt = a->cnt;
    const int32_t err = ld_agent(&cnt->error);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        DevCounters c;
        c.conflict = ld_agent(&cnt->conflict);
        c.error = err;
        c.ticket_snapshot = ld_agent(&a->hot->ticket.v);
        c.clock_base = ld_agent(&a->hot->clock.v);     // the next round begins here
        c.max_ts = ld_agent(&cnt->max_ts);
        c.floor_ts = ld_agent(&cnt->floor_ts);
        c.committed = ld_agent(&cnt->committed);
        c.retries = ld_agent(&cnt->retries);
        c.n_dirty = ld_agent(&cnt->n_dirty);
        c.n_runs = ld_agent(&cnt->n_runs);
        c.retry_txn = ld_agent(&cnt->retry_txn);
        c.scan_ticket = 0;
        c.err_index = ld_agent(&cnt->err_index);
        c.chunk_max_ts = 0;
        c.chunk_min_inv = 0;
        c.chunk_conflict = 0;
        c.log_ticket = 0;
        c.win_pending = 0;
        c.n_undo = ld_agent(&cnt->n_undo);
        c.undo_over = ld_agent(&cnt->undo_over);
        c.apply_floor = ld_agent(&cnt->apply_floor);
        c.apply_ver = 0;
        c.log_spill = 0;
        c.log_ndesc = 0;
        for (uint32_t g = 0; g < kSubTickets; ++g) c.log_sub[g] = c.scan_sub[g] = 0;
        c.doomed = ld_agent(&cnt->doomed);
        // a round queued behind this one may run only once the host has
        // handled an error, or restored the granules of a conflict the undo
        // log could not roll back
        c.hold = err != 0 || (c.conflict && a->policy == HETM_POLICY_CPU_WINS && (!a->undo_cap || c.undo_over));
        st_agent(&cnt->hold, c.hold);
        if (!err) {
            const uint64_t f = c.max_ts > c.floor_ts ? c.max_ts : c.floor_ts;
            c.floor_ts = f;
            st_agent(&cnt->floor_ts, (unsigned long long)f);
            st_agent(&cnt->conflict, 0u);
            st_agent(&a->hot->ticket.v, 0u);
            st_agent(&cnt->clock_base, c.clock_base);
            st_agent(&cnt->max_ts, 0ull);
            st_agent(&cnt->committed, 0ull);
            st_agent(&cnt->retries, 0ull);
            st_agent(&cnt->n_dirty, 0u);
            st_agent(&cnt->n_runs, 0u);
            st_agent(&cnt->win_pending, 0u);    // the next round's first chunk needs no timestamps
            st_agent(&cnt->n_undo, 0u);
            st_agent(&cnt->undo_over, 0u);
            st_agent(&cnt->apply_floor, 0xFFFFFFFFu);
        }
        *snap = c;
    }
    if (err) return;      // keep the round open: the caller can fix the log and merge again
    const uint32_t nbw = a->n_bm_words, nrw = a->n_rs_words;
    uint32_t *rs = (uint32_t *)a->rs;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nrw; i += gridDim.x * blockDim.x) {
        rs[i] = 0u;
        if (i < nbw) a->ws[i] = 0u;
    }
}

// The arguments of the work that follows on the stream; also the start of a
// batch: its work-queue cursors and list lengths go back to zero (every
// batch's kernels follow an argument upload, and no kernel of the previous
// batch is still running on the stream).  A round queued behind one the host
// has not collected yet runs empty (no transactions, no log) if that round
// holds; the host then handles the held round and launches this one again,
// ungated.  An ungated upload means the host has seen every earlier round.
__global__ void k_set_args(DevArgs v, DevArgs *dst) {
    if (threadIdx.x == 0) {
        if (!v.gated) {
            st_agent(&v.cnt->hold, 0u);
        } else if (ld_agent(&v.cnt->hold)) {
            v.n_txns = 0;
            v.n_log = 0;
        }
        *dst = v;
        if (v.hot) {
            st_agent(&v.hot->queue_head.v, 0u);
            st_agent(&v.hot->queue_upd.v, 0u);
            st_agent(&v.hot->n_ro.v, 0u);
            st_agent(&v.hot->n_upd.v, 0u);
        }
    }
}

__global__ void k_clear_error(DevCounters *cnt) {
    if (threadIdx.x == 0) {
        st_agent(&cnt->error, 0);
        st_agent(&cnt->err_index, 0u);
        st_agent(&cnt->retry_txn, 0u);
        st_agent(&cnt->chunk_conflict, 0u);
        st_agent(&cnt->chunk_max_ts, 0ull);
        st_agent(&cnt->chunk_min_inv, 0ull);
        st_agent(&cnt->log_ticket, 0u);
        st_agent(&cnt->log_spill, 0u);
        st_agent(&cnt->log_ndesc, 0u);
        for (uint32_t g = 0; g < kSubTickets; ++g) st_agent(&cnt->log_sub[g], 0u);
    }
}

uint32_t stream_grid(uint64_t items, uint32_t threads, uint32_t cap) {
    uint64_t b = (items + threads - 1) / threads;
    if (b < 1) b = 1;
    return (uint32_t)(b < cap ? b : cap);
}

}  // namespace

void launch_set_args(const DevArgs &host_copy, DevArgs *dev, hipStream_t s) {
    hipLaunchKernelGGL(k_set_args, dim3(1), dim3(64), 0, s, host_copy, dev);
}

const void *set_args_kernel() { return reinterpret_cast<const void *>(&k_set_args); }

void launch_clear_error(DevCounters *cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_error, dim3(1), dim3(64), 0, s, cnt);
}

void launch_compact(const DevArgs *a, uint32_t n_scan_blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_compact_count, dim3(n_scan_blocks), dim3(kScanThreads), 0, s, a);
    hipLaunchKernelGGL(k_compact_emit, dim3(n_scan_blocks * kWordsPerThread), dim3(kScanThreads), 0, s, a);
}

void launch_copy(const DevArgs *a, uint64_t n_words, uint32_t granule, uint32_t word_bytes, bool slot, hipStream_t s) {
    const uint64_t gbytes = (uint64_t)granule * word_bytes;
    const uint64_t n_granules = (n_words + granule - 1) / granule;
    const uint32_t wgrid = stream_grid(n_granules * granule, 256, 16384);
    if (slot) {
        hipLaunchKernelGGL((k_copy<uint32_t, 1>), dim3(wgrid), dim3(256), 0, s, a, granule, make_div32(granule), n_words);
    } else if (gbytes % 16 == 0 && (n_words * word_bytes) % 16 == 0) {
        const uint32_t upg = (uint32_t)(gbytes / 16);
        const uint32_t grid = stream_grid(n_granules * upg, 256, 16384);
        hipLaunchKernelGGL((k_copy<uint4, 0>), dim3(grid), dim3(256), 0, s, a, upg, make_div32(upg),
                           n_words * word_bytes / 16);
    } else if (word_bytes == 4) {
        hipLaunchKernelGGL((k_copy<uint32_t, 0>), dim3(wgrid), dim3(256), 0, s, a, granule, make_div32(granule), n_words);
    } else {
        hipLaunchKernelGGL((k_copy<uint64_t, 0>), dim3(wgrid), dim3(256), 0, s, a, granule, make_div32(granule), n_words);
    }
}

void launch_early_validate(const void *log, uint64_t n, uint32_t word_bytes, const uint8_t *rs, Div32 gdiv,
                           uint64_t n_words, uint32_t epoch, DevCounters *cnt, hipStream_t s) {
    const uint32_t grid = stream_grid(n, 256, 4096);
    if (word_bytes == 4)
        hipLaunchKernelGGL(k_early_validate<Entry4>, dim3(grid), dim3(256), 0, s, (const Entry4 *)log, n, rs, gdiv,
                           n_words, epoch, cnt);
    else
        hipLaunchKernelGGL(k_early_validate<Entry8>, dim3(grid), dim3(256), 0, s, (const Entry8 *)log, n, rs, gdiv,
                           n_words, epoch, cnt);
}

// The gather runs beside validation and apply in the batched round (and
// has the time they take): at most 4 workgroups per CU, so that it leaves
// them most of the GPU (16384 made the round about 1% longer).
constexpr uint32_t kGatherGrid = 1024;

void launch_gather(const DevArgs *a, uint64_t n_words, uint32_t granule, uint32_t word_bytes, bool slot,
                   hipStream_t s) {
    const uint64_t gbytes = (uint64_t)granule * word_bytes;
    const uint64_t n_granules = (n_words + granule - 1) / granule;
    const uint32_t wgrid = stream_grid(n_granules * granule, 256, kGatherGrid);
    if (slot && granule % 4 == 0 && ((granule / 4) & (granule / 4 - 1)) == 0) {
        const uint32_t qpg = granule / 4;
        hipLaunchKernelGGL(k_gather_slots, dim3(stream_grid(n_granules * qpg, 256, kGatherGrid)), dim3(256), 0, s, a,
                           (uint32_t)__builtin_ctz(qpg), n_words);
    } else if (slot) {
        hipLaunchKernelGGL((k_gather<uint32_t, 1>), dim3(wgrid), dim3(256), 0, s, a, granule, make_div32(granule),
                           n_words);
    } else if (gbytes % 16 == 0 && (n_words * word_bytes) % 16 == 0) {
        const uint32_t upg = (uint32_t)(gbytes / 16);
        hipLaunchKernelGGL((k_gather<uint4, 0>), dim3(stream_grid(n_granules * upg, 256, kGatherGrid)), dim3(256), 0, s, a,
                           upg, make_div32(upg), n_words * word_bytes / 16);
    } else if (word_bytes == 4) {
        hipLaunchKernelGGL((k_gather<uint32_t, 0>), dim3(wgrid), dim3(256), 0, s, a, granule, make_div32(granule),
                           n_words);
    } else {
        hipLaunchKernelGGL((k_gather<uint64_t, 0>), dim3(wgrid), dim3(256), 0, s, a, granule, make_div32(granule),
                           n_words);
    }
}

void launch_restore(void *stmr, const void *host, const uint32_t *ids, const uint32_t *count, uint64_t n_words,
                    uint32_t granule, uint32_t word_bytes, bool slot, hipStream_t s) {
    const uint32_t grid = 4096;
    const uint64_t gbytes = (uint64_t)granule * word_bytes;
    if (slot)
        hipLaunchKernelGGL((k_restore<uint32_t, 1>), dim3(grid), dim3(256), 0, s, (uint32_t *)stmr,
                           (const uint32_t *)host, ids, count, granule, make_div32(granule), n_words);
    else if (gbytes % 16 == 0 && (n_words * word_bytes) % 16 == 0)
        hipLaunchKernelGGL((k_restore<uint4, 0>), dim3(grid), dim3(256), 0, s, (uint4 *)stmr, (const uint4 *)host, ids,
                           count, (uint32_t)(gbytes / 16), make_div32((uint32_t)(gbytes / 16)), n_words * word_bytes / 16);
    else if (word_bytes == 4)
        hipLaunchKernelGGL((k_restore<uint32_t, 0>), dim3(grid), dim3(256), 0, s, (uint32_t *)stmr,
                           (const uint32_t *)host, ids, count, granule, make_div32(granule), n_words);
    else
        hipLaunchKernelGGL((k_restore<uint64_t, 0>), dim3(grid), dim3(256), 0, s, (uint64_t *)stmr,
                           (const uint64_t *)host, ids, count, granule, make_div32(granule), n_words);
}

void launch_undo(const DevArgs *a, uint32_t undo_cap, hipStream_t s) {
    if (!undo_cap) return;
    hipLaunchKernelGGL(k_undo, dim3(stream_grid(undo_cap, 256, 2048)), dim3(256), 0, s, a);
}

void launch_version_reset(uint64_t *slots, uint64_t n, HotCounters *hot, DevCounters *cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_version_reset, dim3(stream_grid(n, 256, 16384)), dim3(256), 0, s, slots, n, hot, cnt);
}

void launch_to_slots(const uint32_t *src, uint64_t *slots, uint64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_to_slots, dim3(stream_grid(n, 256, 16384)), dim3(256), 0, s, src, slots, n);
}
void launch_from_slots(const uint64_t *slots, uint32_t *dst, uint64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_from_slots, dim3(stream_grid(n, 256, 16384)), dim3(256), 0, s, slots, dst, n);
}

void launch_finish(const DevArgs *a, DevCounters *snap, uint32_t n_rs_words, hipStream_t s) {
    hipLaunchKernelGGL(k_finish, dim3(stream_grid(n_rs_words, 256, 4096)), dim3(256), 0, s, a, snap);
}

}  // namespace hetm
