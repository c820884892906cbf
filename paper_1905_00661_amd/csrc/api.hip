// api.hip -- the libhetm C ABI: context lifecycle and the orchestration of a
// SHeTM round (§IV-C) on one GPU, in two forms:
//   PLAIN -- one launch per round step; the host (the paper's GPU-controller
//            thread, §IV-A) reads the validation outcome before the merge;
//   GRAPH -- the whole round (argument upload, execution, validation + apply,
//            compaction, merge copy, reset, result download) is captured once
//            as a hipGraph and replayed; the merge reads the outcome on the
//            device, so a round costs one graph launch and one wait.
// Kernels take their arguments from a device-resident DevArgs block, so one
// captured graph serves rounds whose buffers differ.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "hetm.h"
#include "hetm_ctx.h"
#include "hetm_dev.h"

using namespace hetm;

// The device memory of hetm_read_words_noalloc: one copy per GPU, part of
// this file's code object, loaded with it and held until the process ends.
// Host code never passes the array's name to a kernel or a copy (on the host
// it is only a stand-in for the symbol): hetm_alloc_stmr looks up each
// device's copy once with hipGetSymbolAddress, with that device current.
constexpr uint64_t kNoAllocWords = 1ull << 24;   // 64 MiB of u32 values
static __device__ __align__(256) uint32_t scratch[kNoAllocWords];


namespace {

int fail(hetm_ctx *c, int code, const char *fmt, ...) {
    if (c) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(c->err, sizeof c->err, fmt, ap);
        va_end(ap);
    }
    return code;
}

#define HIP_TRY(c, call)                                                                       \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) return fail((c), HETM_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

template <typename T>
int dev_alloc(hetm_ctx *c, T **p, uint64_t bytes) {
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMalloc((void **)p, bytes);
    if (e != hipSuccess) return fail(c, HETM_ENOMEM, "hipMalloc(%llu) failed: %s", (unsigned long long)bytes,
                                     hipGetErrorString(e));
    c->device_bytes += bytes;
    return HETM_OK;
}

bool is_pow2(uint64_t x) { return x && !(x & (x - 1)); }

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;                           // guards g_scratch_ptr
void *g_scratch_ptr[kScratchDevices] = {};         // each device's copy of `scratch`
std::mutex g_scratch_use[kScratchDevices];         // calls on one GPU take turns on its copy

// With `device` current: its copy of `scratch`, looked up on the first call
// for that device.  A device beyond the table gets none (nullptr, HETM_OK):
// only hetm_read_words_noalloc needs it, and it reports the lack.
int scratch_for_device(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= kScratchDevices) return HETM_OK;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HETM_EDEVICE;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return HETM_OK;
}

// Write one byte of every 4 KiB page of a fresh pinned buffer, so that the
// host's first accesses to it (the merge worker's scatter) do not fault page
// by page inside the first rounds.
void touch_pages(void *p, uint64_t bytes) {
    volatile uint8_t *q = (volatile uint8_t *)p;
    for (uint64_t i = 0; i < bytes; i += 4096) q[i] = 0;
}

// Default transaction-kernel grid: one workgroup (4 waves) per compute unit.
// Measured on the large synthetic round (slot layout, waves of one kind):
// 586 us at 1/CU, 647 at 1.5, 714 at 2, 913 at 3 and 655 at 0.75 -- more
// concurrent transactions abort more and queue longer on the same memory
// path, fewer leave it idle.  The autotuner picks per workload.
uint32_t default_exec_workgroups(int cus) { return (uint32_t)cus; }

uint32_t ilog2(uint64_t x) {
    uint32_t r = 0;
    while ((1ull << r) < x) ++r;
    return r;
}

// Device-visible address of a host-or-device pointer: device and pinned
// memory are used in place; anything else gets nullptr.
const void *device_view(const void *p) {
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged) return p;
    if (at.type == hipMemoryTypeHost) return at.devicePointer ? at.devicePointer : p;
    return nullptr;
}

bool is_device_memory(const void *p) {
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeDevice;
}

int push_args(hetm_ctx *c) {
    c->args.epoch = c->epoch;
    launch_set_args(c->args, c->dargs, c->stream);
    HIP_TRY(c, hipGetLastError());
    return HETM_OK;
}

int read_counters(hetm_ctx *c, DevCounters *out) {
    HIP_TRY(c, hipMemcpyAsync(c->cnt_host, c->cnt, sizeof(DevCounters), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    *out = *c->cnt_host;
    return HETM_OK;
}

// Calls that queue work of their own, or read the state, wait until the
// rounds queued by hetm_round_submit have been collected.
int refuse_queued(hetm_ctx *c) {
    return c->q_n ? fail(c, HETM_ESTATE, "%u queued rounds not collected", c->q_n) : HETM_OK;
}

// Returns a latched device error (and clears it so the context stays usable).
int take_device_error(hetm_ctx *c, int32_t code, uint32_t where) {
    if (code == HETM_OK) return HETM_OK;
    launch_clear_error(c->cnt, c->stream);
    (void)hipStreamSynchronize(c->stream);
    return fail(c, code, "device reported %s at index %u", hetm_strerror(code), where);
}

int set_batch_args(hetm_ctx *c, uint32_t program, const void *descs, uint64_t n, void *results, uint32_t *tickets) {
    if (!descs || !results || !tickets) return fail(c, HETM_EINVAL, "null batch argument");
    if (n > c->cfg.batch_capacity) return fail(c, HETM_ECAPACITY, "batch of %llu > capacity", (unsigned long long)n);
    DevArgs &a = c->args;
    a.program = program;
    a.n_txns = (uint32_t)n;
    a.results = results;
    a.tickets = tickets;
    if (program == HETM_PROG_OPLIST) {
        if (c->cfg.word_bytes != 4) return fail(c, HETM_EINVAL, "OPLIST needs 4-byte words");
        const hetm_oplist_desc *d = (const hetm_oplist_desc *)descs;
        if (!d->offsets || !d->idx || !d->n_writes || !d->tid) return fail(c, HETM_EINVAL, "null OPLIST array");
        a.off = d->offsets, a.idx = d->idx, a.nw = d->n_writes, a.tid = d->tid;
    } else if (program == HETM_PROG_TRANSFER) {
        if (c->cfg.word_bytes != 8) return fail(c, HETM_EINVAL, "TRANSFER needs 8-byte words");
        const hetm_transfer_desc *d = (const hetm_transfer_desc *)descs;
        if (!d->src || !d->dst || !d->amt) return fail(c, HETM_EINVAL, "null TRANSFER array");
        a.src = d->src, a.dst = d->dst, a.amt = d->amt;
    } else if (program == HETM_PROG_CACHE) {
        if (c->cfg.word_bytes != 4) return fail(c, HETM_EINVAL, "CACHE needs 4-byte words");
        uint64_t nsets = c->cfg.n_words / 128;
        if (c->cfg.n_words % 128 || nsets < 2 || !is_pow2(nsets))
            return fail(c, HETM_EINVAL, "CACHE needs N = 128 * 2^k words");
        const hetm_cache_desc *d = (const hetm_cache_desc *)descs;
        if (!d->key || !d->op || !d->tid) return fail(c, HETM_EINVAL, "null CACHE array");
        a.key = d->key, a.op = d->op, a.tid = d->tid;
    } else {
        return fail(c, HETM_EINVAL, "unknown program %u", program);
    }
    return HETM_OK;
}

// Places a log chunk where the kernels can read it: device and pinned
// memory in place, pageable host memory through the staging buffer.
int stage_log(hetm_ctx *c, const void *log, uint64_t n, const void **dev_log) {
    const void *v = device_view(log);
    if (v) {
        *dev_log = v;
        return HETM_OK;
    }
    HIP_TRY(c, hipMemcpyAsync(c->log_staging, log, n * c->log_entry_bytes, hipMemcpyHostToDevice, c->stream));
    *dev_log = c->log_staging;
    return HETM_OK;
}

int enqueue_validate(hetm_ctx *c, const void *dev_log, uint64_t n, uint32_t *flags) {
    c->args.log = dev_log;
    c->args.n_log = (uint32_t)n;
    c->args.flags = flags;
    int rc = push_args(c);
    if (rc) return rc;
    launch_validate(c->dargs, c->cfg.word_bytes, c->log_bins, c->log_tiles, c->chunks_in_round > 0, c->cnt,
                    c->stream);
    launch_apply(c->dargs, c->cfg.word_bytes, c->log_bins, c->stream);
    ++c->chunks_in_round;
    HIP_TRY(c, hipGetLastError());
    return HETM_OK;
}

int enqueue_merge(hetm_ctx *c, uint32_t outcome, const void *host_dev, uint32_t *ids_out) {
    // the round closes after its early validations (they read the caller's log chunks)
    if (c->early_used) HIP_TRY(c, hipStreamWaitEvent(c->stream, c->early_ev, 0));
    c->early_used = false;
    c->args.outcome = outcome;
    c->args.host = const_cast<void *>(host_dev);
    c->args.ids_out = ids_out;
    int rc = push_args(c);
    if (rc) return rc;
    launch_undo(c->dargs, c->undo_cap, c->stream);
    launch_compact(c->dargs, c->args.n_scan_blocks, c->stream);
    launch_copy(c->dargs, c->cfg.n_words, c->cfg.granule_words, c->cfg.word_bytes, c->slot, c->stream);
    launch_finish(c->dargs, c->snap_map, c->args.n_rs_words, c->stream);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipEventRecord(c->closed_ev, c->stream));
    c->closed_recorded = true;
    c->chunks_in_round = 0;
    ++c->epoch;
    return HETM_OK;
}

// A whole round that latched a device error is discarded as a conflicting
// round is under CPU wins: the latch is cleared, the GPU's dirty granules
// are restored from the host replica, the bitmaps and counters are reset.
// The round's log chunk was not applied (the apply pass skips on an error).
int discard_round(hetm_ctx *c, int32_t code, uint32_t where, const void *hdev, bool undo_ok) {
    launch_clear_error(c->cnt, c->stream);
    // the merge of a conflicting round rolls it back: from the undo log if
    // it holds the round, else from the host replica
    if (undo_ok)
        c->stats.rollbacks_device++;
    else
        c->stats.rollbacks_host++;
    const uint32_t policy = c->args.policy;
    c->args.policy = HETM_POLICY_CPU_WINS;   // the copy restores the device side
    int rc = enqueue_merge(c, 1u, hdev, nullptr);
    c->args.policy = policy;
    if (rc) return rc;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return fail(c, code, "device reported %s at index %u; the round was discarded", hetm_strerror(code), where);
}

// Slot layout: once the version clock has run past kClockReset, every
// version and the clock go back to 0 before the next round (queued on the
// context's stream, which the next round's work follows).
void maybe_reset_versions(hetm_ctx *c, uint32_t clock) {
    if (!c->slot || clock < kClockReset) return;
    launch_version_reset((uint64_t *)c->stmr, c->cfg.n_words, c->hot, c->cnt, c->stream);
    c->stats.version_resets++;
}

// policy: the round's (a queued round's can differ from the arguments last
// uploaded, which belong to the round behind it).
void account_round(hetm_ctx *c, const DevCounters &s, uint64_t n_txns, uint32_t policy, hetm_round_result *res,
                   bool may_reset = true) {
    if (!s.error && may_reset) maybe_reset_versions(c, s.clock_base);
    const bool gpu_won = s.conflict && policy == HETM_POLICY_GPU_WINS;
    const bool gpu_lost = s.conflict && !gpu_won;
    c->stats.rounds++;
    if (s.conflict) c->stats.rounds_conflicted++;
    if (gpu_lost)
        c->stats.txns_aborted += s.committed;
    else
        c->stats.txns_committed += s.committed;
    c->gpu_losses = gpu_lost ? c->gpu_losses + 1 : 0;
    if (gpu_lost) {
        if (c->undo_cap && !s.undo_over)
            c->stats.rollbacks_device++;
        else
            c->stats.rollbacks_host++;
    }
    c->stats.local_retries += s.retries;
    c->stats.dirty_granules += s.n_dirty;
    c->stats.watermark = s.floor_ts;
    if (res) {
        res->conflict = s.conflict;
        res->error = s.error;
        res->n_committed = gpu_lost ? 0 : s.committed;
        res->n_aborted = gpu_lost ? n_txns : 0;
        res->host_discarded = gpu_won;
        res->gpu_losses = c->gpu_losses;
        res->n_local_retries = s.retries;
        res->n_dirty = s.n_dirty;
        res->n_runs = s.n_runs;
        res->max_ts = s.floor_ts;
        res->doomed = s.doomed == c->epoch - 1;     // the round just closed
    }
}

int check_host_replica(hetm_ctx *c, void *host, const void **dev) {
    if (!host) return fail(c, HETM_EINVAL, "null host replica");
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, host) != hipSuccess || at.type != hipMemoryTypeHost) {
        (void)hipGetLastError();
        return fail(c, HETM_EINVAL, "host replica must be pinned host memory (hipHostMalloc)");
    }
    *dev = at.devicePointer ? at.devicePointer : host;
    return HETM_OK;
}

int issue_merge(hetm_ctx *c, hipEvent_t after);

// Waits until every staged merge copy has reached the host replica.
int drain_merges(hetm_ctx *c) {
    int rc = issue_merge(c, nullptr);
    if (rc) return rc;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->copy_stream) HIP_TRY(c, hipStreamSynchronize(c->copy_stream));
    if (c->merger) {
        const uint64_t last = std::max(c->merge_seq[0], c->merge_seq[1]);
        if (last && hetm::merge_wait(c->merger, last) != HETM_OK)
            return fail(c, HETM_EDEVICE, "merge copy to the host replica failed");
    }
    c->pending[0] = c->pending[1] = false;
    return HETM_OK;
}

void drop_graph(hetm_ctx::RoundGraph &g) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g = hetm_ctx::RoundGraph{};
}

void drop_graphs(hetm_ctx *c) {
    for (auto &g : c->graphs) drop_graph(g);
    for (auto &p : c->sgraphs)
        for (auto &g : p) drop_graph(g);
    for (auto &p : c->qgraphs)
        for (auto &g : p) drop_graph(g);
}

// Captures the round for one merge policy on a private non-blocking stream
// (the default stream cannot be captured); it is launched on the caller's
// stream.  Under CPU wins with the double-buffered merge, compaction and the
// gather of the dirty granules fork off after the transaction kernel and
// join before the finish: they read only the GPU's write set, and a round
// without conflict applies the host log to granules the GPU neither read
// nor wrote (its written granules are in its read set).  In a conflicted
// round the gathered data is not used (the host restores those granules),
// and the staged ids it restores from do not depend on the log.  Under GPU
// wins a conflicted round's apply adds the log's granules to the write set,
// so compaction has to follow it.
// What a captured graph holds: the whole round, or the execution part or
// the tail (validation and apply, merge, finish) of a streamed round.
enum class Part { kWhole, kExec, kTail };

// snap: where the finish kernel stores the round's counter snapshot.
int capture_round(hetm_ctx *c, uint32_t policy, Part part, hetm_ctx::RoundGraph &rg, DevCounters *snap) {
    if (rg.exec) return HETM_OK;
    if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    const bool fork = c->cfg.async_merge && policy == HETM_POLICY_CPU_WINS;
    if (fork && !c->cap_branch) {
        HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_branch, hipStreamNonBlocking));
        HIP_TRY(c, hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
        HIP_TRY(c, hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming));
    }
    hipStream_t s = c->cap_stream;
    HIP_TRY(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    // The arguments enter the graph as the by-value parameters of a one-thread
    // kernel node, updated per round (hipGraphExecKernelNodeSetParams): the
    // host writes kernel parameters into device memory, whereas a host-to-
    // device copy node would issue PCIe reads that queue behind the previous
    // round's merge copy (device-to-host posted writes) and stall the launch.
    launch_set_args(c->args, c->dargs, s);
    hipError_t ce = hipSuccess;
    if (part != Part::kTail)
        launch_exec(c->args.program, c->dargs, c->exec_wg, c->cfg.max_txn_ops, c->slot, c->cfg.batch_capacity, s);
    if (part == Part::kExec) {
        // the execution part ends here
    } else if (fork) {
        hipStream_t br = c->cap_branch;
        if (ce == hipSuccess) ce = hipEventRecord(c->fork_ev, s);
        if (ce == hipSuccess) ce = hipStreamWaitEvent(br, c->fork_ev, 0);
        launch_compact(c->dargs, c->args.n_scan_blocks, br);
        launch_gather(c->dargs, c->cfg.n_words, c->cfg.granule_words, c->cfg.word_bytes, c->slot, br);
        if (ce == hipSuccess) ce = hipEventRecord(c->join_ev, br);
        launch_validate(c->dargs, c->cfg.word_bytes, c->log_bins, c->log_tiles, false, c->cnt, s);
        launch_apply(c->dargs, c->cfg.word_bytes, c->log_bins, s);
        launch_undo(c->dargs, c->undo_cap, s);     // a conflicting round rolls back on the device
        if (ce == hipSuccess) ce = hipStreamWaitEvent(s, c->join_ev, 0);
    } else {
        launch_validate(c->dargs, c->cfg.word_bytes, c->log_bins, c->log_tiles, false, c->cnt, s);
        launch_apply(c->dargs, c->cfg.word_bytes, c->log_bins, s);
        launch_undo(c->dargs, c->undo_cap, s);
        launch_compact(c->dargs, c->args.n_scan_blocks, s);
        if (c->cfg.async_merge)
            launch_gather(c->dargs, c->cfg.n_words, c->cfg.granule_words, c->cfg.word_bytes, c->slot, s);
        else
            launch_copy(c->dargs, c->cfg.n_words, c->cfg.granule_words, c->cfg.word_bytes, c->slot, s);
    }
    if (part != Part::kExec) {
        launch_finish(c->dargs, snap, c->args.n_rs_words, s);
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (e != hipSuccess || ce != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(c, HETM_EDEVICE, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : ce));
    }
    e = hipGraphInstantiate(&rg.exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        rg.exec = nullptr;
        return fail(c, HETM_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
    }
    rg.graph = g;
    rg.program = c->args.program;
    // find the argument-upload node
    size_t nn = 0;
    HIP_TRY(c, hipGraphGetNodes(g, nullptr, &nn));
    hipGraphNode_t nodes[64];
    if (nn > 64) return fail(c, HETM_EDEVICE, "unexpected graph size %zu", nn);
    HIP_TRY(c, hipGraphGetNodes(g, nodes, &nn));
    rg.args_node = nullptr;
    for (size_t i = 0; i < nn; ++i) {
        hipGraphNodeType t;
        if (hipGraphNodeGetType(nodes[i], &t) != hipSuccess || t != hipGraphNodeTypeKernel) continue;
        hipKernelNodeParams kp{};
        if (hipGraphKernelNodeGetParams(nodes[i], &kp) == hipSuccess && kp.func == set_args_kernel()) {
            rg.args_node = nodes[i];
            rg.args_params = kp;
        }
    }
    if (!rg.args_node) return fail(c, HETM_EDEVICE, "argument node not found in the round graph");
    return HETM_OK;
}

int build_graph(hetm_ctx *c, uint32_t policy) {
    return capture_round(c, policy, Part::kWhole, c->graphs[policy], c->snap_map);
}

// Uploads the current arguments into a graph's argument node and launches it.
int launch_round_graph(hetm_ctx *c, hetm_ctx::RoundGraph &rg, hipStream_t s) {
    c->args.epoch = c->epoch;
    DevArgs *dst = c->dargs;
    void *kargs[2] = {&c->args, &dst};
    hipKernelNodeParams kp = rg.args_params;
    kp.kernelParams = kargs;
    kp.extra = nullptr;
    HIP_TRY(c, hipGraphExecKernelNodeSetParams(rg.exec, rg.args_node, &kp));
    HIP_TRY(c, hipGraphLaunch(rg.exec, s));
    return HETM_OK;
}

float elapsed_us(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
        (void)hipGetLastError();
        return 0.f;
    }
    return ms * 1000.f;
}

// Success path of the double-buffered merge for staging buffer b holding D
// packed granules bound for host replica `host`: a copy on the copy stream
// into pinned host staging once the round's graph has ended (event `after`),
// then a job for the merge worker.
int stage_to_host(hetm_ctx *c, int b, uint64_t D, void *host, hipEvent_t after) {
    const uint64_t gbytes = (uint64_t)c->cfg.granule_words * c->cfg.word_bytes;
    // the job that last used this host staging buffer has been scattered out
    // of it (the other buffer's job may still be scattering: this copy
    // overlaps it)
    if (c->merge_seq[b] && hetm::merge_wait(c->merger, c->merge_seq[b]) != HETM_OK)
        return fail(c, HETM_EDEVICE, "merge copy to the host replica failed");
    if (D > c->host_cap[b]) return fail(c, HETM_ECAPACITY, "%llu dirty granules", (unsigned long long)D);
    HIP_TRY(c, hipStreamWaitEvent(c->copy_stream, after, 0));      // after the round's graph
    if (D) {
        HIP_TRY(c, hipMemcpyAsync(c->host_ids[b], c->stage_ids[b], D * 4, hipMemcpyDeviceToHost, c->copy_stream));
        HIP_TRY(c, hipMemcpyAsync(c->host_stage[b], c->staging[b], D * gbytes, hipMemcpyDeviceToHost, c->copy_stream));
    }
    HIP_TRY(c, hipEventRecord(c->copied[b], c->copy_stream));
    const uint64_t seq = hetm::merge_submit(c->merger, c->copied[b], c->host_ids[b], c->host_stage[b], D,
                                            (uint8_t *)host, gbytes, c->cfg.n_words * c->cfg.word_bytes);
    if (!seq) return fail(c, HETM_ENOMEM, "merge job could not be queued");
    c->merge_seq[b] = seq;
    c->round_merge_seq = seq;
    return HETM_OK;
}

// Issues the deferred copy of the last successful round, after `after`
// (nullable) on the device.
int issue_merge(hetm_ctx *c, hipEvent_t after) {
    if (!c->merge_deferred) return HETM_OK;
    c->merge_deferred = false;
    if (after) HIP_TRY(c, hipStreamWaitEvent(c->copy_stream, after, 0));
    return stage_to_host(c, c->deferred_buf, c->deferred_n, c->deferred_host, c->deferred_ev);
}

}  // namespace

namespace hetm {

// Checks a GRAPH round's arguments and sets them up, except the log (a
// whole round stages it, a streamed round takes it in pushed chunks).
int prepare_round(hetm_ctx *c, const hetm_round_args *r, const void **hdev) {
    if (c->cfg.mode != HETM_MODE_GRAPH) return fail(c, HETM_ESTATE, "round_begin needs GRAPH mode");
    if (c->in_validation || c->round_open) return fail(c, HETM_ESTATE, "a round is already open");
    if (r->policy > HETM_POLICY_GPU_WINS) return fail(c, HETM_EINVAL, "bad policy %u", r->policy);
    if (r->n_log > c->cfg.log_capacity) return fail(c, HETM_ECAPACITY, "log %llu > capacity", (unsigned long long)r->n_log);
    if (r->n_log && !r->log) return fail(c, HETM_EINVAL, "null log");
    int rc = check_host_replica(c, r->host_replica, hdev);
    if (rc) return rc;
    c->args.policy = r->policy;
    if (r->n_txns) {
        if ((rc = set_batch_args(c, r->program, r->descs, r->n_txns, r->results, r->tickets))) return rc;
    } else {
        c->args.n_txns = 0;
        if (!c->args.program) c->args.program = HETM_PROG_OPLIST;
    }
    c->args.log = nullptr;
    c->args.n_log = 0;
    c->args.flags = r->flags_bits;
    c->args.outcome = HETM_OUTCOME_DEVICE;
    c->args.host = const_cast<void *>(*hdev);
    c->args.ids_out = r->ids_out;
    c->round_host = r->host_replica;
    if (c->graphs[r->policy].exec && c->graphs[r->policy].program != c->args.program) drop_graphs(c);
    for (auto &p : c->sgraphs)
        if (p[0].exec && p[0].program != c->args.program) drop_graphs(c);
    for (auto &p : c->qgraphs)
        for (auto &g : p)
            if (g.exec && g.program != c->args.program) drop_graphs(c);
    return HETM_OK;
}

// Before a round's graph: the staging buffer it fills must have reached the
// host (double-buffered merge).
int wait_staging(hetm_ctx *c, hipStream_t s) {
    const int b = c->buf;
    if (c->cfg.async_merge) {
        if (c->pending[b]) HIP_TRY(c, hipStreamWaitEvent(s, c->copied[b], 0));
        c->args.staging = c->staging[b];
        c->args.stage_ids = c->stage_ids[b];
        c->args.stage_count = c->stage_count[b];
    }
    return HETM_OK;
}

int round_begin(hetm_ctx *c, const hetm_round_args *r) {
    const void *hdev = nullptr;
    int rc = prepare_round(c, r, &hdev);
    if (rc) return rc;
    const void *dlog = nullptr;
    if (r->n_log && (rc = stage_log(c, r->log, r->n_log, &dlog))) return rc;
    c->args.log = dlog;
    c->args.n_log = (uint32_t)r->n_log;
    if ((rc = build_graph(c, r->policy))) return rc;
    // the graph runs on the caller's stream, after the caller's earlier work
    // there (uploads, a staged log); it was captured on a private stream
    hipStream_t s = c->stream;
    if ((rc = wait_staging(c, s))) return rc;
    HIP_TRY(c, hipEventRecord(c->ev[0], s));
    if ((rc = launch_round_graph(c, c->graphs[r->policy], s))) return rc;
    // the last round's copy to the host is issued once this round's graph
    // is queued (its end event, ev[3], is re-recorded only below)
    if ((rc = issue_merge(c, nullptr))) return rc;
    HIP_TRY(c, hipEventRecord(c->ev[3], s));
    c->round_open = true;
    c->round_streamed = false;
    c->round_hdev = hdev;
    c->round_buf = c->buf;
    return HETM_OK;
}

int stream_push(hetm_ctx *c, const void *log, uint64_t n, uint32_t *doomed_out) {
    if (!c->round_open || !c->round_streamed) return fail(c, HETM_ESTATE, "no streamed round open");
    if (n && !log) return fail(c, HETM_EINVAL, "null log");
    if (n > c->cfg.log_capacity - c->round_pushed)
        return fail(c, HETM_ECAPACITY, "%llu + %llu log entries > capacity %llu", (unsigned long long)c->round_pushed,
                    (unsigned long long)n, (unsigned long long)c->cfg.log_capacity);
    if (n) {
        hipStream_t es = c->early_stream;
        const uint64_t eb = c->log_entry_bytes;
        // after the last round's tail (it read log_staging and cleared the
        // read set), beside this round's execution
        HIP_TRY(c, hipStreamWaitEvent(es, c->exec_queued, 0));
        const void *chunk;
        const bool follows = c->round_pushed == 0 || (c->round_in_place &&
                                                       log == (const uint8_t *)c->round_log + c->round_pushed * eb);
        if (follows && is_device_memory(log)) {
            // chunks in device memory that follow each other in one buffer
            // are read in place, by the early check and by the round's tail
            if (c->round_pushed == 0) {
                c->round_log = log;
                c->round_in_place = true;
            }
            chunk = log;
        } else {
            if (c->round_in_place && c->round_pushed)   // the chunks read in place so far join the buffer
                HIP_TRY(c, hipMemcpyAsync(c->log_staging, c->round_log, c->round_pushed * eb, hipMemcpyDeviceToDevice,
                                          es));
            c->round_in_place = false;
            c->round_log = c->log_staging;
            uint8_t *dst = (uint8_t *)c->log_staging + c->round_pushed * eb;
            HIP_TRY(c, hipMemcpyAsync(dst, log, n * eb, hipMemcpyDefault, es));
            chunk = dst;
        }
        if (c->args.policy == HETM_POLICY_CPU_WINS) {
            launch_early_validate(chunk, n, c->cfg.word_bytes, c->rs, c->args.gdiv, c->cfg.n_words, c->epoch, c->cnt,
                                  es);
            HIP_TRY(c, hipGetLastError());
        }
        HIP_TRY(c, hipEventRecord(c->early_ev, es));
        c->early_used = true;
        c->round_pushed += n;
    }
    if (doomed_out) {
        HIP_TRY(c, hipMemcpyAsync(c->early_host, &c->cnt->doomed, sizeof(uint32_t), hipMemcpyDeviceToHost,
                                  c->early_stream));
        HIP_TRY(c, hipStreamSynchronize(c->early_stream));
        *doomed_out = *c->early_host == c->epoch;
    }
    return HETM_OK;
}

int stream_begin(hetm_ctx *c, const hetm_round_args *r) {
    const void *hdev = nullptr;
    int rc = prepare_round(c, r, &hdev);
    if (rc) return rc;
    hetm_ctx::RoundGraph *g = c->sgraphs[r->policy];
    if ((rc = capture_round(c, r->policy, Part::kExec, g[0], c->snap_map))) return rc;
    if ((rc = capture_round(c, r->policy, Part::kTail, g[1], c->snap_map))) return rc;
    g[1].program = g[0].program;
    hipStream_t s = c->stream;
    if ((rc = wait_staging(c, s))) return rc;
    HIP_TRY(c, hipEventRecord(c->ev[0], s));
    HIP_TRY(c, hipEventRecord(c->exec_queued, s));
    if ((rc = launch_round_graph(c, g[0], s))) return rc;
    if ((rc = issue_merge(c, nullptr))) return rc;
    c->round_open = true;
    c->round_streamed = true;
    c->round_pushed = 0;
    c->round_log = nullptr;
    c->round_in_place = false;
    c->round_args = *r;
    c->round_hdev = hdev;
    c->round_buf = c->buf;
    if (r->n_log && (rc = stream_push(c, r->log, r->n_log, nullptr))) return rc;
    return HETM_OK;
}

// A further batch of the open streamed round, launched eagerly (not as a
// replay of the execution graph, whose argument node the previous replay may
// still be about to read): its argument upload and execution kernels queue
// behind the round's earlier batches on the context's stream, so they read
// the round's read set, clock and ticket counter where the earlier batches
// left them.  The tail validates and merges all batches as one round.
int stream_add(hetm_ctx *c, uint32_t program, const void *descs, uint64_t n, void *results, uint32_t *tickets) {
    if (!c->round_open || !c->round_streamed) return fail(c, HETM_ESTATE, "no streamed round open");
    if (c->round_args.n_txns && program != c->args.program)
        return fail(c, HETM_EINVAL, "batch of program %u in a round of program %u", program, c->args.program);
    if (n == 0) return HETM_OK;
    const DevArgs keep = c->args;
    int rc = set_batch_args(c, program, descs, n, results, tickets);
    if (rc) {
        c->args = keep;      // the round goes on as it was
        return rc;
    }
    if ((rc = push_args(c))) return rc;
    launch_exec(program, c->dargs, c->exec_wg, c->cfg.max_txn_ops, c->slot, c->cfg.batch_capacity, c->stream);
    HIP_TRY(c, hipGetLastError());
    c->round_args.n_txns += n;
    return HETM_OK;
}

int stream_end(hetm_ctx *c, hetm_round_result *res) {
    if (!c->round_open || !c->round_streamed) return fail(c, HETM_ESTATE, "no streamed round open");
    hipStream_t s = c->stream;
    // every pushed chunk is copied (and early-validated) before the tail
    if (c->early_used) HIP_TRY(c, hipStreamWaitEvent(s, c->early_ev, 0));
    c->early_used = false;
    c->args.log = c->round_pushed ? c->round_log : nullptr;
    c->args.n_log = (uint32_t)c->round_pushed;
    int rc = launch_round_graph(c, c->sgraphs[c->args.policy][1], s);
    if (rc) return rc;
    HIP_TRY(c, hipEventRecord(c->ev[3], s));
    hetm_round_args r = c->round_args;
    r.n_log = c->round_pushed;
    c->round_streamed = false;
    return round_end(c, &r, res);
}

int round_end(hetm_ctx *c, const hetm_round_args *r, hetm_round_result *res) {
    if (!c->round_open) return fail(c, HETM_ESTATE, "no round open");
    c->round_open = false;
    ++c->epoch;
    hipStream_t s = c->stream;
    const void *hdev = c->round_hdev;
    const int b = c->round_buf;
    int rc;
    HIP_TRY(c, hipStreamSynchronize(s));
    const DevCounters snap = *c->snap_host;
    c->round_merge_seq = 0;
    const bool undo_ok = c->undo_cap && !snap.undo_over;   // the round's undo log is whole
    if (snap.error) {
        // a restore from the host replica reads it: earlier merges land first
        if (c->cfg.async_merge && !undo_ok && (rc = drain_merges(c))) return rc;
        return discard_round(c, snap.error, snap.err_index, hdev, undo_ok);
    }
    if (c->cfg.async_merge) {
        if (!snap.conflict || c->args.policy == HETM_POLICY_GPU_WINS) {
            // the GPU's granules go to the host replica: a copy of the staged granules to pinned host staging on
            // the copy stream (issued by the next round_begin, or by whatever waits for merges first), then
            // the merge worker scatters them into the host replica.  The merge of the round before the last
            // (the last job on this round's buffer) lands before this round returns.
            if (c->merge_seq[b] && hetm::merge_wait(c->merger, c->merge_seq[b]) != HETM_OK)
                return fail(c, HETM_EDEVICE, "merge copy to the host replica failed");
            c->merge_deferred = true;
            c->deferred_ev = c->ev[3];     // re-recorded only after the next round_begin has issued the copy
            c->deferred_buf = b;
            c->deferred_n = snap.n_dirty;
            c->deferred_host = c->round_host;
            c->pending[b] = true;
            c->last_copy = b;
            c->buf = b ^ 1;
            if (res) res->merge_pending = 1;
        } else if (!undo_ok) {
            // conflict (CPU wins) without a whole undo log: restore the dirty
            // granules from the host replica once the previous round's copy
            // has landed there (with one, the round graph rolled it back)
            if ((rc = drain_merges(c))) return rc;
            launch_restore(c->stmr, hdev, c->stage_ids[b], c->stage_count[b], c->cfg.n_words, c->cfg.granule_words,
                           c->cfg.word_bytes, c->slot, s);
            HIP_TRY(c, hipGetLastError());
            HIP_TRY(c, hipStreamSynchronize(s));
        }
    }
    account_round(c, snap, r->n_txns, c->args.policy, res);
    if (res) res->us_total = elapsed_us(c->ev[0], c->ev[3]);
    c->stats.log_entries += r->n_log;
    return HETM_OK;
}

// Launches queued round q (its arguments checked and set up again) in its
// slot's graph; gated: behind a round the host has not collected.
int launch_queued(hetm_ctx *c, hetm_ctx::Queued &q, bool gated) {
    const void *hdev = nullptr;
    int rc = prepare_round(c, &q.r, &hdev);
    if (rc) return rc;
    const void *dlog = nullptr;
    if (q.r.n_log && (rc = stage_log(c, q.r.log, q.r.n_log, &dlog))) return rc;
    c->args.log = dlog;
    c->args.n_log = (uint32_t)q.r.n_log;
    hetm_ctx::RoundGraph &g = c->qgraphs[q.r.policy][q.slot];
    if ((rc = capture_round(c, q.r.policy, Part::kWhole, g, c->snap_map + q.slot))) return rc;
    // the slot's staging buffer: the copy of the round that last filled it
    // was issued when that round was collected
    hipStream_t s = c->stream;
    const int b = q.slot;
    if (c->pending[b]) HIP_TRY(c, hipStreamWaitEvent(s, c->copied[b], 0));
    c->args.staging = c->staging[b];
    c->args.stage_ids = c->stage_ids[b];
    c->args.stage_count = c->stage_count[b];
    c->args.gated = gated;
    HIP_TRY(c, hipEventRecord(c->q_begin[b], s));
    rc = launch_round_graph(c, g, s);
    c->args.gated = 0;
    if (rc) return rc;
    HIP_TRY(c, hipEventRecord(c->q_end[b], s));
    q.hdev = hdev;
    return HETM_OK;
}

int round_submit(hetm_ctx *c, const hetm_round_args *r) {
    if (c->cfg.mode != HETM_MODE_GRAPH || !c->cfg.async_merge)
        return fail(c, HETM_ESTATE, "round_submit needs GRAPH mode with the double-buffered merge");
    if (c->q_n == 2) return fail(c, HETM_ESTATE, "two rounds are queued: collect one first");
    if (c->in_validation || c->round_open) return fail(c, HETM_ESTATE, "a round is already open");
    if (c->q_n) {
        // the queued rounds' graphs stay as they are
        const uint32_t prog = r->n_txns ? r->program : c->args.program;
        if (prog != c->args.program)
            return fail(c, HETM_ESTATE, "program %u behind a queued round of program %u", prog, c->args.program);
    } else {
        // a staged copy of an earlier round goes out before a slot's buffer
        // is reused (its copied event is recorded as it is issued)
        int rc = issue_merge(c, nullptr);
        if (rc) return rc;
    }
    hetm_ctx::Queued &q = c->queued[(c->q_head + c->q_n) & 1];
    q = hetm_ctx::Queued{};
    q.r = *r;
    q.seq = c->q_seq;
    q.slot = (int)(c->q_seq & 1);
    // gated behind a round whose outcome is still to come (a cancelled one
    // will not run, and the discard before it left a hold this upload lowers)
    const bool gated = c->q_n > 0 && !c->queued[c->q_head].cancelled;
    const DevArgs keep = c->args;
    int rc = launch_queued(c, q, gated);
    if (rc) {
        c->args = keep;
        return rc;
    }
    ++c->q_seq;
    ++c->q_n;
    return HETM_OK;
}

int round_collect(hetm_ctx *c, hetm_round_result *res) {
    if (c->q_n == 0) return fail(c, HETM_ESTATE, "no round queued");
    hetm_ctx::Queued q = c->queued[c->q_head];
    hetm_ctx::Queued *next = c->q_n > 1 ? &c->queued[(c->q_head + 1) & 1] : nullptr;
    c->q_head = (c->q_head + 1) & 1;
    --c->q_n;
    if (q.cancelled) return fail(c, HETM_ESTATE, "round not run: the round queued before it failed");
    HIP_TRY(c, hipEventSynchronize(c->q_end[q.slot]));
    const DevCounters snap = c->snap_host[q.slot];
    ++c->epoch;
    const int b = q.slot;
    c->buf = b ^ 1;                 // a round outside the queue takes the other buffer next
    const bool undo_ok = c->undo_cap && !snap.undo_over;
    int rc;
    if (snap.hold) {
        // the round behind ran empty (its upload saw the hold) and stays
        // cancelled unless it is launched again below; once it has ended the
        // stream is idle and this round is handled as round_end handles it
        if (next) {
            next->cancelled = true;
            HIP_TRY(c, hipEventSynchronize(c->q_end[next->slot]));
        }
        if (snap.error) {
            if (!undo_ok && (rc = drain_merges(c))) return rc;
            return discard_round(c, snap.error, snap.err_index, q.hdev, undo_ok);
        }
        // conflict under CPU wins without a whole undo log: the dirty
        // granules come back from the host replica (done before returning,
        // as hetm_round does), then the round behind runs for real
        if ((rc = drain_merges(c))) return rc;
        launch_restore(c->stmr, q.hdev, c->stage_ids[b], c->stage_count[b], c->cfg.n_words, c->cfg.granule_words,
                       c->cfg.word_bytes, c->slot, c->stream);
        HIP_TRY(c, hipGetLastError());
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if (next) {
            if ((rc = launch_queued(c, *next, false))) return rc;
            next->cancelled = false;
        }
    } else if (!snap.error && (!snap.conflict || q.r.policy == HETM_POLICY_GPU_WINS)) {
        // the GPU's granules go to the host replica: the round behind is
        // already queued, so the copy is issued now (after this round's end)
        if (c->merge_seq[b] && hetm::merge_wait(c->merger, c->merge_seq[b]) != HETM_OK)
            return fail(c, HETM_EDEVICE, "merge copy to the host replica failed");
        c->merge_deferred = true;
        c->deferred_ev = c->q_end[b];
        c->deferred_buf = b;
        c->deferred_n = snap.n_dirty;
        c->deferred_host = q.r.host_replica;
        c->pending[b] = true;
        c->last_copy = b;
        if (res) res->merge_pending = 1;
        if (next && (rc = issue_merge(c, nullptr))) return rc;
    }
    // a version reset queued here runs after the round behind, whose
    // snapshot then still shows the clock from before it
    const uint64_t resets = c->stats.version_resets;
    account_round(c, snap, q.r.n_txns, q.r.policy, res, q.seq >= c->reset_floor_seq);
    if (c->stats.version_resets != resets) c->reset_floor_seq = c->q_seq;
    if (res) res->us_total = elapsed_us(c->q_begin[b], c->q_end[b]);
    c->stats.log_entries += q.r.n_log;
    return HETM_OK;
}

uint64_t last_merge_seq(hetm_ctx *c) { return c->round_merge_seq; }

int issue_deferred_merge(hetm_ctx *c) { return issue_merge(c, nullptr); }

uint64_t merged_seq(hetm_ctx *c) { return c->merger ? merge_done(c->merger) : 0; }

int wait_merged(hetm_ctx *c, uint64_t seq) {
    if (!c->merger || !seq) return HETM_OK;
    return merge_wait(c->merger, seq) == HETM_OK ? HETM_OK : fail(c, HETM_EDEVICE, "merge copy failed");
}

}  // namespace hetm

extern "C" {

const char *hetm_strerror(int code) {
    switch (code) {
    case HETM_OK: return "ok";
    case HETM_EINVAL: return "invalid argument";
    case HETM_ENOMEM: return "out of memory";
    case HETM_EORDER: return "timestamp order violated";
    case HETM_ECAPACITY: return "capacity exceeded";
    case HETM_EDEVICE: return "HIP runtime error";
    case HETM_ERETRY: return "transaction exceeded the local retry cap";
    case HETM_ESTATE: return "call out of round order";
    default: return "unknown error";
    }
}

// detail of the last failed hetm_alloc_stmr of this thread (no context exists then)
static thread_local char g_alloc_err[512] = "no failed allocation";

const char *hetm_last_error(hetm_ctx *ctx) { return ctx ? ctx->err : g_alloc_err; }

namespace {
// Records why an allocation failed (with the pending HIP error, if any),
// releases what the context holds and returns code.
int alloc_fail(hetm_ctx *c, int code, const char *what) {
    const hipError_t e = hipGetLastError();
    snprintf(g_alloc_err, sizeof g_alloc_err, "%s%s%s%s%s", what, c && c->err[0] ? ": " : "", c ? c->err : "",
             e != hipSuccess ? "; HIP: " : "", e != hipSuccess ? hipGetErrorString(e) : "");
    if (c) hetm_free(c);
    return code;
}
}  // namespace

int hetm_alloc_stmr(const hetm_config *cfg, const void *init_image, hetm_ctx **out) {
    if (!cfg || !out) return HETM_EINVAL;
    *out = nullptr;
    const hetm_config &k = *cfg;
    if (k.n_words == 0 || k.n_words >= (1ull << 32) || (k.word_bytes != 4 && k.word_bytes != 8) ||
        k.granule_words == 0 || !is_pow2(k.lock_stripe_words) || k.max_txn_ops == 0 || k.max_txn_ops > 64 ||
        k.batch_capacity == 0 || k.batch_capacity > (1ull << 31) || k.log_capacity == 0 ||
        k.log_capacity > (1ull << 29) || k.mode > HETM_MODE_GRAPH || k.async_merge > 1 ||
        (k.async_merge && k.mode != HETM_MODE_GRAPH))
        return HETM_EINVAL;
    hetm_ctx *c = new (std::nothrow) hetm_ctx();
    if (!c) return HETM_ENOMEM;
    c->cfg = k;
    if (c->cfg.retry_cap == 0) c->cfg.retry_cap = 1u << 24;
    c->device = k.device;
    c->log_entry_bytes = k.word_bytes == 4 ? sizeof(hetm_log_entry4) : sizeof(hetm_log_entry8);
    int rc = HETM_OK;
#define TRY(x)                                   \
    do {                                         \
        rc = (x);                                \
        if (rc) return alloc_fail(c, rc, #x);    \
    } while (0)
    if (hipSetDevice(k.device) != hipSuccess) {
        delete c;
        return alloc_fail(nullptr, HETM_EDEVICE, "hipSetDevice");
    }
    TRY(scratch_for_device(k.device, &c->scratch));
    c->stream = (hipStream_t)k.stream;
    const uint64_t N = k.n_words, G = k.granule_words;
    const uint64_t nG = (N + G - 1) / G;
    const uint64_t nbw = (nG + 31) / 32;
    const uint64_t nrw = (nG + 3) / 4;
    const uint64_t nblocks = (nbw + kScanWordsPerBlock - 1) / kScanWordsPerBlock;
    const uint64_t nlocks = (N + k.lock_stripe_words - 1) / k.lock_stripe_words;
    // u32 words with one lock per word use the slot layout (value, version
    // and lock in one u64); otherwise a value array plus a lock table
    c->slot = k.word_bytes == 4 && k.lock_stripe_words == 1;
    if (c->slot) {
        TRY(dev_alloc(c, &c->stmr, N * 8));
    } else {
        TRY(dev_alloc(c, &c->stmr, N * k.word_bytes));
        TRY(dev_alloc(c, &c->locks, nlocks * 8));
    }
    TRY(dev_alloc(c, &c->ts, N * 8));
    TRY(dev_alloc(c, &c->rs, nrw * 4));
    TRY(dev_alloc(c, &c->ws, nbw * 4));
    c->log_bins = log_bins_for(k.log_capacity);
    c->log_tiles = log_tiles_for(k.log_capacity);
    // at most one spill chunk per bin block and bucket
    TRY(dev_alloc(c, &c->log_desc, (uint64_t)c->log_tiles * c->log_bins * 12));
    TRY(dev_alloc(c, &c->log_bstart, c->log_bins * 4ull));
    TRY(dev_alloc(c, &c->log_bwin, c->log_bins * 4ull));
    TRY(dev_alloc(c, &c->log_head, c->log_bins * 4ull));
    TRY(dev_alloc(c, &c->log_cursor, c->log_bins * 4ull));
    // every bucket has a region of log_region entries; the spill area
    // behind them takes what does not fit (at most the chunk), and a
    // contiguous copy of every bucket that spilled (at most the chunk again)
    c->log_region = log_region_for(k.log_capacity, c->log_bins);
    const uint64_t sorted_entries = (uint64_t)c->log_bins * c->log_region + 2 * k.log_capacity;
    TRY(dev_alloc(c, &c->log_sorted, sorted_entries * c->log_entry_bytes));
    TRY(dev_alloc(c, &c->log_win, sorted_entries * c->log_entry_bytes));
    TRY(dev_alloc(c, &c->blocksums, nblocks * 4));
    TRY(dev_alloc(c, &c->blockruns, nblocks * 4));
    TRY(dev_alloc(c, &c->ids, nG * 4));
    TRY(dev_alloc(c, &c->order, k.batch_capacity * 4));
    // slot layout: the undo log of the fast rollback, one record per word a
    // round's transactions write first, room for 8 per transaction of a batch
    if (c->slot) {
        const uint64_t cap = std::min<uint64_t>({N, 8 * k.batch_capacity, 0xFFFFFFFFull});
        TRY(dev_alloc(c, &c->undo, cap * 8));
        c->undo_cap = (uint32_t)cap;
    }
    // the hot-object chains of the TRANSFER and CACHE programs
    TRY(dev_alloc(c, &c->tx_tab, kTxTabSlots * 8ull));
    TRY(dev_alloc(c, &c->tx_hot, kTxMaxHot * 8ull));
    TRY(dev_alloc(c, &c->tx_chain, kTxChainWords * 4ull));
    TRY(dev_alloc(c, &c->log_staging, k.log_capacity * c->log_entry_bytes));
    TRY(dev_alloc(c, &c->cnt, sizeof(DevCounters)));
    TRY(dev_alloc(c, &c->hot, sizeof(HotCounters)));
    TRY(dev_alloc(c, &c->dargs, sizeof(DevArgs)));
    if (k.async_merge) {
        for (int b = 0; b < 2; ++b) {
            TRY(dev_alloc(c, &c->staging[b], nG * G * k.word_bytes));
            TRY(dev_alloc(c, &c->stage_ids[b], nG * 4));
            TRY(dev_alloc(c, &c->stage_count[b], 256));
            // pinned host staging for every granule: sized once, so no
            // allocation (or the device-wide wait of a free) sits in a round
            if (hipHostMalloc((void **)&c->host_stage[b], nG * G * k.word_bytes, hipHostMallocDefault) != hipSuccess ||
                hipHostMalloc((void **)&c->host_ids[b], nG * 4, hipHostMallocDefault) != hipSuccess)
                return alloc_fail(c, HETM_ENOMEM, "pinned host staging");
            touch_pages(c->host_stage[b], nG * G * k.word_bytes);
            touch_pages(c->host_ids[b], nG * 4);
            c->host_cap[b] = nG;
        }
        if (hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking) != hipSuccess)
            return alloc_fail(c, HETM_EDEVICE, "copy stream");
        c->merger = hetm::merge_worker_create();
        if (!c->merger) return alloc_fail(c, HETM_ENOMEM, "merge worker");
        for (int b = 0; b < 2; ++b)
            if (hipEventCreateWithFlags(&c->copied[b], hipEventDisableTiming) != hipSuccess)
                return alloc_fail(c, HETM_EDEVICE, "merge events");
    }
    if (hipHostMalloc((void **)&c->hargs, sizeof(DevArgs), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&c->snap_host, 2 * sizeof(DevCounters), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&c->cnt_host, sizeof(DevCounters), hipHostMallocDefault) != hipSuccess)
        return alloc_fail(c, HETM_ENOMEM, "pinned host counters");
    // the round's finish kernel stores its counter snapshot straight into
    // pinned host memory (no copy after it on the round's critical path)
    if (hipHostGetDevicePointer((void **)&c->snap_map, c->snap_host, 0) != hipSuccess || !c->snap_map)
        return alloc_fail(c, HETM_EDEVICE, "device address of the pinned snapshot");
    memset(c->snap_host, 0, 2 * sizeof(DevCounters));
    for (hipEvent_t *e : {&c->ev[0], &c->ev[1], &c->ev[2], &c->ev[3], &c->ev_kernel, &c->q_begin[0], &c->q_begin[1],
                          &c->q_end[0], &c->q_end[1]})
        if (hipEventCreate(e) != hipSuccess) return alloc_fail(c, HETM_EDEVICE, "timing events");
    if (hipStreamCreateWithFlags(&c->early_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->closed_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->early_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->exec_queued, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void **)&c->early_host, sizeof(uint32_t), hipHostMallocDefault) != hipSuccess)
        return alloc_fail(c, HETM_EDEVICE, "early-validation stream and events");
    hipStream_t s = c->stream;
    bool ok = (c->slot || hipMemsetAsync(c->locks, 0, nlocks * 8, s) == hipSuccess) &&
              hipMemsetAsync(c->rs, 0, nrw * 4, s) == hipSuccess &&
              hipMemsetAsync(c->log_cursor, 0, c->log_bins * 4ull, s) == hipSuccess &&
              hipMemsetAsync(c->log_head, 0xFF, c->log_bins * 4ull, s) == hipSuccess &&
              hipMemsetAsync(c->ws, 0, nbw * 4, s) == hipSuccess &&
              hipMemsetAsync(c->cnt, 0, sizeof(DevCounters), s) == hipSuccess &&
              hipMemsetAsync(c->hot, 0, sizeof(HotCounters), s) == hipSuccess &&
              hipMemsetAsync(c->blocksums, 0, nblocks * 4, s) == hipSuccess &&
              hipMemsetAsync(c->tx_tab, 0, kTxTabSlots * 8ull, s) == hipSuccess &&
              hipMemsetAsync(c->tx_chain, 0, kTxChainWords * 4ull, s) == hipSuccess;
    static const uint32_t kNoApply = 0xFFFFFFFFu;
    ok = ok && hipMemcpyAsync(&c->cnt->apply_floor, &kNoApply, 4, hipMemcpyHostToDevice, s) == hipSuccess;
    if (!ok) return alloc_fail(c, HETM_EDEVICE, "clearing the context's state");
    if (c->slot && init_image) {
        // the image goes through the TS array (N u64, cleared afterwards)
        if (hipMemcpyAsync(c->ts, init_image, N * 4, hipMemcpyDefault, s) != hipSuccess)
            return alloc_fail(c, HETM_EDEVICE, "copying the initial image");
        (void)hipGetLastError();     // an error left by earlier, unrelated calls must not count here
        launch_to_slots((const uint32_t *)c->ts, (uint64_t *)c->stmr, N, s);
        if (hipPeekAtLastError() != hipSuccess) return alloc_fail(c, HETM_EDEVICE, "slot-layout conversion");
    } else {
        ok = init_image ? hipMemcpyAsync(c->stmr, init_image, N * k.word_bytes, hipMemcpyDefault, s) == hipSuccess
                        : hipMemsetAsync(c->stmr, 0, c->slot ? N * 8 : N * k.word_bytes, s) == hipSuccess;
        if (!ok) return alloc_fail(c, HETM_EDEVICE, "copying the initial image");
    }
    if (hipMemsetAsync(c->ts, 0, N * 8, s) != hipSuccess) return alloc_fail(c, HETM_EDEVICE, "clearing TS");
    if (hipStreamSynchronize(s) != hipSuccess) return alloc_fail(c, HETM_EDEVICE, "initial synchronization");
    hipDeviceProp_t prop;
    int cus = 256;
    if (hipGetDeviceProperties(&prop, k.device) == hipSuccess) cus = prop.multiProcessorCount;
    c->exec_wg = k.exec_workgroups ? k.exec_workgroups : default_exec_workgroups(cus);
    if (exec_prepare(k.max_txn_ops) != hipSuccess) return alloc_fail(c, HETM_EDEVICE, "transaction-kernel LDS limit");

    DevArgs &a = c->args;
    a.stmr = c->stmr, a.locks = c->locks, a.ts = c->ts, a.rs = c->rs, a.ws = c->ws;
    a.word_shift = c->slot ? 1u : 0u;
    a.blocksums = c->blocksums, a.blockruns = c->blockruns, a.ids_scratch = c->ids;
    a.log_desc = c->log_desc, a.log_bstart = c->log_bstart, a.log_bwin = c->log_bwin, a.log_head = c->log_head;
    a.log_cursor = c->log_cursor, a.log_region = c->log_region, a.log_spill_cap = (uint32_t)(2 * c->cfg.log_capacity);
    a.log_sorted = c->log_sorted, a.log_win = c->log_win;
    a.log_bins = c->log_bins, a.log_bin_bits = ilog2(c->log_bins), a.log_tiles = c->log_tiles;
    a.order = c->order;
    a.tx_tab = c->tx_tab, a.tx_hot = c->tx_hot, a.tx_chain = c->tx_chain;
    a.undo = c->undo, a.undo_cap = c->undo_cap;
    a.cnt = c->cnt;
    a.hot = c->hot;
    a.gdiv = make_div32((uint32_t)G);
    a.n_words = N, a.word_bytes = k.word_bytes, a.granule = (uint32_t)G;
    a.stripe_shift = ilog2(k.lock_stripe_words);
    a.n_granules = (uint32_t)nG, a.n_bm_words = (uint32_t)nbw, a.n_rs_words = (uint32_t)nrw;
    a.retry_cap = c->cfg.retry_cap;
    a.max_ops = k.max_txn_ops, a.n_scan_blocks = (uint32_t)nblocks;
    a.outcome = HETM_OUTCOME_DEVICE;
    c->stats.device_bytes = c->device_bytes;
    *out = c;
    return HETM_OK;
#undef TRY
}

int hetm_free(hetm_ctx *c) {
    if (!c) return HETM_EINVAL;
    (void)hipSetDevice(c->device);
    if (c->merge_deferred) (void)issue_merge(c, nullptr);   // the last round's copy still reaches the host
    // every queue of the context drains before its memory goes
    for (hipStream_t s : {c->stream, c->cap_stream, c->cap_branch, c->copy_stream, c->early_stream})
        if (s) (void)hipStreamSynchronize(s);
    hetm::merge_worker_destroy(c->merger);     // finishes the queued scatters first
    for (int b = 0; b < 2; ++b) {
        if (c->host_stage[b]) (void)hipHostFree(c->host_stage[b]);
        if (c->host_ids[b]) (void)hipHostFree(c->host_ids[b]);
    }
    drop_graphs(c);
    if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
    if (c->join_ev) (void)hipEventDestroy(c->join_ev);
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    if (c->ev_kernel) (void)hipEventDestroy(c->ev_kernel);
    for (hipEvent_t e : {c->q_begin[0], c->q_begin[1], c->q_end[0], c->q_end[1]})
        if (e) (void)hipEventDestroy(e);
    void *dev[] = {c->stmr, c->locks, c->ts, c->rs, c->ws, c->log_desc, c->log_bstart, c->log_bwin, c->log_head,
                   c->log_cursor, c->log_sorted, c->log_win, c->blocksums, c->blockruns, c->ids, c->order, c->undo,
                   c->tx_tab, c->tx_hot, c->tx_chain, c->log_staging, c->cnt, c->hot, c->dargs};
    for (void *p : dev)
        if (p) (void)hipFree(p);
    if (c->hargs) (void)hipHostFree(c->hargs);
    if (c->snap_host) (void)hipHostFree(c->snap_host);
    if (c->cnt_host) (void)hipHostFree(c->cnt_host);
    if (c->early_host) (void)hipHostFree(c->early_host);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->cap_branch) (void)hipStreamDestroy(c->cap_branch);
    for (int b = 0; b < 2; ++b) {
        if (c->copied[b]) (void)hipEventDestroy(c->copied[b]);
        if (c->staging[b]) (void)hipFree(c->staging[b]);
        if (c->stage_ids[b]) (void)hipFree(c->stage_ids[b]);
        if (c->stage_count[b]) (void)hipFree(c->stage_count[b]);
    }
    if (c->copy_stream) (void)hipStreamDestroy(c->copy_stream);
    if (c->early_stream) (void)hipStreamDestroy(c->early_stream);
    if (c->closed_ev) (void)hipEventDestroy(c->closed_ev);
    if (c->early_ev) (void)hipEventDestroy(c->early_ev);
    if (c->exec_queued) (void)hipEventDestroy(c->exec_queued);
    delete c;
    return HETM_OK;
}

int hetm_submit_batch(hetm_ctx *c, uint32_t program, const void *descs, uint64_t n_txns, void *results,
                      uint32_t *tickets) {
    if (!c) return HETM_EINVAL;
    if (int rc = refuse_queued(c)) return rc;
    if (c->in_validation) return fail(c, HETM_ESTATE, "submit after validation started in this round");
    c->args.policy = HETM_POLICY_CPU_WINS;     // the step API applies each chunk as it comes
    if (n_txns == 0) return HETM_OK;
    int rc = set_batch_args(c, program, descs, n_txns, results, tickets);
    if (rc) return rc;
    if ((rc = push_args(c))) return rc;
    launch_exec(program, c->dargs, c->exec_wg, c->cfg.max_txn_ops, c->slot, c->cfg.batch_capacity, c->stream);
    HIP_TRY(c, hipGetLastError());
    return HETM_OK;
}

int hetm_validate_apply_log(hetm_ctx *c, const void *log, uint64_t n, uint32_t *flags_bits, uint32_t *conflict_out) {
    if (!c) return HETM_EINVAL;
    if (int rc = refuse_queued(c)) return rc;
    if (n > c->cfg.log_capacity) return fail(c, HETM_ECAPACITY, "log chunk %llu > capacity", (unsigned long long)n);
    if (n && !log) return fail(c, HETM_EINVAL, "null log");
    c->in_validation = true;
    c->args.policy = HETM_POLICY_CPU_WINS;
    if (n) {
        const void *dlog = nullptr;
        int rc = stage_log(c, log, n, &dlog);
        if (rc) return rc;
        if ((rc = enqueue_validate(c, dlog, n, flags_bits))) return rc;
    }
    if (conflict_out) {
        DevCounters k;
        int rc = read_counters(c, &k);
        if (rc) return rc;
        *conflict_out = k.conflict;
        if (k.error) return take_device_error(c, k.error, k.err_index);
    }
    return HETM_OK;
}

int hetm_copyback_dirty(hetm_ctx *c, uint32_t conflict, void *host_replica, uint64_t *n_dirty_out,
                        uint32_t *ids_out) {
    if (!c) return HETM_EINVAL;
    if (int rc = refuse_queued(c)) return rc;
    if (conflict > 1 && conflict != HETM_OUTCOME_DEVICE) return fail(c, HETM_EINVAL, "bad outcome %u", conflict);
    const void *hdev = nullptr;
    int rc = check_host_replica(c, host_replica, &hdev);
    if (rc) return rc;
    if ((rc = enqueue_merge(c, conflict, hdev, ids_out))) return rc;
    c->in_validation = false;
    if (n_dirty_out) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        const DevCounters s = *c->snap_host;
        if (s.error) return take_device_error(c, s.error, s.err_index);
        account_round(c, s, 0, c->args.policy, nullptr);
        *n_dirty_out = s.n_dirty;
    }
    return HETM_OK;
}

int hetm_round(hetm_ctx *c, const hetm_round_args *r, hetm_round_result *res) {
    if (!c || !r) return HETM_EINVAL;
    if (res) memset(res, 0, sizeof *res);
    if (int rc = refuse_queued(c)) return rc;
    if (c->cfg.mode == HETM_MODE_GRAPH) {
        int rc = hetm::round_begin(c, r);
        if (rc) return rc;
        return hetm::round_end(c, r, res);
    }
    if (c->in_validation) return fail(c, HETM_ESTATE, "hetm_round inside an open round");
    if (r->policy > HETM_POLICY_GPU_WINS) return fail(c, HETM_EINVAL, "bad policy %u", r->policy);
    c->args.policy = r->policy;
    if (r->n_log > c->cfg.log_capacity) return fail(c, HETM_ECAPACITY, "log %llu > capacity", (unsigned long long)r->n_log);
    if (r->n_log && !r->log) return fail(c, HETM_EINVAL, "null log");
    const void *hdev = nullptr;
    int rc = check_host_replica(c, r->host_replica, &hdev);
    if (rc) return rc;
    if (r->n_txns) {
        if ((rc = set_batch_args(c, r->program, r->descs, r->n_txns, r->results, r->tickets))) return rc;
    } else {
        c->args.n_txns = 0;
    }
    hipStream_t s = c->stream;
    // PLAIN: one launch per step, outcome read on the host
    HIP_TRY(c, hipEventRecord(c->ev[0], s));
    if (r->n_txns) {
        if ((rc = push_args(c))) return rc;
        launch_exec(r->program, c->dargs, c->exec_wg, c->cfg.max_txn_ops, c->slot, c->cfg.batch_capacity, s,
                    c->ev_kernel);
        HIP_TRY(c, hipGetLastError());
    }
    HIP_TRY(c, hipEventRecord(c->ev[1], s));
    if (r->n_log) {
        const void *dlog = nullptr;
        if ((rc = stage_log(c, r->log, r->n_log, &dlog))) return rc;
        if ((rc = enqueue_validate(c, dlog, r->n_log, r->flags_bits))) return rc;
    }
    HIP_TRY(c, hipEventRecord(c->ev[2], s));
    DevCounters k;
    if ((rc = read_counters(c, &k))) return rc;
    if (k.error) return discard_round(c, k.error, k.err_index, hdev, c->undo_cap && !k.undo_over);
    if ((rc = enqueue_merge(c, k.conflict, hdev, r->ids_out))) return rc;
    HIP_TRY(c, hipEventRecord(c->ev[3], s));
    HIP_TRY(c, hipStreamSynchronize(s));
    const DevCounters snap = *c->snap_host;
    if (snap.error) return take_device_error(c, snap.error, snap.err_index);
    account_round(c, snap, r->n_txns, c->args.policy, res);
    c->stats.log_entries += r->n_log;
    if (res) {
        res->us_exec = elapsed_us(c->ev[0], c->ev[1]);
        res->us_exec_kernel = r->n_txns ? elapsed_us(c->ev_kernel, c->ev[1]) : 0.0;
        res->us_validate = elapsed_us(c->ev[1], c->ev[2]);
        res->us_merge = elapsed_us(c->ev[2], c->ev[3]);
        res->us_total = elapsed_us(c->ev[0], c->ev[3]);
    }
    return HETM_OK;
}

int hetm_round_begin(hetm_ctx *c, const hetm_round_args *r) {
    if (!c || !r) return HETM_EINVAL;
    if (int rc = refuse_queued(c)) return rc;
    return hetm::stream_begin(c, r);
}

int hetm_round_submit(hetm_ctx *c, const hetm_round_args *r) {
    if (!c || !r) return HETM_EINVAL;
    return hetm::round_submit(c, r);
}

int hetm_round_collect(hetm_ctx *c, hetm_round_result *res) {
    if (!c) return HETM_EINVAL;
    if (res) memset(res, 0, sizeof *res);
    return hetm::round_collect(c, res);
}

int hetm_round_push(hetm_ctx *c, const void *log, uint64_t n, uint32_t *doomed_out) {
    if (!c) return HETM_EINVAL;
    return hetm::stream_push(c, log, n, doomed_out);
}

int hetm_round_add(hetm_ctx *c, uint32_t program, const void *descs, uint64_t n_txns, void *results,
                   uint32_t *tickets) {
    if (!c) return HETM_EINVAL;
    return hetm::stream_add(c, program, descs, n_txns, results, tickets);
}

int hetm_round_end(hetm_ctx *c, hetm_round_result *res) {
    if (!c) return HETM_EINVAL;
    if (res) memset(res, 0, sizeof *res);
    return hetm::stream_end(c, res);
}

int hetm_early_validate(hetm_ctx *c, const void *log, uint64_t n, uint32_t *doomed_out) {
    if (!c || (n && !log)) return HETM_EINVAL;
    if (int rc = refuse_queued(c)) return rc;
    if (c->cfg.mode != HETM_MODE_PLAIN) return fail(c, HETM_ESTATE, "early validation needs the step API");
    if (n) {
        const void *dlog = device_view(log);
        if (!dlog) return fail(c, HETM_EINVAL, "early validation needs a device or pinned log");
        // the context's stream carries the batch: wait only for the last round's bitmap reset
        if (c->closed_recorded) HIP_TRY(c, hipStreamWaitEvent(c->early_stream, c->closed_ev, 0));
        launch_early_validate(dlog, n, c->cfg.word_bytes, c->rs, c->args.gdiv, c->cfg.n_words, c->epoch, c->cnt,
                              c->early_stream);
        HIP_TRY(c, hipGetLastError());
        HIP_TRY(c, hipEventRecord(c->early_ev, c->early_stream));
        c->early_used = true;
    }
    if (doomed_out) {
        HIP_TRY(c, hipMemcpyAsync(c->early_host, &c->cnt->doomed, sizeof(uint32_t), hipMemcpyDeviceToHost,
                                  c->early_stream));
        HIP_TRY(c, hipStreamSynchronize(c->early_stream));
        *doomed_out = *c->early_host == c->epoch;
    }
    return HETM_OK;
}

int hetm_set_version_clock(hetm_ctx *c, uint32_t value) {
    if (!c) return HETM_EINVAL;
    if (int rc = refuse_queued(c)) return rc;
    if (!c->slot) return fail(c, HETM_ESTATE, "the context keeps no version clock (split layout)");
    if (c->round_open || c->in_validation) return fail(c, HETM_ESTATE, "a round is open");
    if (value >= kClockLimit) return fail(c, HETM_EINVAL, "clock %u past the limit", value);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    uint32_t cur = 0;
    HIP_TRY(c, hipMemcpy(&cur, &c->hot->clock.v, 4, hipMemcpyDeviceToHost));
    if (value < cur) return fail(c, HETM_EINVAL, "the clock only moves forward (%u < %u)", value, cur);
    HIP_TRY(c, hipMemcpy(&c->hot->clock.v, &value, 4, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(&c->cnt->clock_base, &value, 4, hipMemcpyHostToDevice));
    return HETM_OK;
}

int hetm_set_exec_workgroups(hetm_ctx *c, uint32_t workgroups) {
    if (!c || c->round_open) return HETM_EINVAL;
    if (int rc = refuse_queued(c)) return rc;
    if (workgroups == 0) {
        hipDeviceProp_t prop;
        int cus = 256;
        if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) cus = prop.multiProcessorCount;
        workgroups = default_exec_workgroups(cus);
    }
    c->exec_wg = workgroups;
    if (c->graphs[0].exec || c->graphs[1].exec) {
        (void)hipStreamSynchronize(c->stream);
        drop_graphs(c);
    }
    return HETM_OK;
}

int hetm_sync(hetm_ctx *c) {
    if (!c) return HETM_EINVAL;
    int dr = drain_merges(c);
    if (dr) return dr;
    DevCounters k;
    int rc = read_counters(c, &k);
    if (rc) return rc;
    return take_device_error(c, k.error, k.err_index);
}

int hetm_stats_get(hetm_ctx *c, hetm_stats *out) {
    if (!c || !out) return HETM_EINVAL;
    *out = c->stats;
    if (c->merger) hetm::merge_times(c->merger, &out->us_host_scatter, &out->us_merge_wait);
    return HETM_OK;
}

uint64_t hetm_state_bytes(hetm_ctx *c, uint32_t what) {
    if (!c) return 0;
    const uint64_t N = c->cfg.n_words;
    switch (what) {
    case HETM_STATE_STMR: return N * c->cfg.word_bytes;
    case HETM_STATE_RS:
    case HETM_STATE_WS: return (uint64_t)c->args.n_bm_words * 4;
    case HETM_STATE_LOCKS: return ((N + c->cfg.lock_stripe_words - 1) / c->cfg.lock_stripe_words) * 8;
    default: return 0;
    }
}

int hetm_read_state(hetm_ctx *c, uint32_t what, void *dst, uint64_t bytes) {
    if (!c || !dst) return HETM_EINVAL;
    if (int rc = refuse_queued(c)) return rc;
    const void *src = what == HETM_STATE_STMR ? c->stmr
                      : what == HETM_STATE_RS  ? (const void *)c->rs
                      : what == HETM_STATE_WS  ? (const void *)c->ws
                      : what == HETM_STATE_LOCKS ? (c->slot ? c->stmr : (const void *)c->locks)
                                                 : nullptr;
    if (!src || bytes != hetm_state_bytes(c, what)) return fail(c, HETM_EINVAL, "bad state request");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    int dr = drain_merges(c);
    if (dr) return dr;
    if (what == HETM_STATE_STMR && c->slot) {
        // the values of the slots, through a scratch buffer
        uint32_t *tmp = nullptr;
        HIP_TRY(c, hipMalloc((void **)&tmp, bytes ? bytes : 4));
        launch_from_slots((const uint64_t *)c->stmr, tmp, c->cfg.n_words, c->stream);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e == hipSuccess) e = hipMemcpy(dst, tmp, bytes, hipMemcpyDefault);
        (void)hipFree(tmp);
        if (e != hipSuccess) return fail(c, HETM_EDEVICE, "%s", hipGetErrorString(e));
        return HETM_OK;
    }
    if (what == HETM_STATE_RS) {
        // the device keeps one byte per granule; callers get the bitmap
        const uint64_t nG = c->args.n_granules;
        const uint64_t off = (nG + 3) & ~3ull;
        uint8_t *bytes_map = new (std::nothrow) uint8_t[off + bytes];
        if (!bytes_map) return fail(c, HETM_ENOMEM, "read-set copy");
        uint32_t *bits = (uint32_t *)(bytes_map + off);
        memset(bits, 0, bytes);
        hipError_t e = hipMemcpy(bytes_map, src, nG, hipMemcpyDeviceToHost);
        if (e == hipSuccess) {
            for (uint64_t g = 0; g < nG; ++g)
                if (bytes_map[g]) bits[g >> 5] |= 1u << (g & 31);
            e = hipMemcpy(dst, bits, bytes, hipMemcpyDefault);
        }
        delete[] bytes_map;
        if (e != hipSuccess) return fail(c, HETM_EDEVICE, "%s", hipGetErrorString(e));
        return HETM_OK;
    }
    HIP_TRY(c, hipMemcpy(dst, src, bytes, hipMemcpyDefault));
    return HETM_OK;
}

int hetm_read_words_noalloc(hetm_ctx *c, uint64_t first_word, uint64_t n_words, void *dst) {
    if (!c || (!dst && n_words)) return HETM_EINVAL;
    if (int rc = refuse_queued(c)) return rc;
    if (n_words > kNoAllocWords)
        return fail(c, HETM_ECAPACITY, "hetm_read_words_noalloc: %llu words exceed the limit of %llu per call",
                    (unsigned long long)n_words, (unsigned long long)kNoAllocWords);
    if (first_word > c->cfg.n_words || n_words > c->cfg.n_words - first_word)
        return fail(c, HETM_EINVAL, "hetm_read_words_noalloc: words [%llu, +%llu) outside the replica",
                    (unsigned long long)first_word, (unsigned long long)n_words);
    if (n_words == 0) return HETM_OK;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    int dr = drain_merges(c);
    if (dr) return dr;
    const uint64_t bytes = n_words * c->cfg.word_bytes;
    if (!c->slot) {
        // a value array: the words are already what the caller reads
        HIP_TRY(c, hipMemcpyAsync(dst, (const uint8_t *)c->stmr + first_word * c->cfg.word_bytes, bytes,
                                  hipMemcpyDefault, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        return HETM_OK;
    }
    if (!c->scratch) return fail(c, HETM_EDEVICE, "hetm_read_words_noalloc: no scratch array on device %d", c->device);
    // the slots' values through this device's array; every word copied out
    // is written first, so what the last call left there does not matter
    std::lock_guard<std::mutex> g(g_scratch_use[c->device]);
    launch_from_slots((const uint64_t *)c->stmr + first_word, (uint32_t *)c->scratch, n_words, c->stream);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipMemcpyAsync(dst, c->scratch, bytes, hipMemcpyDefault, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return HETM_OK;
}

}  // extern "C"
