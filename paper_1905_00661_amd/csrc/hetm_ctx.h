// hetm_ctx.h -- the context behind the opaque hetm_ctx handle, and the
// internal round steps shared by the C ABI and the serve loop.
#pragma once

#include <hip/hip_runtime.h>

#include "hetm.h"
#include "hetm_dev.h"
#include "merge_host.h"

using hetm::DevArgs;
using hetm::DevCounters;
using hetm::HotCounters;

struct hetm_ctx {
    hetm_config cfg{};
    hipStream_t stream = nullptr;      // the caller's stream (nullptr = default stream)
    hipStream_t cap_stream = nullptr;  // private non-blocking stream the round graphs are captured on
    int device = 0;
    uint32_t exec_wg = 0;
    uint32_t log_entry_bytes = 16;

    // device state
    bool slot = false;                 // u32 words in the slot layout (stmr holds N u64 slots, no lock table)
    void *stmr = nullptr;
    uint64_t *locks = nullptr;
    uint64_t *ts = nullptr;
    uint8_t *rs = nullptr;             // read set, one byte per granule
    uint32_t *ws = nullptr;
    // the log chunk bucketed by word (validation and apply)
    uint32_t log_bins = 0, log_tiles = 0;
    uint32_t *log_desc = nullptr, *log_bstart = nullptr, *log_bwin = nullptr, *log_head = nullptr;
    uint32_t *log_cursor = nullptr;    // entries of each bucket
    uint32_t log_region = 0;           // entries a bucket's region holds
    void *log_sorted = nullptr, *log_win = nullptr;
    uint32_t *blocksums = nullptr, *blockruns = nullptr, *ids = nullptr;
    uint32_t *order = nullptr;    // batch_capacity transaction ids (OPLIST kind split, TRANSFER chains)
    uint64_t *tx_tab = nullptr, *tx_hot = nullptr;   // TRANSFER: sample counts, hot accounts
    uint64_t *undo = nullptr;                        // slot layout: the round's undo log
    uint32_t undo_cap = 0;
    uint32_t *tx_chain = nullptr;                    // TRANSFER: chain counts, starts, cursors, order
    void *log_staging = nullptr;
    DevCounters *cnt = nullptr;
    HotCounters *hot = nullptr;
    DevCounters *snap_map = nullptr;   // snap_host as the device addresses it (the finish kernel writes it);
                                       // two snapshots: [0] every round but queued ones, [s] queued slot s
    DevArgs *dargs = nullptr;
    uint64_t device_bytes = 0;
    void *scratch = nullptr;           // this device's copy of the no-allocation read array

    // pinned host mirrors
    DevArgs *hargs = nullptr;        // argument block uploaded by the graph
    DevCounters *snap_host = nullptr;
    DevCounters *cnt_host = nullptr;

    DevArgs args{};                  // host copy of the current arguments
    hipEvent_t ev[4] = {};
    hipEvent_t ev_kernel = nullptr;    // PLAIN rounds: just before the transaction kernel
    // The round graph, one per merge policy (captured on first use).  With
    // the double-buffered merge and CPU wins, the dirty-granule compaction
    // and gather run on a branch of their own beside validation and apply.
    struct RoundGraph {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        uint32_t program = 0;
        hipGraphNode_t args_node = nullptr;   // the argument-upload kernel node
        hipKernelNodeParams args_params{};
    } graphs[2];
    // A streamed round (hetm_round_begin / push / end) is the same round in
    // two graphs, per merge policy: [0] argument upload and execution,
    // [1] argument upload, validation and apply of every pushed chunk, merge
    // and finish.  Chunks pushed in between are copied into log_staging and
    // early-validated on early_stream.
    RoundGraph sgraphs[2][2];
    bool round_streamed = false;
    uint64_t round_pushed = 0;              // log entries pushed so far
    const void *round_log = nullptr;        // where they are: the caller's device buffer, or log_staging
    bool round_in_place = false;            // every chunk so far read in place (device memory, consecutive)
    hetm_round_args round_args{};           // the streamed round's arguments
    hipEvent_t exec_queued = nullptr;       // before the streamed round's execution graph
    hipStream_t cap_branch = nullptr;       // capture only: the merge branch
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;

    // A successful round's copy to the host is issued once the next round's
    // graph is queued (or when something waits for merges): issued at the
    // round's end instead, the copy's host-bound writes delayed the next
    // round's first, host-reading steps (argument upload, kernel dispatch).
    bool merge_deferred = false;
    hipEvent_t deferred_ev = nullptr;       // the end of the round whose copy is deferred
    int deferred_buf = 0;
    uint64_t deferred_n = 0;
    void *deferred_host = nullptr;

    // double-buffered merge (GRAPH mode with async_merge)
    hipStream_t copy_stream = nullptr;
    hipStream_t early_stream = nullptr;     // early validation, beside the running batch
    hipEvent_t closed_ev = nullptr;         // PLAIN: the last round's bitmaps are cleared
    hipEvent_t early_ev = nullptr;          // the last early validation of the round
    bool early_used = false;                // an early validation is queued in the open round
    bool closed_recorded = false;           // closed_ev has been recorded
    uint32_t *early_host = nullptr;         // pinned: doomed flag read back
    uint32_t epoch = 1;                     // number of the open round (tags a doomed round)
    hipEvent_t copied[2] = {};
    bool pending[2] = {false, false};
    int buf = 0;
    int last_copy = -1;
    void *staging[2] = {};
    uint32_t *stage_ids[2] = {};
    uint32_t *stage_count[2] = {};
    uint8_t *host_stage[2] = {};            // pinned: the copied granules, scattered by the merge worker
    uint32_t *host_ids[2] = {};
    uint64_t host_cap[2] = {0, 0};          // granules the pinned staging holds (all of them)
    uint64_t merge_seq[2] = {0, 0};         // worker job that last read host_stage[b]
    uint64_t round_merge_seq = 0;           // the last closed round's merge job (0: none pending)
    hetm::MergeWorker *merger = nullptr;

    // Rounds queued by hetm_round_submit, oldest first, up to two: slot s
    // has its own graph per policy, snapshot, staging buffer and events, so
    // the round behind is launched while the one ahead runs.
    struct Queued {
        hetm_round_args r{};
        const void *hdev = nullptr;
        uint64_t seq = 0;
        int slot = 0;
        bool cancelled = false;      // not run: the round ahead of it failed
    } queued[2];
    uint32_t q_head = 0, q_n = 0;
    uint64_t q_seq = 0;
    uint64_t reset_floor_seq = 0;   // queued rounds below this number saw the clock before a queued reset
    RoundGraph qgraphs[2][2];       // [policy][slot]
    hipEvent_t q_begin[2] = {}, q_end[2] = {};

    // the GRAPH round between round_begin and round_end
    bool round_open = false;
    const void *round_hdev = nullptr;
    void *round_host = nullptr;
    int round_buf = 0;

    bool in_validation = false;      // this round's log has started
    uint32_t chunks_in_round = 0;    // log chunks the open round has taken (step API)
    uint32_t gpu_losses = 0;         // rounds in a row whose GPU transactions aborted
    hetm_stats stats{};
    char err[512] = {0};
};

namespace hetm {
// GRAPH-mode round split in two so a caller can overlap host work with it:
// round_begin checks the arguments, uploads them and launches the captured
// graph; round_end waits for it and handles the outcome (error, staged or
// synchronous merge, restore on conflict) and fills *res.
int round_begin(hetm_ctx *c, const hetm_round_args *r);
int round_end(hetm_ctx *c, const hetm_round_args *r, hetm_round_result *res);
// Streamed GRAPH round: stream_begin launches the execution part;
// stream_push copies a log chunk into the round's log and early-validates
// it beside the execution; stream_end launches the tail (validation and
// apply of every pushed chunk, merge, finish) and ends as round_end does.
int stream_begin(hetm_ctx *c, const hetm_round_args *r);
int stream_push(hetm_ctx *c, const void *log, uint64_t n, uint32_t *doomed_out);
// stream_add launches one more batch into the open streamed round, after
// its earlier batches and before its tail.
int stream_add(hetm_ctx *c, uint32_t program, const void *descs, uint64_t n_txns, void *results, uint32_t *tickets);
int stream_end(hetm_ctx *c, hetm_round_result *res);
// Queued whole rounds: round_submit launches a round behind the ones already
// queued (up to two); round_collect waits for the oldest and handles its
// outcome as round_end does, relaunching or cancelling the round behind it
// when the oldest held it.
int round_submit(hetm_ctx *c, const hetm_round_args *r);
int round_collect(hetm_ctx *c, hetm_round_result *res);
// Double-buffered merge progress.  A successful round's copy to the host is
// issued by the next round_begin (after it queues its graph) or by
// issue_deferred_merge; last_merge_seq is the most recently issued job (0
// after a round that left nothing to merge), merged_seq the last job whose
// granules are in the host replica, wait_merged a wait for a job.
int issue_deferred_merge(hetm_ctx *c);
uint64_t last_merge_seq(hetm_ctx *c);
uint64_t merged_seq(hetm_ctx *c);
int wait_merged(hetm_ctx *c, uint64_t seq);
}  // namespace hetm
