/*
 * hetm.h -- C ABI of libhetm, the GPU side of one Speculative HeTM (SHeTM)
 * synchronization round on an AMD Instinct MI355X (gfx950).
 *
 * Paper: D. Castro, P. Romano, A. Ilic, A. M. Khan, "HeTM: Transactional
 * Memory for Heterogeneous Systems" (arXiv:1905.00661).
 *
 * A round (§IV-C) has three phases:
 *   execution  -- batches of GPU transactions run speculatively against the
 *                 GPU's replica of the shared region (STMR); each committed
 *                 transaction marks its read and written granules in the
 *                 read-set and write-set bitmaps (§IV-B, GPU instrumentation);
 *   validation -- the host's write log of <word, value, timestamp> entries
 *                 (§IV-B, CPU instrumentation) is checked against the
 *                 read-set bitmap and always applied to the GPU replica under
 *                 the per-word timestamp freshness rule (§IV-C.2);
 *   merge      -- the write-set granules are copied GPU->host on success, or
 *                 host->GPU on conflict (§IV-C.3; CPU-wins policy, §IV-E).
 *
 * Conventions for every call:
 *   - Pointers named "device" must be device memory or pinned host memory
 *     (hipHostMalloc) of this context's GPU; "host" pointers are ordinary
 *     host memory; "host-or-device" accepts either.  Sizes are in elements.
 *   - The caller owns every buffer it passes; the library only borrows it
 *     until the call's work has finished on the context's stream.  The
 *     context owns all device state it allocates.
 *   - Calls return HETM_OK (0) or a negative HETM_E* code and never throw.
 *     Errors detected on the device (bad log entries, retry cap) are latched
 *     and returned by the next call that synchronizes.  A failed call leaves
 *     the context usable unless it returned HETM_EDEVICE.
 *   - A context is driven by one host thread (the paper's GPU-controller
 *     thread, §IV-A); calls on one context are not reentrant.  Work is
 *     queued on the context's stream in call order.
 */
#ifndef HETM_H
#define HETM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ error codes */
#define HETM_OK          0
#define HETM_EINVAL     (-1)  /* bad argument, or a log word outside the STMR   */
#define HETM_ENOMEM     (-2)  /* device or pinned allocation failed             */
#define HETM_EORDER     (-3)  /* log timestamp not above the watermark, >= 2^63,
                                 or two entries carry one word's winning ts     */
#define HETM_ECAPACITY  (-4)  /* batch or log larger than the context capacity  */
#define HETM_EDEVICE    (-5)  /* a HIP runtime call failed                      */
#define HETM_ERETRY     (-6)  /* a transaction exceeded the local retry cap     */
#define HETM_ESTATE     (-7)  /* call out of round order                        */

/* --------------------------------------------------------------- programs */
/* Built-in transactional kernels (the paper's "transactional kernel",
 * §IV-A: one kernel runs a whole batch of transactions of one type). */
#define HETM_PROG_OPLIST   1u  /* word-list read / read-modify-write (§V-A)  */
#define HETM_PROG_TRANSFER 2u  /* int64 bank transfer                         */
#define HETM_PROG_CACHE    3u  /* 8-way set-associative object cache (§V-D)  */

/* ------------------------------------------------------------------ modes */
#define HETM_MODE_PLAIN 0u  /* one launch per round step, host reads the outcome */
#define HETM_MODE_GRAPH 1u  /* whole round replayed as one captured hipGraph,
                               outcome decided on the device                    */

/* Pass as `conflict` to hetm_copyback_dirty to use the outcome the device
 * accumulated during validation instead of a host-supplied one. */
#define HETM_OUTCOME_DEVICE 0xFFFFFFFFu

/* Inter-device conflict resolution of a round (§IV-E).  CPU_WINS (the
 * default): the GPU's transactions of the round abort, the host log is
 * applied and the GPU's dirty granules are restored from the host replica.
 * GPU_WINS: the host's round is discarded instead -- validation runs over
 * the whole log first and the log is applied only if it found no conflict;
 * on a conflict the GPU's transactions commit, nothing of the log is
 * applied, the watermark stays as it was, and the granules written by
 * either side are copied GPU -> host replica, which undoes the host's
 * writes there (the host must also discard the rest of its round's
 * effects, e.g. from a shadow copy). */
#define HETM_POLICY_CPU_WINS 0u
#define HETM_POLICY_GPU_WINS 1u

typedef struct hetm_ctx hetm_ctx;

typedef struct {
    uint64_t n_words;            /* N: STMR size in words, 1 <= N < 2^32         */
    uint32_t word_bytes;         /* W: 4 (OPLIST, CACHE) or 8 (TRANSFER)         */
    uint32_t granule_words;      /* G: words per bitmap bit, >= 1                */
    uint32_t lock_stripe_words;  /* S: words per lock, power of two, >= 1        */
    uint32_t max_txn_ops;        /* longest OPLIST transaction, 1..64            */
    uint64_t batch_capacity;     /* most transactions per hetm_submit_batch, 1..2^31 */
    uint64_t log_capacity;       /* most log entries per hetm_validate_apply_log,
                                    1..2^29                                      */
    uint32_t mode;               /* HETM_MODE_*                                  */
    int32_t  device;             /* HIP device ordinal                           */
    void    *stream;             /* hipStream_t for all work; NULL = the device's
                                    default (null) stream                        */
    uint32_t exec_workgroups;    /* transaction-kernel workgroups; 0 = auto      */
    uint32_t retry_cap;          /* local attempts per transaction; 0 = 1<<24    */
    uint32_t async_merge;        /* GRAPH mode only: 1 = double-buffered merge --
                                    the round gathers its dirty granules into one
                                    of two HBM staging buffers; a copy on a copy
                                    stream moves them to pinned host staging and
                                    a library thread scatters them into the host
                                    replica while the next round executes (GPU
                                    double buffering, §IV-D; costs 2*N*W bytes
                                    of HBM and of pinned host memory); 0 = the
                                    merge copy ends the round                   */
} hetm_config;

/* One host log entry (§IV-B, CPU instrumentation): the word a committed
 * host transaction updated, its new value and a timestamp that totally
 * orders the updates of that word.  W = 4 uses hetm_log_entry4 (16 bytes),
 * W = 8 uses hetm_log_entry8 (24 bytes). */
typedef struct { uint32_t word; uint32_t value; uint64_t ts; } hetm_log_entry4;
typedef struct { uint32_t word; uint32_t pad; uint64_t value; uint64_t ts; } hetm_log_entry8;

/* Batch descriptors: a host struct of device pointers, one per program.
 *
 * OPLIST: transaction i reads words idx[offsets[i] .. offsets[i+1]) in
 * order, then writes each of its first n_writes[i] words with
 * (value read + tid[i]) mod 2^32.  1 <= length <= max_txn_ops,
 * n_writes[i] <= length.  Results: uint32 per op, results[offsets[i]+j] is
 * the value read by op j.
 *
 * TRANSFER: reads accounts src[i] and dst[i]; if src != dst and the source
 * balance is >= amt[i], moves amt[i] from src to dst.  Results: int64
 * [3 * n]: results[i] = source balance read, results[n+i] = destination
 * balance read, results[2n+i] = 1 if applied else 0.
 *
 * CACHE: op[i] = 0 GET or 1 PUT of key[i] (nonzero) by tid[i].  STMR
 * layout: one 128-word record per set (N/128 sets, a power of two >= 2):
 * words 0..15 keys of ways 0..7 (u64, low word first, 0 = empty), 16..23
 * LRU stamps, 24 set PUT stamp, 32..95 values (8 words per way, word 7 a
 * checksum).  set(key) = (splitmix64-finalizer(key) mod nsets) with the low
 * bit replaced by the key's low bit.  Results: uint32 [9 * n]: status
 * (GET hit 0x100|way, GET miss 0, PUT 0x200|(0x100 if key present)|way)
 * then the 8 value words read or written.
 */
typedef struct {
    const uint32_t *offsets;   /* [n + 1] */
    const uint32_t *idx;       /* [offsets[n]] word indices < N */
    const uint8_t  *n_writes;  /* [n] */
    const uint32_t *tid;       /* [n] value added by the writes */
} hetm_oplist_desc;

typedef struct {
    const uint32_t *src;       /* [n] account indices < N */
    const uint32_t *dst;       /* [n] */
    const uint32_t *amt;       /* [n] */
} hetm_transfer_desc;

typedef struct {
    const uint64_t *key;       /* [n] nonzero */
    const uint8_t  *op;        /* [n] 0 GET, 1 PUT */
    const uint32_t *tid;       /* [n] LRU stamp / value seed */
} hetm_cache_desc;

/* ------------------------------------------------------------- lifecycle */

/* Allocates the GPU replica of the STMR (N words of W bytes), its lock table
 * (one u64 per S words: bit 63 lock, bits 0..62 version), the per-word
 * timestamp array TS (u64, zeroed; §IV-C.2; written only for rounds that
 * take several log chunks), the read-set and write-set granule bitmaps
 * (N/G bits each, §IV-B), the bucketed log and round scratch, all in HBM and
 * outside the STMR, so merges may overwrite the STMR non-transactionally
 * (§IV-B, additional assumptions).  init_image (host-or-device, N*W bytes,
 * NULL = zeros) becomes the replica.  The watermark starts at 0.
 * Errors: EINVAL (bad config), ENOMEM, EDEVICE. */
int hetm_alloc_stmr(const hetm_config *cfg, const void *init_image, hetm_ctx **out);

/* Waits for outstanding work and releases everything the context owns. */
int hetm_free(hetm_ctx *ctx);

/* ------------------------------------------------------------- the round */

/* Execution phase (§IV-C.1): runs n_txns transactions of `program` against
 * the GPU replica with the library's GPU TM (versioned lock table, local
 * conflicts only, retry until local commit) and marks the committed
 * attempts' read and written granules in the bitmaps.  descs points to the
 * program's descriptor struct (host struct, device arrays).  results
 * (device) and tickets (device, uint32 [n]) receive each transaction's
 * values and its commit ticket: ascending tickets give a serial order that
 * explains every result (gaps allowed).  For u32 words with stripe 1,
 * read-only transactions that read at the same snapshot of the version
 * clock share an even ticket (they commute; any order among them explains
 * the results); every writing transaction's ticket is odd and unique.
 * Tickets compare within one round.  Results stay speculative until the
 * round's outcome is known (§III).  Asynchronous; may be called several
 * times per round.  Errors: EINVAL, ECAPACITY (n > batch_capacity),
 * ESTATE (after validation started in this round); ERETRY latched. */
int hetm_submit_batch(hetm_ctx *ctx, uint32_t program, const void *descs, uint64_t n_txns,
                      void *results, uint32_t *tickets);

/* Validation phase (§IV-C.2) for one chunk of the host log (host-or-device,
 * n entries of the context's entry type, n <= log_capacity).  Entry k is
 * flagged iff the granule of its word is set in the read-set bitmap; flags
 * accumulate into the round outcome.  The chunk is then applied even if it
 * conflicts: word w takes the value of the chunk's entry with the largest ts
 * for w, unless an earlier chunk of the round applied an entry for w with a
 * larger ts (per-word timestamps, §IV-C.2; entries of earlier rounds are
 * older than every entry by the watermark precondition).  Checked on the
 * device before anything of the chunk is applied -- a chunk failing a
 * check applies nothing: word < N (else EINVAL); watermark < ts < 2^63
 * (else EORDER); the ts that would win a word is carried by one entry only,
 * of this chunk or of the round's earlier chunks (else EORDER); the entries
 * of one bucket of the chunk fit the resolve table (else ECAPACITY; only a
 * chunk whose words collide by the thousand in the bucketing hashes fails
 * it).
 * The latched index is the entry's position for the first two checks and
 * the word for a tie.
 * flags_bits (device, nullable, ceil(n/32) uint32) receives bit k = flag k
 * (unspecified if the chunk fails its preconditions).
 * conflict_out (host, nullable): if given, the call synchronizes and
 * stores the round outcome so far (0/1), returning any latched error. */
int hetm_validate_apply_log(hetm_ctx *ctx, const void *log, uint64_t n, uint32_t *flags_bits,
                            uint32_t *conflict_out);

/* Early validation (§IV-D), step API of a PLAIN context: validates, without
 * applying, a chunk of the host log (n entries, device memory or pinned host
 * memory, complete when the call is made: the CPU's transactions wrote it)
 * against the read-set map as it stands while batches submitted with
 * hetm_submit_batch may still be executing: it sees the marks of finished
 * batches, and those of the running one once their cache lines reach
 * device memory.  It runs on a stream of its own,
 * ordered only after the previous round's merge, so it overlaps the
 * transaction kernels.  A hit dooms the round: the CPU wins, so the running
 * transaction kernel stops at its next iteration, later batches of the round
 * execute nothing, and the round's outcome is a conflict.  Every chunk must
 * still go through hetm_validate_apply_log, which applies it; early
 * validation may miss a conflict (the read set is still growing), never
 * invent one.  Entries that fail the log's preconditions are skipped here and
 * reported by hetm_validate_apply_log.  The chunk is read until the round's
 * merge starts.
 * doomed_out (host, nullable): if given, waits for this chunk and stores 1 if
 * an early validation of the open round found a conflict.
 * Errors: EINVAL, ESTATE (a GRAPH context, whose round is one graph launch). */
int hetm_early_validate(hetm_ctx *ctx, const void *log, uint64_t n, uint32_t *doomed_out);

/* Merge phase (§IV-C.3) and round end.  conflict: 0 success, 1 conflict,
 * or HETM_OUTCOME_DEVICE.  On success the write-set granules are copied
 * GPU->host_replica, on conflict host_replica->GPU (undoing the GPU
 * transactions, CPU-wins, §IV-E); either way the replicas agree on return.
 * Contiguous dirty granules are found by a prefix sum over the write-set
 * bitmap.  host_replica: pinned host memory (hipHostMalloc), N*W bytes,
 * holding the host's state with its own writes of this round.
 * n_dirty_out (host, nullable; synchronizes), ids_out (device, nullable,
 * ceil(N/G) uint32: ascending dirty granule ids).  Then clears the
 * bitmaps and raises the watermark to the largest ts applied.
 * Errors: EINVAL, ESTATE, latched device errors when synchronizing. */
int hetm_copyback_dirty(hetm_ctx *ctx, uint32_t conflict, void *host_replica, uint64_t *n_dirty_out,
                        uint32_t *ids_out);

typedef struct {
    uint32_t    program;       /* HETM_PROG_* */
    const void *descs;         /* as hetm_submit_batch */
    uint64_t    n_txns;
    void       *results;       /* device */
    uint32_t   *tickets;       /* device */
    const void *log;           /* device (log entries resident in HBM) or host */
    uint64_t    n_log;         /* <= log_capacity */
    uint32_t   *flags_bits;    /* device, nullable */
    void       *host_replica;  /* pinned host, N*W bytes */
    uint32_t   *ids_out;       /* device, nullable */
    uint32_t    policy;        /* HETM_POLICY_* (hetm_round only) */
    uint32_t    pad_;
} hetm_round_args;

typedef struct {
    uint32_t conflict;         /* 1: GPU transactions of the round aborted      */
    int32_t  error;            /* latched device error, HETM_OK if none         */
    uint64_t n_committed;      /* transactions committed by the round           */
    uint64_t n_aborted;        /* transactions discarded by the round           */
    uint64_t n_local_retries;  /* attempts beyond the first (local conflicts)   */
    uint64_t n_dirty;          /* write-set granules merged                     */
    uint64_t n_runs;           /* maximal runs of consecutive dirty granules    */
    uint64_t max_ts;           /* watermark after the round                     */
    uint32_t merge_pending;    /* 1: the copy to the host replica is still to
                                  be issued or in flight (async_merge);
                                  hetm_sync issues it and waits for it         */
    uint32_t doomed;           /* 1: early validation found the conflict and the
                                  transaction kernels stopped short            */
    double   us_exec;          /* step times from HIP events (PLAIN mode)       */
    double   us_validate;
    double   us_merge;
    double   us_total;
    uint32_t host_discarded;   /* 1: GPU_WINS resolved a conflict against the
                                  host's round, whose log was not applied      */
    uint32_t gpu_losses;       /* rounds in a row, this one included, whose GPU
                                  transactions aborted (starvation signal)     */
    double   us_exec_kernel;   /* PLAIN: the transaction kernel alone (us_exec
                                  also covers the batch set-up kernels)        */
} hetm_round_result;

/* A whole round: execution, validation+apply, merge, reset, in the
 * context's mode.  With async_merge, a successful round returns as soon as
 * its dirty granules are staged in HBM (merge_pending = 1); their copy to
 * the host is issued once the next round's graph is queued, and the host
 * replica holds them after hetm_sync or once the round after the next
 * returns (two rounds' merges may be in flight, one per staging buffer).
 * Until then the caller must not write the host replica: the merge would
 * overwrite granules it shares with those writes.  A conflicting round
 * first waits for every earlier merge, then restores its dirty granules
 * from the host replica before returning.  PLAIN launches one kernel per
 * step and reads the outcome on the host before the merge; GRAPH replays
 * one captured hipGraph whose merge kernels read the outcome on the
 * device.  Synchronizes and
 * fills *res.  On conflict every transaction of the round is reported
 * aborted and the caller may resubmit it.  A round that latches a device
 * error (a malformed transaction or log entry, the retry cap) returns it
 * and is discarded as a conflicting round under CPU wins: its GPU
 * transactions are undone (their granules restored from the host
 * replica), its log chunk is not applied, its bitmaps and counters are
 * cleared.  The host writes of that log reach the GPU replica once a
 * corrected log carrying them is applied in a later round. */
int hetm_round(hetm_ctx *ctx, const hetm_round_args *args, hetm_round_result *res);

/* A streamed round (GRAPH mode): the round of hetm_round in three calls, so
 * that the host can keep executing while its log is shipped in chunks (the
 * CPU blocks only for the last chunks, §IV-D) and each chunk is validated
 * early against the GPU's read set while the GPU still executes (early
 * validation, §IV-D, which cuts the GPU work wasted on a round the CPU is
 * going to win).
 *
 * hetm_round_begin checks the arguments as hetm_round does, launches the
 * execution part of the round (one captured graph) and returns without
 * waiting.  args->log / n_log, if given, is the first chunk, pushed as by
 * hetm_round_push.  Errors: EINVAL, ECAPACITY, ESTATE (PLAIN context, or a
 * round already open). */
int hetm_round_begin(hetm_ctx *ctx, const hetm_round_args *args);

/* Appends n log entries (host or device memory, read until hetm_round_end
 * returns) to the open streamed round's log.  Chunks in device memory that
 * follow each other in one buffer (the first chunk, then each starting where
 * the last ended) are read in place; any other chunk, and from then on every
 * chunk of the round, is copied into the context's log buffer on a stream of
 * its own, beside the running transactions.  Under CPU wins each chunk is
 * checked at once against the read set as it stands -- without applying
 * anything.  A hit dooms the round: the CPU
 * wins, so the transaction kernel stops at its next iteration and the
 * round's outcome is a conflict.  Early validation may miss a conflict (the
 * read set is still growing) but never invents one: hetm_round_end
 * validates every pushed entry again.  The chunks of a round hold at most
 * log_capacity entries together (else ECAPACITY and nothing is appended).
 * doomed_out (host, nullable): waits for this chunk's check and stores 1 if
 * the open round is doomed.  Errors: EINVAL, ECAPACITY, ESTATE (no streamed
 * round open). */
int hetm_round_push(hetm_ctx *ctx, const void *log, uint64_t n, uint32_t *doomed_out);

/* Adds a batch to the open streamed round (the execution phase takes
 * transactions for as long as it lasts, §IV-C): its n_txns transactions run
 * after the round's earlier batches and before its tail, against the
 * replica, read set, write set and version clock as those batches left
 * them; their tickets continue the round's serial order (a round's tickets
 * order all its batches together).  They belong to the round: validated,
 * merged or rolled back with it, and reported in hetm_round_end's counts.
 * Arguments as in hetm_submit_batch: program must be the round's (that of
 * hetm_round_begin's batch, or of the first added batch if it had none);
 * descs, results and tickets are device memory, read and written until
 * hetm_round_end returns, each batch with its own results and tickets.
 * n_txns = 0 does nothing.  Errors: EINVAL (another program, a null or
 * malformed descriptor), ECAPACITY (n_txns > batch_capacity), ESTATE (no
 * streamed round open); a rejected batch leaves the round as it was. */
int hetm_round_add(hetm_ctx *ctx, uint32_t program, const void *descs, uint64_t n_txns, void *results,
                   uint32_t *tickets);

/* Ends the open streamed round: validates and applies every pushed entry as
 * one chunk (in push order: flags_bits of hetm_round_begin, if given, gets
 * bit k for the k-th pushed entry, ceil(entries pushed / 32) words), then
 * merges and finishes exactly as hetm_round, synchronizes and fills *res
 * (res->doomed = 1 if an early validation stopped the round).  Errors: as
 * hetm_round; ESTATE without an open streamed round. */
int hetm_round_end(hetm_ctx *ctx, hetm_round_result *res);

/* Queued rounds (GRAPH mode with async_merge): the rounds of hetm_round,
 * submitted up to two ahead so that the GPU starts the next round as soon
 * as one ends, without waiting for the host to take the last outcome and
 * launch again (the CPU-GPU synchronization point of §IV-C stays at the end
 * of every round; only the launch of the next round moves ahead of it).
 *
 * hetm_round_submit checks the arguments as hetm_round does and launches
 * the round behind those already queued, without waiting.  Everything
 * args points to (descriptors, results, tickets, log, flags_bits, ids_out,
 * host_replica) is read or written until the round is collected.  A round
 * submitted behind another has the same program.  Errors: EINVAL,
 * ECAPACITY; ESTATE (PLAIN mode or no async_merge, two rounds queued, a
 * streamed or step-API round open, another program behind a queued round).
 *
 * hetm_round_collect waits for the oldest queued round and handles and
 * reports it exactly as hetm_round would have (res as there; us_total is
 * the round's graph time).  The host replica rules of hetm_round apply per
 * collected round: writes the host makes for a round submitted behind
 * another must avoid the granules the round ahead may still merge -- its
 * GPU write set, and under GPU wins every granule its log wrote.  A round whose outcome needs the host before the next
 * may run -- a latched device error, or a conflict under CPU wins that the
 * undo log cannot roll back -- holds the round queued behind it, which then
 * runs empty; collect handles the held round (discard, or restore from the
 * host replica) and launches the one behind it again, so its result is
 * that of a round run after the held one.  After a device error the round
 * behind is cancelled instead: its collect returns ESTATE and it did not
 * run (resubmit it).  Errors: as hetm_round for the collected round;
 * ESTATE (nothing queued, or the round was cancelled).
 *
 * While rounds are queued, every other call that queues work or reads the
 * state (hetm_round, hetm_round_begin, the step API, hetm_serve, the state
 * reads, hetm_set_*) returns ESTATE; hetm_sync waits for the queued rounds
 * without collecting them. */
int hetm_round_submit(hetm_ctx *ctx, const hetm_round_args *args);
int hetm_round_collect(hetm_ctx *ctx, hetm_round_result *res);

/* ------------------------------------------------------------- auxiliary */

const char *hetm_strerror(int code);
const char *hetm_last_error(hetm_ctx *ctx);   /* detail of the context's last failure;
                                                 NULL: of this thread's last failed
                                                 hetm_alloc_stmr */
int hetm_sync(hetm_ctx *ctx);                 /* waits for all work, including
                                                 pending merge copies; returns a
                                                 latched error */

typedef struct {
    uint64_t rounds, rounds_conflicted, txns_committed, txns_aborted, local_retries;
    uint64_t log_entries, dirty_granules, watermark;
    uint64_t device_bytes;     /* HBM the context allocated */
    double   us_host_scatter;  /* double-buffered merge: host time scattering
                                  copied granules into the host replica       */
    double   us_merge_wait;    /* time calls spent waiting for such merges    */
    uint64_t version_resets;   /* slot layout: version-clock resets so far    */
    uint64_t rollbacks_device; /* conflicting or discarded rounds rolled back
                                  on the device from the undo log            */
    uint64_t rollbacks_host;   /* ... restored from the host replica instead
                                  (no undo log, or it ran out of room)       */
} hetm_stats;
int hetm_stats_get(hetm_ctx *ctx, hetm_stats *out);

/* Sets the number of workgroups of the transaction kernel (0 = occupancy x
 * compute units) for later batches; a captured round graph is re-captured.
 * Used by the autotuner.  Errors: EINVAL. */
int hetm_set_exec_workgroups(hetm_ctx *ctx, uint32_t workgroups);

/* Slot layout (u32 words, stripe 1): GPU transactions validate reads against
 * a version clock that persists across rounds (versions are clock values, 31
 * bits).  When a round ends with the clock past 2^30 -- checked where the
 * round's outcome reaches the host: hetm_round, or hetm_copyback_dirty with
 * n_dirty_out -- the library resets every version and the clock to 0 before
 * the next round; a writer that would run the clock out latches
 * HETM_ECAPACITY.  This call moves the
 * clock forward between rounds -- for callers that want to exercise that
 * reset.  Errors: EINVAL (backwards or past the limit), ESTATE (split
 * layout, or a round is open). */
int hetm_set_version_clock(hetm_ctx *ctx, uint32_t value);

/* Copies context state out (synchronizes).  what: 0 STMR (N*W bytes),
 * 2 read-set bitmap, 3 write-set bitmap (ceil(ceil(N/G)/32) u32 each, bit g
 * of word g/32 for granule g; the device keeps the read set as one byte per
 * granule and this call packs it), 4 lock table (ceil(N/S) u64: bit 63
 * lock, the rest version; for u32 words with S = 1 the replica keeps value,
 * version and lock of a word in one u64 -- bits 0..31 value, 32..62
 * version, 63 lock -- and this returns those words).  1 is not a state: the
 * per-word timestamps of the apply are kept only while a round takes
 * several log chunks (hetm_validate_apply_log).  dst host-or-device,
 * bytes = its size. */
#define HETM_STATE_STMR 0u
#define HETM_STATE_RS   2u
#define HETM_STATE_WS   3u
#define HETM_STATE_LOCKS 4u
int hetm_read_state(hetm_ctx *ctx, uint32_t what, void *dst, uint64_t bytes);
uint64_t hetm_state_bytes(hetm_ctx *ctx, uint32_t what);

/* The replica's values without allocating: for callers that cannot allocate
 * device memory (serving loops, harnesses that forbid hipMalloc).  Copies the
 * values of words [first_word, first_word + n_words) of the GPU replica to
 * dst (host or device, n_words * W bytes), as hetm_read_state(STMR) returns
 * them; synchronizes and waits for pending merges like it.  In the slot
 * layout (u32 words, S = 1) the values pass through an array of 2^24 u32
 * (64 MiB) of device memory that the library holds once per GPU, from the
 * first context created on it until the process ends (devices 0..63; a
 * context on a later device gets EDEVICE here); other layouts copy straight
 * from the replica.  Allocates nothing, on the device or the host.
 * n_words <= 2^24 (else ECAPACITY, nothing copied; read larger ranges in
 * pieces); the range must lie inside the replica (else EINVAL).  The array
 * is shared by every context on one GPU: calls on one GPU take turns on it
 * (a lock per device), and it keeps the last call's values, which the next
 * call overwrites before it copies anything out.  Errors: EINVAL, ECAPACITY,
 * EDEVICE, latched merge errors. */
int hetm_read_words_noalloc(hetm_ctx *ctx, uint64_t first_word, uint64_t n_words, void *dst);

/* ---------------------------------------------------------------- serving */

/* A request loop over one context (the GPU-controller thread of §IV-A):
 * OPLIST requests arrive open-loop at given times; rounds are formed from
 * the requests that have arrived, admitted in arrival order (aborted ones
 * first) while the round's device footprint -- descriptors and results
 * (8 B per op + 17 B per request), the host log chunk and the two bitmaps
 * -- fits mem_budget_bytes, at most max_batch per round.  Before each round
 * the host commits its next host_log_per_round entries of the host log
 * stream (entries in timestamp order, above the context's watermark) to
 * host_replica, and they are validated and applied in the round.
 *
 * pipelined = 1 (continuous batching; needs a GRAPH context): while a round
 * runs on the GPU the next one is packed and uploaded on an upload stream.
 * With async_merge a round's requests commit when its double-buffered merge
 * reaches the host replica, overlapping the next round's execution; the
 * host's writes of the next round go into the host replica once that merge
 * has landed, while the GPU already runs the round.  pipelined = 0: one
 * round at a time through hetm_round (a context without async_merge).
 * With round_period_us > 0 (pipelined only) a round is an execution phase
 * of that length (§IV-C): the requests that arrive while it is open join it
 * as further batches, each launched as soon as it is packed, behind the
 * round's earlier batches (hetm_round_add), while the round's footprint
 * and max_batch allow; then the round closes and is validated and merged
 * as one.  Without it a round is one batch, and arrivals wait for the next
 * round.
 *
 * A conflicting round is aborted (CPU wins, §IV-E) and its requests are
 * admitted again first.  Starvation guard (§IV-E): with starvation_limit K,
 * after K aborted rounds in a row the next round to be packed carries no
 * host writes, so it validates; the host's log waits for the round after.
 * A request's latency runs from its arrival to the commit of the round that
 * executed it successfully.  The first rounds served in a process, and the
 * first on a context, carry one-time set-up (first kernel launches, graph
 * capture, first copies of each kind), whose backlog shows in that call's
 * tail latency; a later call on the context runs without it.  All arrays
 * are host memory owned by the caller.  Errors: EINVAL, ESTATE (context
 * mode), ECAPACITY (a request larger than the budget), latched device
 * errors. */
typedef struct {
    uint64_t        n_requests;
    const double   *arrival_s;          /* [n] seconds from the start, non-decreasing */
    const uint32_t *offsets;            /* [n+1] CSR into idx */
    const uint32_t *idx;                /* [offsets[n]] word indices < N */
    const uint8_t  *n_writes;           /* [n] */
    const uint32_t *tid;                /* [n] */
    const hetm_log_entry4 *host_log;    /* [host_log_len] the host's log stream */
    uint64_t        host_log_len;
    uint64_t        host_log_per_round;
    uint64_t        max_batch;          /* <= the context's batch_capacity */
    uint64_t        mem_budget_bytes;
    uint32_t        pipelined;
    uint32_t        starvation_limit;   /* 0: off; else after this many aborted
                                           rounds in a row the host holds back
                                           its writes for one round (§IV-E) */
    uint32_t        early_validation;   /* pipelined only: 1 = streamed rounds
                                           (hetm_round_begin / push / end): the
                                           host commits a round's writes in
                                           pieces of push_entries while the GPU
                                           runs it and pushes each piece as it
                                           is committed, early-validated
                                           (§IV-D); a hit stops the round */
    uint32_t        push_entries;       /* entries per pushed piece; 0 = 3072
                                           (48 KB of 16-byte entries, §IV-D) */
    double          round_period_us;    /* pipelined only: 0 = a round is one
                                           batch; > 0 = a round stays open this
                                           long after it starts (the execution
                                           phase, §IV-C) and requests arriving
                                           meanwhile join it as further batches
                                           (hetm_round_add) while its budget
                                           allows; the round then ends at once */
} hetm_serve_spec;

typedef struct {
    uint64_t  served;                   /* requests committed */
    uint64_t  rounds;
    uint64_t  conflicted_rounds;
    uint64_t  requeued;                 /* request executions discarded by conflicts */
    double    wall_s;                   /* first arrival to last commit */
    double    throughput;               /* served / wall_s */
    double    p50_latency_us, p99_latency_us, mean_latency_us, max_latency_us;
    double   *latency_us;               /* out [n], nullable */
    uint32_t *results;                  /* out [offsets[n]], nullable: values read by the committed execution */
    uint64_t *commit_seq;               /* out [n], nullable: (round << 32) | ticket of the committed execution */
    uint8_t  *round_conflict;           /* out [max_rounds], nullable: 1 for an aborted round */
    uint64_t  max_rounds;
    uint64_t *round_log_end;            /* out [max_rounds], nullable: host log entries consumed after round r */
    /* where the serving thread's time went, microseconds: admission and
       packing, waiting for rounds (round_end), settling results, the host's
       own log commits, waiting for merges, waiting for arrivals */
    double    us_pack, us_wait_round, us_settle, us_host_commit, us_wait_merge, us_idle;
    uint64_t  starved_rounds;           /* rounds run without host writes by the starvation guard */
    uint64_t  batches;                  /* batches launched (one per round without a round period) */
} hetm_serve_report;

int hetm_serve(hetm_ctx *ctx, const hetm_serve_spec *spec, void *host_replica, hetm_serve_report *rep);

/* --------------------------------------------------- host side of a round */

/* The host's worker threads (§IV-A) running transactions on the host
 * replica and producing the round's write log: at each commit the
 * <word, value, timestamp> of every updated word is appended to a
 * thread-local log (§IV-B, CPU instrumentation); the logs are concatenated
 * at the round cut, in no particular order.  Concurrency control: two-phase
 * locking over per-stripe spinlocks (stripe = lock_stripe_words words),
 * commit timestamps from one global clock starting after ts_start, taken
 * while the locks are held, so timestamps totally order the updates of each
 * word.  host_replica (host memory, N*W bytes) is borrowed for the handle's
 * lifetime.  Errors: EINVAL, ENOMEM. */
typedef struct hetm_host_tm hetm_host_tm;
int hetm_host_tm_create(void *host_replica, uint64_t n_words, uint32_t word_bytes, uint32_t lock_stripe_words,
                        uint64_t ts_start, hetm_host_tm **out);
int hetm_host_tm_free(hetm_host_tm *tm);
uint64_t hetm_host_tm_clock(hetm_host_tm *tm);     /* last timestamp handed out */

/* n bank transfers (W = 8: move amt[i] from src[i] to dst[i] if src != dst
 * and the source balance covers it) on n_threads threads.  ts_out[i]
 * (host, n) receives transaction i's commit timestamp; log_out (host,
 * log_capacity entries) receives two entries per applied transfer;
 * *n_log_out the entry count (ECAPACITY if it exceeds log_capacity). */
int hetm_host_run_transfers(hetm_host_tm *tm, const uint32_t *src, const uint32_t *dst, const uint32_t *amt,
                            uint64_t n, uint32_t n_threads, uint64_t *ts_out, hetm_log_entry8 *log_out,
                            uint64_t log_capacity, uint64_t *n_log_out);

/* n PUTs of keys[i] (nonzero) into the CACHE layout (W = 4) with way and
 * set stamps := (uint32_t) commit timestamp; 12 log entries per PUT. */
int hetm_host_run_cache_puts(hetm_host_tm *tm, const uint64_t *keys, uint64_t n, uint32_t n_threads,
                             uint64_t *ts_out, hetm_log_entry4 *log_out, uint64_t log_capacity,
                             uint64_t *n_log_out);

#ifdef __cplusplus
}
#endif
#endif /* HETM_H */
