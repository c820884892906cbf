// merge_host.h -- host half of the double-buffered merge (§IV-C.3, §IV-D).
//
// The staged granules of a committed round cross the host link as one
// runtime copy of the packed staging buffer into pinned host staging, on the
// copy stream, and a host worker thread scatters them into the host replica
// once the copy's event completes.  (The runtime runs that copy as a kernel
// of its own beside the next round's transaction kernel; copy kernels of
// this library on 8 to 256 workgroups, with plain or nontemporal stores,
// slowed the transaction kernel more.)  Jobs complete in submission order;
// each gets a sequence number.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace hetm {

struct MergeWorker;

// nullptr if the worker thread cannot be started
MergeWorker *merge_worker_create();
// Waits for every queued job, then stops the thread.
void merge_worker_destroy(MergeWorker *w);
// After `ready` completes, copies granule k of `data` (gbytes each, packed)
// to host + ids[k] * gbytes, clipped to total_bytes.  A null `ready` is a
// job whose data is in place already (host-only; nothing to wait for).
// Returns the job's sequence number (> 0), or 0 if the job could not be
// queued.
uint64_t merge_submit(MergeWorker *w, hipEvent_t ready, const uint32_t *ids, const uint8_t *data, uint64_t n,
                      uint8_t *host, uint64_t gbytes, uint64_t total_bytes);
// Blocks until job `seq` (and all before it) is done; HETM_OK or the first
// error a job met.
int merge_wait(MergeWorker *w, uint64_t seq);
// Sequence number of the last finished job.
uint64_t merge_done(MergeWorker *w);
// Host time spent scattering, and time merge_wait blocked, in microseconds.
void merge_times(MergeWorker *w, double *us_scatter, double *us_wait);

}  // namespace hetm
