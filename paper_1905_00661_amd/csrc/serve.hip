// serve.hip -- the request loop of the GPU-controller thread (§IV-A): open-loop
// arrivals, admission by the round's device footprint, continuous batching
// over the double-buffered round, commit-latency accounting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include "hetm.h"
#include "hetm_ctx.h"
#include "host_pool.h"

namespace {

// Streamed serving rounds ship the host's writes in pieces of 48 KB of
// 16-byte log entries, the chunk size the paper settles on for shipping
// logs while the CPU keeps running (§IV-D).
constexpr uint64_t kServePushEntries = 48 * 1024 / sizeof(hetm_log_entry4);

using clk = std::chrono::steady_clock;

double seconds_since(clk::time_point t0) { return std::chrono::duration<double>(clk::now() - t0).count(); }

// Adds the time from its construction to its destruction to *acc (microseconds).
struct Span {
    double *acc;
    clk::time_point t = clk::now();
    explicit Span(double *a) : acc(a) {}
    ~Span() { *acc += std::chrono::duration<double, std::micro>(clk::now() - t).count(); }
};

// The requests of a round: the aborted ones it re-admits, by id, then a
// contiguous run [lo, hi) of new arrivals (whose word lists, write counts
// and ids are contiguous in the caller's arrays too).
struct ReqList {
    std::vector<uint64_t> ids;
    uint64_t lo = 0, hi = 0;
    uint64_t size() const { return ids.size() + (hi - lo); }
    bool empty() const { return size() == 0; }
    uint64_t operator[](uint64_t k) const { return k < ids.size() ? ids[k] : lo + (k - ids.size()); }
    void clear() {
        ids.clear();
        lo = hi = 0;
    }
};

// One batch of a round: its requests and where they sit in the round's
// packing area (request k0 on, operation o0 on).
struct Part {
    ReqList reqs;
    uint64_t k0 = 0, o0 = 0;
};

// One set of round buffers: pinned packing area and device copies.  A round
// packs its batches one after the other into one set.
struct RoundSet {
    uint32_t *h_off = nullptr, *h_idx = nullptr, *h_tid = nullptr;
    uint8_t *h_nw = nullptr;
    hetm_log_entry4 *h_log = nullptr;
    uint32_t *h_res = nullptr, *h_tick = nullptr;
    uint32_t *d_off = nullptr, *d_idx = nullptr, *d_tid = nullptr, *d_res = nullptr, *d_tick = nullptr;
    uint8_t *d_nw = nullptr;
    hetm_log_entry4 *d_log = nullptr;
    hipEvent_t uploaded = nullptr;
    std::vector<Part> parts;      // the round's batches in packing order
    uint64_t n_req = 0, n_ops = 0, n_log = 0;   // packed so far
    uint64_t bytes = 0;           // the round's device footprint so far
    uint64_t log_end = 0;         // host log entries consumed once this round is in
    void clear() {
        parts.clear();
        n_req = n_ops = bytes = 0;
    }
};

struct Serve {
    hetm_ctx *c;
    const hetm_serve_spec &sp;
    void *host;
    hetm_serve_report *rep;
    hipStream_t upload = nullptr;
    hipEvent_t batch_done[2] = {nullptr, nullptr};   // ends of the open round's last two batches
    RoundSet set[2];
    hetm::Pool pool;
    std::deque<uint64_t> requeue;
    uint64_t head = 0;            // next request not yet admitted
    uint64_t log_pos = 0;         // host log entries consumed
    uint64_t round_no = 0;
    uint32_t losses = 0;          // aborted rounds in a row
    bool starve_next = false;     // the next packed round carries no host writes
    uint64_t max_ops_round = 0;
    std::vector<double> latency_us;
    std::vector<uint64_t> pos_of;  // request -> first op in spec CSR
    clk::time_point t0;
    uint64_t served = 0;
    double last_commit_s = 0;
    int err = HETM_OK;

    Serve(hetm_ctx *c_, const hetm_serve_spec &s_, void *h_, hetm_serve_report *r_) : c(c_), sp(s_), host(h_), rep(r_) {}

    uint64_t req_ops(uint64_t i) const { return sp.offsets[i + 1] - sp.offsets[i]; }

    int alloc() {
        const uint64_t mb = sp.max_batch;
        max_ops_round = mb * c->cfg.max_txn_ops;
        const uint64_t nl = std::max<uint64_t>(sp.host_log_per_round, 1);
        if (hipStreamCreateWithFlags(&upload, hipStreamNonBlocking) != hipSuccess) return HETM_EDEVICE;
        for (auto &e : batch_done)
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return HETM_EDEVICE;
        pool.start();
        for (auto &r : set) {
            bool ok = hipHostMalloc((void **)&r.h_off, (mb + 1) * 4, 0) == hipSuccess &&
                      hipHostMalloc((void **)&r.h_idx, max_ops_round * 4, 0) == hipSuccess &&
                      hipHostMalloc((void **)&r.h_tid, mb * 4, 0) == hipSuccess &&
                      hipHostMalloc((void **)&r.h_nw, mb, 0) == hipSuccess &&
                      hipHostMalloc((void **)&r.h_log, nl * sizeof(hetm_log_entry4), 0) == hipSuccess &&
                      hipHostMalloc((void **)&r.h_res, max_ops_round * 4, 0) == hipSuccess &&
                      hipHostMalloc((void **)&r.h_tick, mb * 4, 0) == hipSuccess &&
                      hipMalloc((void **)&r.d_off, (mb + 1) * 4) == hipSuccess &&
                      hipMalloc((void **)&r.d_idx, max_ops_round * 4) == hipSuccess &&
                      hipMalloc((void **)&r.d_tid, mb * 4) == hipSuccess &&
                      hipMalloc((void **)&r.d_nw, mb) == hipSuccess &&
                      hipMalloc((void **)&r.d_log, nl * sizeof(hetm_log_entry4)) == hipSuccess &&
                      hipMalloc((void **)&r.d_res, max_ops_round * 4) == hipSuccess &&
                      hipMalloc((void **)&r.d_tick, mb * 4) == hipSuccess &&
                      hipEventCreateWithFlags(&r.uploaded, hipEventDisableTiming) == hipSuccess;
            if (!ok) return HETM_ENOMEM;
            // touch the host buffers now: their first writes would otherwise
            // fault page by page inside the first rounds
            memset(r.h_off, 0, (mb + 1) * 4);
            memset(r.h_idx, 0, max_ops_round * 4);
            memset(r.h_tid, 0, mb * 4);
            memset(r.h_nw, 0, mb);
            memset(r.h_log, 0, nl * sizeof(hetm_log_entry4));
            memset(r.h_res, 0, max_ops_round * 4);
            memset(r.h_tick, 0, mb * 4);
        }
        return HETM_OK;
    }
    void release() {
        if (upload) (void)hipStreamSynchronize(upload);
        for (auto &r : set) {
            for (void *p : {(void *)r.h_off, (void *)r.h_idx, (void *)r.h_tid, (void *)r.h_nw, (void *)r.h_log,
                            (void *)r.h_res, (void *)r.h_tick})
                if (p) (void)hipHostFree(p);
            for (void *p : {(void *)r.d_off, (void *)r.d_idx, (void *)r.d_tid, (void *)r.d_nw, (void *)r.d_log,
                            (void *)r.d_res, (void *)r.d_tick})
                if (p) (void)hipFree(p);
            if (r.uploaded) (void)hipEventDestroy(r.uploaded);
        }
        if (upload) (void)hipStreamDestroy(upload);
        for (auto &e : batch_done)
            if (e) (void)hipEventDestroy(e);
        pool.finish();
    }

    uint64_t arrived() const {
        const double now = seconds_since(t0);
        return (uint64_t)(std::upper_bound(sp.arrival_s, sp.arrival_s + sp.n_requests, now) - sp.arrival_s);
    }
    bool work_waiting() const { return !requeue.empty() || head < arrived(); }

    // Admission of one batch into round r: aborted requests first, then
    // arrivals in order, while the round's footprint (its log and bitmaps,
    // then each request's descriptor and results) fits the budget and its
    // packing area has room.  Returns false if nothing was admitted.
    bool admit(RoundSet &r) {
        if (r.parts.empty())
            r.bytes = sp.host_log_per_round * sizeof(hetm_log_entry4) + 2ull * ((c->args.n_bm_words) * 4ull);
        Part p;
        p.k0 = r.n_req;
        p.o0 = r.n_ops;
        uint64_t bytes = r.bytes, n_ops = r.n_ops;
        const uint64_t arr = arrived();
        auto fits = [&](uint64_t i) {
            const uint64_t b = req_ops(i) * 8 + 17;
            if (p.k0 + p.reqs.size() >= sp.max_batch || bytes + b > sp.mem_budget_bytes ||
                n_ops + req_ops(i) > max_ops_round)
                return false;
            bytes += b;
            n_ops += req_ops(i);
            p.reqs.ids.push_back(i);
            return true;
        };
        while (!requeue.empty() && fits(requeue.front())) requeue.pop_front();
        p.reqs.lo = p.reqs.hi = head;
        if (requeue.empty() && head < arr) {
            // then the arrivals [head, j) for the largest j whose footprint
            // fits (the CSR offsets are prefix sums of the operation counts,
            // and every bound grows with j: a binary search)
            const uint64_t nq = p.reqs.ids.size();
            auto ok = [&](uint64_t j) {
                const uint64_t k = j - head, ops = sp.offsets[j] - sp.offsets[head];
                return p.k0 + nq + k <= sp.max_batch && n_ops + ops <= max_ops_round &&
                       bytes + ops * 8 + k * 17 <= sp.mem_budget_bytes;
            };
            uint64_t lo = head, hi = arr;
            while (lo < hi) {
                const uint64_t mid = lo + (hi - lo + 1) / 2;
                if (ok(mid))
                    lo = mid;
                else
                    hi = mid - 1;
            }
            const uint64_t k = lo - head, ops = sp.offsets[lo] - sp.offsets[head];
            n_ops += ops;
            bytes += ops * 8 + k * 17;
            p.reqs.hi = lo;
            head = lo;
        }
        if (p.reqs.empty()) return false;
        r.n_req += p.reqs.size();
        r.n_ops = n_ops;
        r.bytes = bytes;
        r.parts.push_back(std::move(p));
        return true;
    }

    // Packs the round's last admitted batch (and, with its first batch, the
    // host's next log chunk) and uploads them.
    int pack_upload(RoundSet &r) {
        const Part &p = r.parts.back();
        const ReqList &q = p.reqs;
        const uint64_t nq = q.ids.size(), nr = q.hi - q.lo, k0 = p.k0;
        uint32_t o = (uint32_t)p.o0;
        for (size_t k = 0; k < nq; ++k) {        // re-admitted requests: a sequential prefix sum
            r.h_off[k0 + k] = o;
            o += (uint32_t)req_ops(q.ids[k]);
        }
        pool.run(nq, 2048, [&](uint64_t lo, uint64_t hi) {
            for (uint64_t k = lo; k < hi; ++k) {
                const uint64_t i = q.ids[k];
                const uint32_t *src = sp.idx + sp.offsets[i];
                uint32_t *dst = r.h_idx + r.h_off[k0 + k];
                for (uint32_t j = 0, L = (uint32_t)req_ops(i); j < L; ++j) dst[j] = src[j];
                r.h_nw[k0 + k] = sp.n_writes[i];
                r.h_tid[k0 + k] = sp.tid[i];
            }
        });
        // the run of arrivals: offsets shifted from the caller's, the rest copied as blocks
        const uint64_t base = sp.offsets[q.lo], run_ops = sp.offsets[q.hi] - base;
        const uint32_t o_run = o;
        pool.run(nr + 1, 1 << 16, [&](uint64_t lo, uint64_t hi) {
            for (uint64_t t = lo; t < hi; ++t) r.h_off[k0 + nq + t] = o_run + (uint32_t)(sp.offsets[q.lo + t] - base);
        });
        pool.run(run_ops, 1 << 18, [&](uint64_t lo, uint64_t hi) {
            memcpy(r.h_idx + o_run + lo, sp.idx + base + lo, (hi - lo) * 4);
        });
        pool.run(nr, 1 << 16, [&](uint64_t lo, uint64_t hi) {
            memcpy(r.h_nw + k0 + nq + lo, sp.n_writes + q.lo + lo, hi - lo);
            memcpy(r.h_tid + k0 + nq + lo, sp.tid + q.lo + lo, (hi - lo) * 4);
        });
        o = o_run + (uint32_t)run_ops;
        const bool first = r.parts.size() == 1;
        if (first) {
            r.n_log = std::min<uint64_t>(sp.host_log_per_round, sp.host_log_len - log_pos);
            if (starve_next) {       // the GPU lost too often: hold the host's writes back one round
                r.n_log = 0;
                starve_next = false;
                rep->starved_rounds++;
            }
            if (r.n_log) memcpy(r.h_log, sp.host_log + log_pos, r.n_log * sizeof(hetm_log_entry4));
            log_pos += r.n_log;
            r.log_end = log_pos;
        }
        const uint64_t n = q.size(), o0 = p.o0, ops = o - o0;
        bool ok = hipMemcpyAsync(r.d_off + k0, r.h_off + k0, (n + 1) * 4, hipMemcpyHostToDevice, upload) == hipSuccess &&
                  (ops == 0 || hipMemcpyAsync(r.d_idx + o0, r.h_idx + o0, ops * 4, hipMemcpyHostToDevice, upload) ==
                                   hipSuccess) &&
                  hipMemcpyAsync(r.d_nw + k0, r.h_nw + k0, n, hipMemcpyHostToDevice, upload) == hipSuccess &&
                  hipMemcpyAsync(r.d_tid + k0, r.h_tid + k0, n * 4, hipMemcpyHostToDevice, upload) == hipSuccess &&
                  (!first || r.n_log == 0 ||
                   hipMemcpyAsync(r.d_log, r.h_log, r.n_log * sizeof(hetm_log_entry4), hipMemcpyHostToDevice,
                                  upload) == hipSuccess) &&
                  hipEventRecord(r.uploaded, upload) == hipSuccess;
        return ok ? HETM_OK : HETM_EDEVICE;
    }

    // The host commits its log chunk to its replica (entries in ts order).
    void host_commit(const RoundSet &r) {
        uint32_t *H = (uint32_t *)host;
        for (uint64_t k = 0; k < r.n_log; ++k) H[r.h_log[k].word] = r.h_log[k].value;
    }

    // Streamed round: the host commits the round's writes piece by piece
    // while the GPU runs it and ships each piece once committed (pushed into
    // the round's log and early-validated against the read set as it stands).
    int host_commit_streamed(const RoundSet &r) {
        uint32_t *H = (uint32_t *)host;
        const uint64_t per = sp.push_entries ? sp.push_entries : kServePushEntries;
        for (uint64_t lo = 0; lo < r.n_log; lo += per) {
            const uint64_t hi = std::min<uint64_t>(r.n_log, lo + per);
            for (uint64_t k = lo; k < hi; ++k) H[r.h_log[k].word] = r.h_log[k].value;
            int e = hetm::stream_push(c, r.d_log + lo, hi - lo, nullptr);
            if (e) return e;
        }
        return HETM_OK;
    }

    // The descriptor of batch p of round r (offsets index the round's
    // packing area, so every batch shares its word lists and results).
    static hetm_oplist_desc part_desc(const RoundSet &r, const Part &p) {
        return {r.d_off + p.k0, r.d_idx, r.d_nw + p.k0, r.d_tid + p.k0};
    }

    hetm_round_args round_args(RoundSet &r, hetm_oplist_desc &d) {
        const Part &p = r.parts.front();
        d = part_desc(r, p);
        hetm_round_args a{};
        a.program = HETM_PROG_OPLIST;
        a.descs = &d;
        a.n_txns = p.reqs.size();
        a.results = r.d_res;
        a.tickets = r.d_tick;
        a.log = r.d_log;
        a.n_log = r.n_log;
        a.host_replica = host;
        return a;
    }

    // Queues the copies of a round's results and tickets to pinned host
    // memory behind its last batch, so they run before the round's merge
    // copy is queued (the merge copy would hold them back).
    int fetch_after_round(RoundSet &r) {
        if (!r.n_req) return HETM_OK;
        if ((r.n_ops && hipMemcpyAsync(r.h_res, r.d_res, r.n_ops * 4, hipMemcpyDeviceToHost, c->stream) != hipSuccess) ||
            hipMemcpyAsync(r.h_tick, r.d_tick, r.n_req * 4, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
            return HETM_EDEVICE;
        return HETM_OK;
    }

    // After a round's compute: conflict -> requeue; success -> copy results
    // out (unless fetch_after_round already did) and queue the requests for
    // commit stamping.
    int settle(RoundSet &r, const hetm_round_result &res, std::deque<std::pair<uint64_t, ReqList>> *pend,
               std::vector<ReqList> &done_now, bool fetched = false) {
        const uint64_t rn = round_no++;
        if (rep->round_conflict && rn < rep->max_rounds) rep->round_conflict[rn] = res.conflict ? 1 : 0;
        if (rep->round_log_end && rn < rep->max_rounds) rep->round_log_end[rn] = r.log_end;
        rep->rounds++;
        rep->batches += r.parts.size();
        losses = res.conflict ? losses + 1 : 0;
        if (sp.starvation_limit && losses >= sp.starvation_limit) {
            starve_next = true;
            losses = 0;
        }
        if (res.conflict) {
            // every batch of the round goes back, in admission order, ahead of what waits
            rep->conflicted_rounds++;
            rep->requeued += r.n_req;
            for (auto pt = r.parts.rbegin(); pt != r.parts.rend(); ++pt) {
                const ReqList &q = pt->reqs;
                for (uint64_t i = q.hi; i-- > q.lo;) requeue.push_front(i);
                for (auto it = q.ids.rbegin(); it != q.ids.rend(); ++it) requeue.push_front(*it);
            }
            return HETM_OK;
        }
        if (r.n_req && !fetched) {
            if ((r.n_ops && hipMemcpy(r.h_res, r.d_res, r.n_ops * 4, hipMemcpyDeviceToHost) != hipSuccess) ||
                hipMemcpy(r.h_tick, r.d_tick, r.n_req * 4, hipMemcpyDeviceToHost) != hipSuccess)
                return HETM_EDEVICE;
        }
        const uint64_t seq = hetm::last_merge_seq(c);
        for (const Part &p : r.parts) {
            const ReqList &q = p.reqs;
            const uint64_t n = q.size(), nq = q.ids.size(), k0 = p.k0;
            if (rep->results) {
                pool.run(nq, 2048, [&](uint64_t lo, uint64_t hi) {
                    for (uint64_t k = lo; k < hi; ++k) {
                        const uint32_t *src = r.h_res + r.h_off[k0 + k];
                        uint32_t *dst = rep->results + sp.offsets[q.ids[k]];
                        for (uint32_t j = 0, L = r.h_off[k0 + k + 1] - r.h_off[k0 + k]; j < L; ++j) dst[j] = src[j];
                    }
                });
                // the run's results are one block, in the caller's order
                const uint64_t base = sp.offsets[q.lo], run_ops = sp.offsets[q.hi] - base;
                pool.run(run_ops, 1 << 18, [&](uint64_t lo, uint64_t hi) {
                    memcpy(rep->results + base + lo, r.h_res + r.h_off[k0 + nq] + lo, (hi - lo) * 4);
                });
            }
            if (rep->commit_seq)
                pool.run(n, 1 << 14, [&](uint64_t lo, uint64_t hi) {
                    for (uint64_t k = lo; k < hi; ++k) rep->commit_seq[q[k]] = (rn << 32) | r.h_tick[k0 + k];
                });
            if (pend && seq)
                pend->emplace_back(seq, q);
            else
                done_now.push_back(q);
        }
        return HETM_OK;
    }

    void stamp(const ReqList &q) {
        const double now = seconds_since(t0);
        for (uint64_t i : q.ids) latency_us[i] = (now - sp.arrival_s[i]) * 1e6;
        pool.run(q.hi - q.lo, 1 << 15, [&](uint64_t lo, uint64_t hi) {
            for (uint64_t i = q.lo + lo; i < q.lo + hi; ++i) latency_us[i] = (now - sp.arrival_s[i]) * 1e6;
        });
        served += q.size();
        last_commit_s = now;
    }
    void stamp(const std::vector<ReqList> &qs) {
        for (const ReqList &q : qs) stamp(q);
    }

    // Sleeps until shortly before the next arrival, at most `cap` seconds.
    void wait_for_arrival(double cap = 1e30) {
        if (head < sp.n_requests) {
            const double dt = std::min(sp.arrival_s[head] - seconds_since(t0), cap);
            if (dt > 2e-4) std::this_thread::sleep_for(std::chrono::duration<double>(dt - 1e-4));
        }
    }

    int run_plain() {
        RoundSet &r = set[0];
        while (served < sp.n_requests) {
            if (!work_waiting()) {
                Span t(&rep->us_idle);
                wait_for_arrival();
                continue;
            }
            {
                Span t(&rep->us_pack);
                r.clear();
                if (!admit(r)) return HETM_ECAPACITY;    // a request larger than the budget
                if ((err = pack_upload(r))) return err;
                if (hipStreamSynchronize(upload) != hipSuccess) return HETM_EDEVICE;
            }
            {
                Span t(&rep->us_host_commit);
                host_commit(r);
            }
            hetm_oplist_desc d;
            hetm_round_args a = round_args(r, d);
            hetm_round_result res;
            {
                Span t(&rep->us_wait_round);
                if ((err = hetm_round(c, &a, &res))) return err;
            }
            Span t(&rep->us_settle);
            std::vector<ReqList> done;
            if ((err = settle(r, res, nullptr, done))) return err;
            stamp(done);
        }
        return HETM_OK;
    }

    // Pipelined rounds: the next round is packed while the current one runs
    // and starts as soon as it ends, beside its merge.  With a round period
    // the round stays open that long after it starts (the execution phase,
    // §IV-C), and requests that arrive meanwhile join it as further batches,
    // each launched as soon as it is packed, while the round's budget and
    // packing area have room; such rounds and those with early validation
    // are streamed rounds.
    int run_pipelined() {
        std::deque<std::pair<uint64_t, ReqList>> pend;   // merge job, its requests
        int cur = -1;            // set of the round on the GPU
        int nxt = -1;            // set packed and uploaded for the next round
        hetm_oplist_desc d[2];
        hetm_round_args a[2];
        const double period_s = sp.round_period_us * 1e-6;
        const bool streamed = sp.early_validation || period_s > 0;
        clk::time_point cur_start;
        bool admitting = false;  // the open round still takes batches
        uint64_t nb = 0;         // batches launched in the open round
        auto poll = [&](bool block) {
            while (!pend.empty()) {
                if (block) {
                    if (hetm::wait_merged(c, pend.front().first) != HETM_OK) return HETM_EDEVICE;
                } else if (hetm::merged_seq(c) < pend.front().first) {
                    break;
                }
                stamp(pend.front().second);
                pend.pop_front();
            }
            return HETM_OK;
        };
        while (served < sp.n_requests) {
            if (admitting) {
                const double left = period_s - std::chrono::duration<double>(clk::now() - cur_start).count();
                if (left > 0 && work_waiting()) {
                    // one batch waits behind the running one: the next is
                    // admitted once the batch before the last has finished,
                    // so it takes everything that arrived meanwhile
                    const hipError_t q = hipEventQuery(batch_done[nb & 1]);
                    if (q == hipErrorNotReady) {
                        Span t(&rep->us_idle);
                        for (int k = 0; k < 256; ++k) __builtin_ia32_pause();
                        continue;
                    }
                    if (q != hipSuccess) return HETM_EDEVICE;
                    Span t(&rep->us_pack);
                    RoundSet &r = set[cur];
                    if (!admit(r)) {            // the round is full: it ends now
                        admitting = false;
                        continue;
                    }
                    if ((err = pack_upload(r))) return err;
                    const Part &p = r.parts.back();
                    hetm_oplist_desc pd = part_desc(r, p);
                    if (hipStreamWaitEvent(c->stream, r.uploaded, 0) != hipSuccess) return HETM_EDEVICE;
                    if ((err = hetm::stream_add(c, HETM_PROG_OPLIST, &pd, p.reqs.size(), r.d_res, r.d_tick + p.k0)))
                        return err;
                    if (hipEventRecord(batch_done[nb & 1], c->stream) != hipSuccess) return HETM_EDEVICE;
                    ++nb;
                    continue;
                }
                if (left > 0 && head < sp.n_requests) {   // until the next arrival or the period's end
                    Span t(&rep->us_idle);
                    wait_for_arrival(left);
                    continue;
                }
                admitting = false;
            }
            if (nxt < 0 && work_waiting()) {
                Span t(&rep->us_pack);
                const int s = cur < 0 ? 0 : cur ^ 1;
                set[s].clear();
                if (admit(set[s])) {
                    if ((err = pack_upload(set[s]))) return err;
                    nxt = s;
                } else if (cur < 0) {
                    return HETM_ECAPACITY;      // a request larger than the budget
                }
            }
            if (cur >= 0) {
                hetm_round_result res{};
                {
                    Span t(&rep->us_wait_round);
                    if (period_s > 0 && (err = fetch_after_round(set[cur]))) return err;   // behind its last batch
                    err = streamed ? hetm::stream_end(c, &res) : hetm::round_end(c, &a[cur], &res);
                    if (err) return err;
                    // a served request completes when its round's merge lands:
                    // start the copy now rather than with the next round
                    if ((err = hetm::issue_deferred_merge(c))) return err;
                }
                Span t(&rep->us_settle);
                std::vector<ReqList> done;
                if ((err = settle(set[cur], res, &pend, done, true))) return err;
                stamp(done);
                cur = -1;
                if ((err = poll(false))) return err;
            }
            if (cur < 0 && nxt >= 0) {
                RoundSet &r = set[nxt];
                a[nxt] = round_args(r, d[nxt]);
                // round_begin orders the graph after the caller's stream
                if (hipStreamWaitEvent(c->stream, r.uploaded, 0) != hipSuccess) return HETM_EDEVICE;
                {
                    Span t(&rep->us_wait_round);
                    if (sp.early_validation) {
                        a[nxt].log = nullptr;         // shipped in pieces as the host commits them
                        a[nxt].n_log = 0;
                    }
                    err = streamed ? hetm::stream_begin(c, &a[nxt]) : hetm::round_begin(c, &a[nxt]);
                    if (err) return err;
                    cur_start = clk::now();
                    admitting = period_s > 0;
                    if (admitting) {
                        if (hipEventRecord(batch_done[0], c->stream) != hipSuccess) return HETM_EDEVICE;
                        nb = 1;
                    }
                    if (period_s == 0 && (err = fetch_after_round(r))) return err;
                }
                // the host's writes of this round go into the host replica
                // while the GPU runs it, after the last round's merge has
                // landed there (it must not overwrite them)
                {
                    Span t(&rep->us_wait_merge);
                    if ((err = hetm::wait_merged(c, hetm::last_merge_seq(c)))) return err;
                }
                {
                    Span t(&rep->us_host_commit);
                    if (sp.early_validation) {
                        if ((err = host_commit_streamed(r))) return err;
                    } else {
                        host_commit(r);
                    }
                }
                Span t(&rep->us_settle);
                if ((err = poll(false))) return err;    // the last round's merge has landed
                cur = nxt;
                nxt = -1;
            } else if (cur < 0 && nxt < 0) {
                Span t(&rep->us_idle);
                if (!pend.empty())
                    poll(true);
                else
                    wait_for_arrival();
            }
        }
        return poll(true);
    }
};

}  // namespace

extern "C" int hetm_serve(hetm_ctx *c, const hetm_serve_spec *sp, void *host_replica, hetm_serve_report *rep) {
    if (!c || !sp || !rep || !host_replica) return HETM_EINVAL;
    if (c->cfg.word_bytes != 4 || sp->max_batch == 0 || sp->max_batch > c->cfg.batch_capacity ||
        sp->host_log_per_round > c->cfg.log_capacity || (sp->n_requests && (!sp->arrival_s || !sp->offsets || !sp->idx ||
                                                                           !sp->n_writes || !sp->tid)) ||
        (sp->host_log_len && !sp->host_log))
        return HETM_EINVAL;
    if (sp->pipelined && c->cfg.mode != HETM_MODE_GRAPH) return HETM_ESTATE;
    if (c->q_n) return HETM_ESTATE;     // rounds queued by hetm_round_submit are not collected
    if (sp->early_validation && !sp->pipelined) return HETM_EINVAL;
    if (!(sp->round_period_us >= 0) || (sp->round_period_us > 0 && !sp->pipelined)) return HETM_EINVAL;
    if (!sp->pipelined && c->cfg.async_merge) return HETM_ESTATE;
    for (uint64_t i = 0; i < sp->n_requests; ++i)
        if (sp->offsets[i + 1] < sp->offsets[i] || sp->offsets[i + 1] - sp->offsets[i] > c->cfg.max_txn_ops ||
            (i && sp->arrival_s[i] < sp->arrival_s[i - 1]))
            return HETM_EINVAL;
    for (uint64_t k = 0; k < sp->host_log_len; ++k)
        if (sp->host_log[k].word >= c->cfg.n_words) return HETM_EINVAL;
    double *lat_out = rep->latency_us;
    uint32_t *res_out = rep->results;
    uint64_t *seq_out = rep->commit_seq;
    uint8_t *rc_out = rep->round_conflict;
    uint64_t *rl_out = rep->round_log_end;
    const uint64_t max_rounds = rep->max_rounds;
    memset(rep, 0, sizeof *rep);
    rep->latency_us = lat_out, rep->results = res_out, rep->commit_seq = seq_out;
    rep->round_conflict = rc_out, rep->max_rounds = max_rounds, rep->round_log_end = rl_out;

    Serve S(c, *sp, host_replica, rep);
    int rc;
    try {   // no C++ exception crosses the C ABI
        S.latency_us.assign(sp->n_requests, 0.0);
        rc = S.alloc();
        if (rc == HETM_OK) {
            S.t0 = clk::now();
            rc = sp->pipelined ? S.run_pipelined() : S.run_plain();
            if (rc == HETM_OK) rc = hetm_sync(c);
        }
    } catch (const std::bad_alloc &) {
        rc = HETM_ENOMEM;
    } catch (...) {
        rc = HETM_EDEVICE;
    }
    S.release();
    if (rc) return rc;
    rep->served = S.served;
    rep->wall_s = S.last_commit_s - (sp->n_requests ? sp->arrival_s[0] : 0.0);
    rep->throughput = rep->wall_s > 0 ? S.served / rep->wall_s : 0;
    if (sp->n_requests) {
        std::vector<double> l;
        try {
            l = S.latency_us;
        } catch (...) {
            return HETM_ENOMEM;
        }
        std::sort(l.begin(), l.end());
        auto pct = [&](double q) { return l[std::min<size_t>(l.size() - 1, (size_t)(q * (l.size() - 1) + 0.5))]; };
        rep->p50_latency_us = pct(0.50);
        rep->p99_latency_us = pct(0.99);
        rep->max_latency_us = l.back();
        double sum = 0;
        for (double x : l) sum += x;
        rep->mean_latency_us = sum / l.size();
        if (lat_out) memcpy(lat_out, S.latency_us.data(), sp->n_requests * sizeof(double));
    }
    return HETM_OK;
}
