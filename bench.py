"""Benchmark: whole SHeTM rounds (GPU side) on one MI355X.

Workload (the large synthetic STMR configuration): 2^28 u32 words (1 GiB),
batches of 2^20 GPU transactions (90% read-only with 16 reads, 10% update
with 4 read-modify-writes), 1% hot set drawing 50% of the accesses, a host
log of 2^20 entries per round in the host-owned half, granule 16 words.

A step is one whole round: execution of the batch, validation + apply of the
log, dirty-granule compaction, merge copy into the pinned host replica and
reset.  Inputs (descriptors, per-round logs) are resident in HBM before the
timed region.  The headline form replays the round as one captured hipGraph;
the plain form (one launch per step, host reads the outcome) is timed beside
it and provides per-kernel event timings for the roofline.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def exec_alg_bytes(batch) -> float:
    """Algorithmic bytes the execution kernel moves for a batch of u32 words
    in the slot layout (value, version and lock in one u64 per word), one
    attempt per transaction: per transaction, its list entry 4 B, offsets
    8 B, n_writes 1 B, tid 4 B, ticket 4 B; per read, index 4 B, slot 8 B,
    result 4 B, read-set byte 1 B; per read of an updating transaction, the
    revalidating slot load 8 B; per write, the CAS that locks the slot 16 B,
    the store that publishes it 8 B, the write-set bitmap word 4 B."""
    L = np.diff(batch.offsets.astype(np.int64))
    nw = batch.n_writes.astype(np.int64)
    return float(batch.n * 21 + L.sum() * 17 + L[nw > 0].sum() * 8 + nw.sum() * 28)


VALIDATE_APPLY_BYTES_PER_ENTRY = 40.0   # 16 B entry + 4 B bitmap + 8+8 B TS + 4 B value


KERNEL_SOURCES = {"k_exec_oplist": ("exec.hip", "hetm_dev.h")}
TRAFFIC_FILES = {"k_exec_oplist": "exec_oplist_large_traffic.md"}


def source_hash(kernel: str) -> str:
    """Hash of the sources a kernel is compiled from."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1905_00661_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    only if it was taken on the kernel's current sources."""
    if kernel not in TRAFFIC_FILES:
        return None
    try:
        text = open(os.path.join(PROFILES, TRAFFIC_FILES[kernel])).read()
    except OSError:
        return None
    h = re.search(r"^source_hash: (\w+)", text, re.M)
    b = re.search(r"^bytes_per_launch: (\d+)", text, re.M)
    if not h or not b or h.group(1) != source_hash(kernel):
        return None
    return int(b.group(1))


def serve_forms(args, hm, wl, torch) -> dict:
    """The serving configuration: open-loop Poisson arrivals of lognormal
    (median 4, capped at 64 ops) transactions over a 2^27-word STMR with 5%
    hot words; rounds admitted under a 2 GiB budget; continuous batching
    (pipelined) against plain per-round serving at the same rate.  Each form
    serves the stream once untimed on its context (first kernel launches,
    graph capture, first copies of the process and context), then again
    for the reported figures, its host log moved later in time so that it
    follows the first call's."""
    N = 1 << 27
    host_lo = N - N // 16
    g = wl.rng("c5", 0, 3)
    init = g.integers(0, 2 ** 32, size=N, dtype=np.uint64).astype(np.uint32)
    req = wl.c5_requests(g, args.serve_requests, args.serve_rate, n_words=N, host_lo=host_lo)
    per_round = 1 << 16
    hlog = wl.host_log_uniform(np.random.default_rng(5), 1 << 23, host_lo, N, 0, shuffle_ts=False)
    res = {"workload": f"2^27 u32 words, {args.serve_requests} requests at {args.serve_rate:g} txn/s Poisson, "
                       f"lognormal lengths (median 4, max 64), 5% hot words, host log {per_round}/round, "
                       f"budget 2 GiB, granule 64"}
    forms = (("pipelined", True, dict(mode=1, async_merge=True)),
             ("pipelined_sync_merge", True, dict(mode=1)),
             ("plain", False, dict(mode=0)))
    for name, pipelined, kw in forms:
        if args.serve_forms and name not in args.serve_forms.split(","):
            continue
        log(f"served form: {name} ...")
        ctx = hm.Context(N, 4, 64, init=init, max_ops=64, batch_capacity=1 << 20, log_capacity=per_round, **kw)
        host = hm.pinned(N * 4)
        host.numpy()[:] = init.view(np.uint8)
        ctx.serve(req["arrival_s"], req["batch"], host, hlog, per_round, 1 << 20, 2 << 30, pipelined)
        ctx.sync()
        later = hlog.copy()
        later["ts"] += np.uint64(1 << 40)
        st0 = ctx.stats()
        o = ctx.serve(req["arrival_s"], req["batch"], host, later, per_round, 1 << 20, 2 << 30, pipelined)
        st = ctx.stats()
        ctx.close()
        res[name] = {"throughput_txn_s": o["throughput"], "p50_latency_us": o["p50_latency_us"],
                     "p99_latency_us": o["p99_latency_us"], "rounds": int(o["rounds"]),
                     "conflicted_rounds": int(o["conflicted_rounds"]),
                     "host_scatter_ms": (st.us_host_scatter - st0.us_host_scatter) / 1e3,
                     "merge_wait_ms": (st.us_merge_wait - st0.us_merge_wait) / 1e3,
                     "serving_thread_ms": {k: round(o["us_" + k] / 1e3, 2) for k in
                                           ("pack", "wait_round", "settle", "host_commit", "wait_merge", "idle")}}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # a job of 50 rounds: the final drain (the last round's merge copy, part
    # of the job) weighs on the per-round figure as it would in a longer run
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--log2-words", type=int, default=28)
    ap.add_argument("--log2-txns", type=int, default=20)
    ap.add_argument("--log2-log", type=int, default=20)
    ap.add_argument("--granule", type=int, default=16)
    ap.add_argument("--p-hot", type=float, default=0.5)
    ap.add_argument("--stripe", type=int, default=1)
    ap.add_argument("--exec-wg", type=int, default=0, help="transaction-kernel workgroups (0 = occupancy x CUs)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-rate", type=float, default=3e7, help="Poisson arrival rate of the served form (txn/s)")
    ap.add_argument("--serve-requests", type=int, default=1 << 21)
    ap.add_argument("--serve-forms", default="", help="comma list of served forms to run (default: all)")
    ap.add_argument("--serve-only", action="store_true", help="run only the served forms")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calibrate", action="store_true",
                    help="first run a plain 1 GiB device copy, the known-size reference for HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs a round on one GPU; there is no multi-GPU path, so --gpus must be 1"}))
        sys.exit(2)

    import torch

    from paper_1905_00661_amd import hetm as hm
    from paper_1905_00661_amd import workloads as wl

    if args.serve_only:
        print(json.dumps({"served": serve_forms(args, hm, wl, torch)}), flush=True)
        return

    N, n_txn, n_log = 1 << args.log2_words, 1 << args.log2_txns, 1 << args.log2_log
    G = args.granule
    t0 = time.time()
    ri = wl.c2(n_words=N, n_txn=n_txn, n_log=n_log, p_hot=args.p_hot, granule=G)
    log(f"inputs generated in {time.time() - t0:.1f}s")
    dev = "cuda:0"
    torch.cuda.set_device(0)
    if args.calibrate:
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        a.fill_(1)
        big = torch.empty(1 << 30, dtype=torch.uint8, device=dev)   # evicts `a` from the caches
        big.fill_(2)
        del big
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    rounds = args.warmup + args.steps

    # per-round logs resident in HBM: same words/values, timestamps shifted
    base_log = hm.to_device(ri.log, dev)
    logs = []
    for r in range(rounds + 1):
        t = base_log.clone()
        ts = t.view(torch.int64).view(-1, 2)[:, 1]
        ts.add_(r * n_log)
        logs.append(t)
    torch.cuda.synchronize()

    host = hm.pinned(N * 4)
    host.numpy()[:] = ri.init.view(np.uint8)

    def run(mode: int, k_steps: int, warm: int, async_merge: bool = False):
        ctx = hm.Context(N, 4, G, init=ri.init, stripe=args.stripe, max_ops=16, batch_capacity=n_txn,
                         log_capacity=n_log, mode=mode, exec_workgroups=args.exec_wg, async_merge=async_merge)
        b = hm.Batch(hm.HETM_PROG_OPLIST, ri.batch, dev)
        flags = torch.zeros(((n_log + 31) // 32) * 4, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        res = []
        for r in range(warm):
            ctx.round(b, logs[r], n_log, host, flags)
        torch.cuda.synchronize()
        lat = []
        t_start = time.perf_counter()
        for r in range(warm, warm + k_steps):
            t1 = time.perf_counter()
            rr = ctx.round(b, logs[r], n_log, host, flags)
            lat.append(time.perf_counter() - t1)
            res.append(rr.as_dict())
        ctx.sync()                       # the last round's merge copy has landed
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        tickets = b.tickets_np().copy()
        st = ctx.stats()
        ctx.close()
        run.scatter_ms = st.us_host_scatter / 1e3 / (warm + k_steps)
        return elapsed, lat, res, tickets

    log("batched form (graph + double-buffered merge) ...")
    el_g, lat_g, res_g, tickets = run(hm.HETM_MODE_GRAPH, args.steps, args.warmup, async_merge=True)
    committed = sum(r["n_committed"] for r in res_g)
    value = committed / el_g
    out = {
        "metric": "committed txns/s + validate/apply GB/s vs HBM peak; p50/p99 commit latency",
        "value": value, "unit": "txn/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * el_g / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"large synthetic STMR: 2^{args.log2_words} u32 words, 2^{args.log2_txns} txns/batch "
                               f"(90% RO x16 reads, 10% 4RMW), hot 1% at p={args.p_hot}, host log "
                               f"2^{args.log2_log}, granule {G}, lock stripe {args.stripe}",
                   "form": "batched: hipGraph round, persistent transaction kernel, double-buffered merge"},
        "p50_round_ms": 1e3 * float(np.percentile(lat_g, 50)),
        "p99_round_ms": 1e3 * float(np.percentile(lat_g, 99)),
        "conflict_rounds": sum(r["conflict"] for r in res_g),
        "local_retries_per_round": float(np.mean([r["n_local_retries"] for r in res_g])),
        "dirty_granules_per_round": float(np.mean([r["n_dirty"] for r in res_g])),
        "graph_us": float(np.mean([r["us_total"] for r in res_g])),
        "host_scatter_ms_per_round": run.scatter_ms,
    }
    log("graph form, merge inside the round ...")
    el_s, lat_s, res_s, _ = run(hm.HETM_MODE_GRAPH, args.steps, args.warmup)
    out["graph_sync_merge"] = {"value": sum(r["n_committed"] for r in res_s) / el_s,
                               "ms_per_step": 1e3 * el_s / args.steps}

    if not args.no_plain:
        log("plain form ...")
        el_p, lat_p, res_p, _ = run(hm.HETM_MODE_PLAIN, args.steps, args.warmup)
        us = {k: float(np.mean([r[k] for r in res_p]))
              for k in ("us_exec", "us_exec_kernel", "us_validate", "us_merge", "us_total")}
        out["plain"] = {"value": sum(r["n_committed"] for r in res_p) / el_p, "ms_per_step": 1e3 * el_p / args.steps,
                        "p50_round_ms": 1e3 * float(np.percentile(lat_p, 50)),
                        "p99_round_ms": 1e3 * float(np.percentile(lat_p, 99)), **us}
        out["batched_vs_plain"] = value / out["plain"]["value"]
        va_bytes = VALIDATE_APPLY_BYTES_PER_ENTRY * n_log
        out["validate_apply"] = {"achieved_GBps": va_bytes / (us["us_validate"] * 1e-6) / 1e9,
                                 "frac_of_hbm_peak": va_bytes / (us["us_validate"] * 1e-6) / 1e9 / HBM_PEAK_GBPS,
                                 "bytes_per_entry": VALIDATE_APPLY_BYTES_PER_ENTRY}
        # the transaction kernel alone (events on its stream just before and
        # after it); us_exec also covers the batch set-up kernels
        steps_us = {"exec": us["us_exec_kernel"], "validate_apply": us["us_validate"], "merge": us["us_merge"]}
        dominant = max(steps_us, key=steps_us.get)
        if dominant == "exec":
            alg = exec_alg_bytes(ri.batch)
            kern = "k_exec_oplist"
        elif dominant == "validate_apply":
            alg = va_bytes
            kern = "k_validate+k_apply"
        else:
            alg = 2.0 * out["dirty_granules_per_round"] * G * 4
            kern = "k_compact+k_copy"
        ach = alg / (steps_us[dominant] * 1e-6) / 1e9
        out["roofline"] = {"bound": "hbm", "kernel": kern, "achieved": ach, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                           "frac": ach / HBM_PEAK_GBPS, "traffic": load_traffic(kern),
                           "alg_bytes_per_launch": alg, "avg_launch_us": steps_us[dominant]}

    if not args.no_serve:
        out["served"] = serve_forms(args, hm, wl, torch)

    if not args.no_cpu:
        import oracle as orc
        log("cpu baseline (oracle, whole rounds for ~10 s) ...")
        order = orc.order_from_tickets(tickets, even_ties=True)
        el_c, n_rounds, committed = 0.0, 0, 0
        while el_c < 10.0 and n_rounds < 40:
            S, H = ri.init.copy(), ri.init.copy()
            TS = np.zeros(N, np.uint64)
            t1 = time.perf_counter()
            o = orc.round_oplist(S, H, TS, G, ri.batch, order, ri.log, 0)
            el_c += time.perf_counter() - t1
            n_rounds += 1
            committed += 0 if o["conflict"] else ri.batch.n
            del S, H, TS
        out["cpu_baseline"] = {"value": committed / el_c, "unit": "txn/s", "cores": 1, "kind": "oracle",
                               "sample": f"{n_rounds} whole rounds of the same workload ({ri.batch.n} txns, {n_log} "
                                         f"log entries each, replayed in the GPU's commit order) by the "
                                         f"single-threaded C oracle: {el_c:.1f} s"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
