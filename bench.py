"""Benchmark: whole SHeTM rounds (GPU side) on one MI355X.

Headline (`value`): the large synthetic STMR configuration -- 2^28 u32 words
(1 GiB), batches of 2^20 GPU transactions (90% read-only with 16 reads, 10%
update with 4 read-modify-writes), 1% hot set drawing 50% of the accesses, a
host log of 2^20 entries per round in the host-owned half, granule 16 words
-- in the queued batched form (one captured hipGraph per round, each round
submitted while the one before runs and collected after it, persistent
transaction kernel, double-buffered merge), with each round's inputs
(descriptors, log) resident in HBM when the timed region starts.  A step is
one whole round: execution, validation + apply of the log, dirty-granule
compaction, merge into the pinned host replica, reset.

Beside it, on the same GPU:
  batched_per_call          the same rounds one hetm_round call at a time;
  graph_sync_merge / plain  the same rounds with the merge inside the round,
                            and one launch per step (per-step event timings);
  ingest                    the batched rounds with every round's descriptors
                            and log uploaded from pinned host memory and its
                            results and tickets fetched back, overlapped on
                            two copy streams (the host-link-inclusive rate);
  small                     round latency of the plain single round (2^16
                            words, 4096 4R/4W transactions, 10,000-entry log,
                            granule 64) and of its partitioned variant;
  conflict                  the large rounds with one log entry redirected
                            into the batch's read set in 1% and 10% of the
                            rounds;
  early                     early validation on and off over a sweep of
                            conflicting-round fractions (streamed rounds);
  bank / cache              the bank-transfer and object-cache
                            configurations at full size (retries per commit);
  served                    the request loop swept over arrival rates, for the
                            pipelined form, the pipelined form with early
                            validation or a round period, and one round at
                            a time;
  cpu_baseline              the C oracle replaying whole large rounds on one
                            pinned host core;
  sweep (not by default)    the large rounds over granules 16..4096 and hot
                            fractions 0, 0.5, 0.9.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
METRIC = "committed txns/s + validate/apply GB/s vs HBM peak; p50/p99 commit latency"


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


def exec_scope_bytes(batch) -> float:
    """The same work counted with the scope table's per-transaction figures
    for a lock table of one u64 per word: a 16-read read-only transaction
    452 B, a 4-read-modify-write update 228 B."""
    nw = batch.n_writes.astype(np.int64)
    return float((nw == 0).sum() * 452 + (nw > 0).sum() * 228)


# validate + apply, bytes per log entry: the scope table's algorithmic count
# (16 B entry, 4 B bitmap word, 8 + 8 B timestamp read and write, 4 B value)
# and the bytes the bucketed passes stream (bin reads the entry and a
# read-set byte and writes the entry into its bucket; resolve reads it and
# writes the winner; apply reads the winner and stores its 8-byte slot)
VALIDATE_APPLY_BYTES_PER_ENTRY = 40.0
VALIDATE_APPLY_STREAM_BYTES_PER_ENTRY = 16 + 1 + 16 + 32 + 16 + 8


KERNEL_SOURCES = {"k_exec_oplist": ("exec.hip", "hetm_dev.h"),
                  "validate_apply": ("log_apply.hip", "hetm_dev.h")}
TRAFFIC_FILES = {"k_exec_oplist": "exec_oplist_large_traffic.md",
                 "validate_apply": "round_kernels_large_traffic.md"}


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


def cpu_info() -> dict:
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "model": model}


def device_info(torch) -> dict:
    """What the runtime reports about the GPU the figures come from."""
    p = torch.cuda.get_device_properties(0)
    return {"name": p.name, "arch": getattr(p, "gcnArchName", None), "compute_units": p.multi_processor_count,
            "memory_GiB": round(p.total_memory / 2 ** 30, 1),
            "l2_MiB_per_xcd": round(getattr(p, "L2_cache_size", 0) / 2 ** 20, 1) or None}


def pct(a, q):
    return float(np.percentile(np.asarray(a), q)) if len(a) else None


# ------------------------------------------------------------------- legs

def shifted_logs(torch, hm, base_log: np.ndarray, n_log: int, rounds: int, dev: str, inject=None):
    """Per-round logs resident in HBM: the same words and values, timestamps
    shifted past the previous round's; inject(r, copy) may return an edited
    copy (copy() makes one) of round r's log, else None."""
    base = hm.to_device(base_log, dev)
    logs = []
    for r in range(rounds):
        lr = inject(r, base_log.copy) if inject is not None else None
        t = hm.to_device(lr, dev) if lr is not None else base.clone()
        t.view(torch.int64).view(-1, 2)[:, 1].add_(r * n_log)
        logs.append(t)
    torch.cuda.synchronize()
    return logs


def tune_exec(args, hm, torch, ri, dev) -> dict:
    """Chooses the transaction kernel's workgroup count for the large
    configuration by timing whole batched rounds at a few widths, cached by
    workload signature (outside every timed region)."""
    from paper_1905_00661_amd import autotune
    N, G, n_log = ri.n_words, ri.granule, ri.log.shape[0]
    workload = {"program": "oplist", "n_words": N, "word_bytes": 4, "granule": G, "stripe": args.stripe,
                "n_txns": ri.batch.n, "n_log": n_log, "p_hot": args.p_hot, "ops": "16 reads | 4 rmw",
                "form": "graph, double-buffered merge"}
    sig = autotune.signature(workload, torch.cuda.get_device_name(0), autotune.library_hash())
    cache = autotune.TuneCache(args.tune_cache)
    if cache.get(sig) is not None:
        hit = cache.get(sig)
        return {**hit, "cached": True, "signature": sig}
    ctx = hm.Context(N, 4, G, init=ri.init, stripe=args.stripe, max_ops=16, batch_capacity=ri.batch.n,
                     log_capacity=n_log, mode=hm.HETM_MODE_GRAPH, async_merge=True)
    b = hm.Batch(hm.HETM_PROG_OPLIST, ri.batch, dev)
    host = hm.pinned(N * 4)
    host.numpy()[:] = ri.init.view(np.uint8)
    base = hm.to_device(ri.log, dev)
    log_t = base.clone()
    shift = [0]

    def run_round():
        log_t.copy_(base)
        log_t.view(torch.int64).view(-1, 2)[:, 1].add_(shift[0])   # timestamps past the last round's
        shift[0] += n_log
        ctx.round(b, log_t, n_log, host)

    def sync():
        ctx.sync()
        torch.cuda.synchronize()

    cus = torch.cuda.get_device_properties(0).multi_processor_count
    res = autotune.tune_exec_workgroups(ctx.set_exec_workgroups, run_round, cus, sig=sig, cache=cache, sync=sync)
    ctx.close()
    return {**res, "signature": sig}


def large_forms(args, hm, wl, torch, ri, dev) -> dict:
    """The large configuration in the batched, graph-with-merge and plain forms,
    inputs resident in HBM."""
    N, G, n_log = ri.n_words, ri.granule, ri.log.shape[0]
    n_txn = ri.batch.n
    rounds = args.warmup + args.steps
    logs = shifted_logs(torch, hm, ri.log, n_log, rounds + 1, dev)
    host = hm.pinned(N * 4)
    host.numpy()[:] = ri.init.view(np.uint8)

    def run(mode: int, async_merge: bool = False, queued: bool = False):
        ctx = hm.Context(N, 4, G, init=ri.init, stripe=args.stripe, max_ops=16, batch_capacity=n_txn,
                         log_capacity=n_log, mode=mode, exec_workgroups=args.exec_wg, async_merge=async_merge)
        b = hm.Batch(hm.HETM_PROG_OPLIST, ri.batch, dev)
        flags = torch.zeros(((n_log + 31) // 32) * 4, dtype=torch.uint8, device=dev)
        # every round's argument and result records are built before the
        # timed region; the loop only calls hetm_round
        argv = [ctx._round_args(b, logs[r], n_log, host, flags, None, hm.HETM_POLICY_CPU_WINS) for r in range(rounds)]
        outs = [hm.hetm_round_result() for _ in range(rounds)]
        pa = [ctypes.byref(x) for x in argv]
        po = [ctypes.byref(x) for x in outs]
        call, handle = hm.lib().hetm_round, ctx.ctx
        sub, col = hm.lib().hetm_round_submit, hm.lib().hetm_round_collect

        def check(rc, what):
            if rc:
                raise RuntimeError(f"{what} failed: {hm.lib().hetm_last_error(handle)}")

        def queued_rounds(first, last, lat):
            # round r is submitted while round r - 1 runs, then r - 1 is
            # collected; lat: the time between successive collects
            t_prev = time.perf_counter()
            for r in range(first, last):
                check(sub(handle, pa[r]), "hetm_round_submit")
                if r > first:
                    check(col(handle, po[r - 1]), "hetm_round_collect")
                    t = time.perf_counter()
                    lat.append(t - t_prev)
                    t_prev = t
            if last > first:
                check(col(handle, po[last - 1]), "hetm_round_collect")
                lat.append(time.perf_counter() - t_prev)

        torch.cuda.synchronize()
        if queued:
            queued_rounds(0, args.warmup, [])
        else:
            for r in range(args.warmup):
                check(call(handle, pa[r], po[r]), "hetm_round")
        ctx.sync()
        torch.cuda.synchronize()
        lat = []
        t_start = time.perf_counter()
        if queued:
            queued_rounds(args.warmup, rounds, lat)
        else:
            for r in range(args.warmup, rounds):
                t1 = time.perf_counter()
                check(call(handle, pa[r], po[r]), "hetm_round")
                lat.append(time.perf_counter() - t1)
        ctx.sync()                       # the last round's merge copy has landed
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        res = [o.as_dict() for o in outs[args.warmup:]]
        tickets = b.tickets_np().copy()
        st = ctx.stats()
        ctx.close()
        return {"elapsed": elapsed, "lat": lat, "res": res, "tickets": tickets,
                "scatter_ms": st.us_host_scatter / 1e3 / rounds}

    def summary(g):
        return {"value": sum(r["n_committed"] for r in g["res"]) / g["elapsed"],
                "ms_per_step": 1e3 * g["elapsed"] / args.steps,
                "p50_round_ms": 1e3 * pct(g["lat"], 50), "p99_round_ms": 1e3 * pct(g["lat"], 99),
                "conflict_rounds": sum(r["conflict"] for r in g["res"]),
                "local_retries_per_round": float(np.mean([r["n_local_retries"] for r in g["res"]])),
                "dirty_granules_per_round": float(np.mean([r["n_dirty"] for r in g["res"]])),
                "graph_us": float(np.mean([r["us_total"] for r in g["res"]])),
                "host_scatter_ms_per_round": g["scatter_ms"]}

    out = {}
    log("large: queued form (batched rounds submitted one ahead) ...")
    g = run(hm.HETM_MODE_GRAPH, async_merge=True, queued=True)
    out["queued"] = summary(g)
    out["tickets"] = g["tickets"]
    log("large: batched form (graph + double-buffered merge), one round per call ...")
    out["batched"] = summary(run(hm.HETM_MODE_GRAPH, async_merge=True))
    log("large: graph form, merge inside the round ...")
    s = run(hm.HETM_MODE_GRAPH)
    out["graph_sync_merge"] = {"value": sum(r["n_committed"] for r in s["res"]) / s["elapsed"],
                               "ms_per_step": 1e3 * s["elapsed"] / args.steps}
    log("large: plain form ...")
    p = run(hm.HETM_MODE_PLAIN)
    us = {k: float(np.mean([r[k] for r in p["res"]]))
          for k in ("us_exec", "us_exec_kernel", "us_validate", "us_merge", "us_total")}
    out["plain"] = {"value": sum(r["n_committed"] for r in p["res"]) / p["elapsed"],
                    "ms_per_step": 1e3 * p["elapsed"] / args.steps,
                    "p50_round_ms": 1e3 * pct(p["lat"], 50), "p99_round_ms": 1e3 * pct(p["lat"], 99), **us}
    return out


def ingest_form(args, hm, wl, torch, ri, dev) -> dict:
    """Batched rounds whose inputs start in pinned host memory: round r+1's
    descriptors and log go up on one copy stream while round r runs, round
    r's results and tickets come back on another while round r+1 runs."""
    N, G, n_log = ri.n_words, ri.granule, ri.log.shape[0]
    bt = ri.batch
    rounds = args.warmup + args.steps
    arrays = [bt.offsets, bt.idx, bt.n_writes, bt.tid]
    h_desc = []
    for a in arrays:
        t = hm.pinned(a.nbytes)
        t.numpy()[:] = np.ascontiguousarray(a).view(np.uint8).reshape(-1)
        h_desc.append(t)
    h_logs = []
    for r in range(rounds):
        t = hm.pinned(ri.log.nbytes)
        lr = ri.log.copy()
        lr["ts"] += np.uint64(r * n_log)
        t.numpy()[:] = lr.view(np.uint8)
        h_logs.append(t)
    n_res = int(bt.offsets[-1])
    h_res = hm.pinned(n_res * 4)
    h_tick = hm.pinned(bt.n * 4)
    sets = []
    for _ in range(2):
        d = [torch.empty(t.numel(), dtype=torch.uint8, device=dev) for t in h_desc]
        sets.append({"desc": hm.hetm_oplist_desc(*[x.data_ptr() for x in d]), "bufs": d,
                     "log": torch.empty(ri.log.nbytes, dtype=torch.uint8, device=dev),
                     "res": torch.empty(n_res * 4, dtype=torch.uint8, device=dev),
                     "tick": torch.empty(bt.n * 4, dtype=torch.uint8, device=dev)})

    class DevBatch:                         # the binding's Batch interface over one buffer set
        def __init__(self, st):
            self.program, self.n, self.desc = hm.HETM_PROG_OPLIST, bt.n, st["desc"]
            self.results, self.tickets = st["res"], st["tick"]

    host = hm.pinned(N * 4)
    host.numpy()[:] = ri.init.view(np.uint8)
    ctx = hm.Context(N, 4, G, init=ri.init, stripe=args.stripe, max_ops=16, batch_capacity=bt.n,
                     log_capacity=n_log, mode=hm.HETM_MODE_GRAPH, exec_workgroups=args.exec_wg, async_merge=True)
    main = torch.cuda.current_stream()
    up, down = torch.cuda.Stream(), torch.cuda.Stream()
    ev_up = [torch.cuda.Event() for _ in range(2)]
    ev_done = [torch.cuda.Event() for _ in range(2)]
    ev_fetched = [torch.cuda.Event() for _ in range(2)]

    def upload(r):
        st = sets[r % 2]
        with torch.cuda.stream(up):
            up.wait_event(ev_fetched[r % 2])          # round r-2's results have left this set
            for d, h in zip(st["bufs"], h_desc):
                d.copy_(h, non_blocking=True)
            st["log"].copy_(h_logs[r], non_blocking=True)
            ev_up[r % 2].record(up)

    def fetch(r):
        st = sets[r % 2]
        with torch.cuda.stream(down):
            down.wait_event(ev_done[r % 2])
            h_res.copy_(st["res"], non_blocking=True)
            h_tick.copy_(st["tick"], non_blocking=True)
            ev_fetched[r % 2].record(down)

    torch.cuda.synchronize()
    upload(0)
    t_start, res = None, []
    for r in range(rounds):
        if r == args.warmup:
            ctx.sync()
            torch.cuda.synchronize()
            t_start = time.perf_counter()
        if r + 1 < rounds:
            upload(r + 1)
        main.wait_event(ev_up[r % 2])
        rr = ctx.round(DevBatch(sets[r % 2]), sets[r % 2]["log"], n_log, host)
        ev_done[r % 2].record(main)
        fetch(r)
        if r >= args.warmup:
            res.append(rr.as_dict())
    ctx.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ctx.close()
    committed = sum(r["n_committed"] for r in res)
    h2d = sum(a.nbytes for a in arrays) + ri.log.nbytes
    d2h = n_res * 4 + bt.n * 4
    return {"value": committed / elapsed, "unit": "txn/s", "ms_per_step": 1e3 * elapsed / args.steps,
            "h2d_MB_per_round": h2d / 1e6, "d2h_MB_per_round": d2h / 1e6,
            "merge_d2h_MB_per_round": float(np.mean([r["n_dirty"] for r in res])) * G * 4 / 1e6,
            "form": "batched rounds, descriptors and log uploaded from pinned host memory and results fetched, "
                    "overlapped on two copy streams"}


def small_round(args, hm, wl, torch, dev) -> dict:
    """Latency of the plain single round (2^16 words, 4096 4R/4W, 10,000
    entries, granule 64) and of its partitioned variant, per form."""
    out = {}
    for variant in ("", "p"):
        ri = wl.c1(variant)
        n_log = ri.log.shape[0]
        rounds = 20 + args.small_rounds
        logs = shifted_logs(torch, hm, ri.log, n_log, rounds, dev)
        res_v = {}
        for name, mode in (("plain", hm.HETM_MODE_PLAIN), ("graph", hm.HETM_MODE_GRAPH)):
            ctx = hm.Context(ri.n_words, 4, ri.granule, init=ri.init, max_ops=4, batch_capacity=ri.batch.n,
                             log_capacity=n_log, mode=mode)
            host = hm.pinned(ri.n_words * 4)
            host.numpy()[:] = ri.init.view(np.uint8)
            b = hm.Batch(hm.HETM_PROG_OPLIST, ri.batch, dev)
            torch.cuda.synchronize()
            lat, conf, steps = [], 0, []
            for r in range(rounds):
                t1 = time.perf_counter()
                rr = ctx.round(b, logs[r], n_log, host)
                if r >= 20:
                    lat.append(1e6 * (time.perf_counter() - t1))
                    conf += rr.conflict
                    steps.append(rr.as_dict())
            ctx.close()
            res_v[name] = {"p50_us": pct(lat, 50), "p99_us": pct(lat, 99), "conflict_rounds": conf}
            if mode == hm.HETM_MODE_PLAIN:   # per step, from the round's HIP events
                res_v[name]["p50_step_us"] = {k[3:]: pct([x[k] for x in steps], 50)
                                              for k in ("us_exec", "us_validate", "us_merge")}
        out["as_named" if variant == "" else "partitioned"] = res_v
    out["workload"] = ("2^16 u32 words, 4096 txns of 4 reads + 4 writes, 10,000-entry host log, granule 64 "
                       "(as named every granule is read, so every round conflicts; partitioned: GPU lower half, "
                       "log upper half)")
    out["rounds"] = args.small_rounds
    return out


def conflict_form(args, hm, wl, torch, ri, dev, rate: float = 0.1) -> dict:
    """Batched large rounds where, in a seeded fraction `rate` of the rounds,
    one log entry is redirected to a word the batch reads (CPU wins: the
    round's GPU transactions abort and the device rolls them back)."""
    N, G, n_log = ri.n_words, ri.granule, ri.log.shape[0]
    steps = max(args.steps, min(500, int(math.ceil(5 / rate))))   # about five conflicting rounds at least
    rounds = args.warmup + steps
    g = np.random.default_rng(0x190500661)
    hits = set(int(r) for r in np.flatnonzero(g.random(rounds) < rate))

    def inject(r, copy):
        if r not in hits:
            return None
        lr = copy()
        lr["word"][int(g.integers(0, n_log))] = ri.batch.idx[int(g.integers(0, ri.batch.idx.shape[0]))]
        return lr

    logs = shifted_logs(torch, hm, ri.log, n_log, rounds, dev, inject=inject)
    host = hm.pinned(N * 4)
    host.numpy()[:] = ri.init.view(np.uint8)
    ctx = hm.Context(N, 4, G, init=ri.init, stripe=args.stripe, max_ops=16, batch_capacity=ri.batch.n,
                     log_capacity=n_log, mode=hm.HETM_MODE_GRAPH, exec_workgroups=args.exec_wg, async_merge=True)
    b = hm.Batch(hm.HETM_PROG_OPLIST, ri.batch, dev)
    for r in range(args.warmup):
        ctx.round(b, logs[r], n_log, host)
    ctx.sync()
    torch.cuda.synchronize()
    lat_ok, lat_cf, committed = [], [], 0
    t0 = time.perf_counter()
    for r in range(args.warmup, rounds):
        t1 = time.perf_counter()
        rr = ctx.round(b, logs[r], n_log, host)
        (lat_cf if rr.conflict else lat_ok).append(1e3 * (time.perf_counter() - t1))
        committed += rr.n_committed
    ctx.sync()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ctx.close()
    return {"value": committed / el, "unit": "txn/s", "rounds": steps, "conflict_rounds": len(lat_cf),
            "p50_clean_round_ms": pct(lat_ok, 50), "p50_conflict_round_ms": pct(lat_cf, 50),
            "max_conflict_round_ms": max(lat_cf) if lat_cf else None,
            "form": f"batched, CPU wins, r = {rate:.0%} of rounds conflicting"}


def sweep_form(args, hm, wl, torch, dev) -> dict:
    """The large configuration over granules G in {16, 64, 256, 1024, 4096}
    and hot fractions {0, 0.5, 0.9}: batched rounds (GRAPH, double-buffered
    merge), 5 untimed and args.sweep_rounds timed per point, inputs in HBM."""
    N, n_txn, n_log = 1 << args.log2_words, 1 << args.log2_txns, 1 << args.log2_log
    pts = []
    for p_hot in (0.0, 0.5, 0.9):
        for G in (16, 64, 256, 1024, 4096):
            ri = wl.c2(n_words=N, n_txn=n_txn, n_log=n_log, p_hot=p_hot, granule=G)
            rounds = 5 + args.sweep_rounds
            logs = shifted_logs(torch, hm, ri.log, n_log, rounds, dev)
            host = hm.pinned(N * 4)
            host.numpy()[:] = ri.init.view(np.uint8)
            ctx = hm.Context(N, 4, G, init=ri.init, stripe=args.stripe, max_ops=16, batch_capacity=n_txn,
                             log_capacity=n_log, mode=hm.HETM_MODE_GRAPH, exec_workgroups=args.exec_wg,
                             async_merge=True)
            b = hm.Batch(hm.HETM_PROG_OPLIST, ri.batch, dev)
            for r in range(5):
                ctx.round(b, logs[r], n_log, host)
            ctx.sync()
            torch.cuda.synchronize()
            res = []
            t0 = time.perf_counter()
            for r in range(5, rounds):
                res.append(ctx.round(b, logs[r], n_log, host).as_dict())
            ctx.sync()
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            ctx.close()
            dirty = float(np.mean([x["n_dirty"] for x in res]))
            pts.append({"granule": G, "p_hot": p_hot, "ms_per_round": 1e3 * el / args.sweep_rounds,
                        "txn_per_s": sum(x["n_committed"] for x in res) / el, "dirty_granules": dirty,
                        "merge_MB_per_round": dirty * G * 4 / 1e6,
                        "retries_per_round": float(np.mean([x["n_local_retries"] for x in res]))})
            log(f"sweep G={G} p_hot={p_hot}: {pts[-1]['ms_per_round']:.3f} ms/round, "
                f"{pts[-1]['merge_MB_per_round']:.1f} MB merged")
            del logs, host
    return {"form": "batched (GRAPH, double-buffered merge), inputs in HBM", "rounds_per_point": args.sweep_rounds,
            "points": pts}


def early_form(args, hm, wl, torch, ri, dev) -> dict:
    """Early validation on and off (§IV-D; the contention sweep of §V-C):
    batched large rounds in which a given fraction of the rounds carries one
    log entry on a word the batch reads.  Off: hetm_round validates the log
    after execution.  On: a streamed round whose log is pushed in 16 chunks
    paced over the execution (a host producing its log as it runs), each
    chunk early-validated; a hit stops the transaction kernel."""
    N, G, n_log = ri.n_words, ri.granule, ri.log.shape[0]
    rounds = args.early_rounds
    n_chunks = 16
    per = (n_log + n_chunks - 1) // n_chunks
    eb = ri.log.dtype.itemsize
    b_idx = ri.batch.idx
    out = {"form": "batched (GRAPH, double-buffered merge), CPU wins; on: log pushed in 16 chunks paced over "
                   "the clean round's execution time, each early-validated",
           "rounds_per_point": rounds, "points": []}
    ctx = hm.Context(N, 4, G, init=ri.init, stripe=args.stripe, max_ops=16, batch_capacity=ri.batch.n,
                     log_capacity=n_log, mode=hm.HETM_MODE_GRAPH, exec_workgroups=args.exec_wg, async_merge=True)
    b = hm.Batch(hm.HETM_PROG_OPLIST, ri.batch, dev)
    host = hm.pinned(N * 4)
    host.numpy()[:] = ri.init.view(np.uint8)
    shift = [0]

    def logs_for(frac, seed):
        g = np.random.default_rng(seed)
        hits = g.random(rounds) < frac

        def inject(r, copy):
            if not hits[r]:
                return None
            lr = copy()
            lr["word"][int(g.integers(0, n_log))] = b_idx[int(g.integers(0, b_idx.shape[0]))]
            return lr
        ls = shifted_logs(torch, hm, ri.log, n_log, rounds, dev, inject=inject)
        for t in ls:
            t.view(torch.int64).view(-1, 2)[:, 1].add_(shift[0])
        shift[0] += rounds * n_log
        torch.cuda.synchronize()
        return ls

    # warm both forms up and time the clean round's execution for the pacing
    for t in logs_for(0.0, 1)[:3]:
        ctx.round(b, t, n_log, host)
    warm = logs_for(0.0, 2)
    for t in warm[:3]:
        ctx.round_begin(b, host)
        for k in range(n_chunks):
            lo = k * per
            ctx.round_push(t[lo * eb:min(lo + per, n_log) * eb], min(per, n_log - lo))
        ctx.round_end()
    ctx.sync()
    pace_s = 0.8 * 1e-3 * args.early_exec_ms / n_chunks
    for frac in args.early_fracs:
        point = {"conflict_fraction": frac}
        for mode in ("off", "on"):
            ls = logs_for(frac, 1000 + int(frac * 100))
            st0 = ctx.stats()
            ctx.sync()
            torch.cuda.synchronize()
            lat_ok, lat_cf, committed, doomed = [], [], 0, 0
            t0 = time.perf_counter()
            for t in ls:
                t1 = time.perf_counter()
                if mode == "off":
                    rr = ctx.round(b, t, n_log, host)
                else:
                    ctx.round_begin(b, host)
                    for k in range(n_chunks):
                        lo = k * per
                        ctx.round_push(t[lo * eb:min(lo + per, n_log) * eb], min(per, n_log - lo))
                        t_next = t1 + (k + 1) * pace_s
                        while time.perf_counter() < t_next:
                            pass
                    rr = ctx.round_end()
                (lat_cf if rr.conflict else lat_ok).append(1e3 * (time.perf_counter() - t1))
                committed += rr.n_committed
                doomed += rr.doomed
            ctx.sync()
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            st1 = ctx.stats()
            n_cf = len(lat_cf)
            point[mode] = {"txn_per_s": committed / el, "ms_per_round": 1e3 * el / rounds,
                           "conflict_rounds": n_cf, "doomed_rounds": doomed,
                           "mean_clean_round_ms": float(np.mean(lat_ok)) if lat_ok else None,
                           "mean_conflict_round_ms": float(np.mean(lat_cf)) if lat_cf else None,
                           "txns_run_per_conflict_round": (st1.txns_aborted - st0.txns_aborted) / n_cf if n_cf else None}
        out["points"].append(point)
        log(f"early validation, conflict fraction {frac}: off {point['off']['ms_per_round']:.3f} ms/round, "
            f"on {point['on']['ms_per_round']:.3f} ms/round")
    ctx.close()
    out["batch_txns"] = ri.batch.n
    return out


# Algorithmic bytes per committed transaction of the bank and cache
# programs: the descriptor, the words the transaction must read and write,
# its results and ticket (no lock or map traffic).  TRANSFER: src, dst, amt
# (12) + two balances read (16) and written (16) + three results (24) +
# ticket (4).  CACHE: key, op, tid (13) + the set's 8 keys (64) + 9 result
# words (36) + ticket (4), and a GET's 8-word value read (32) or a PUT's
# key, value and stamps written (48).
TRANSFER_BYTES = 12 + 16 + 16 + 24 + 4
CACHE_BYTES = 13 + 64 + 36 + 4
CACHE_GET_BYTES, CACHE_PUT_BYTES = 32, 48


def small_roofline(bytes_per_s: float) -> dict:
    gbps = bytes_per_s / 1e9
    return {"bound": "hot-object serialization (chains run one transaction per lane step)",
            "alg_GBps": gbps, "peak_GBps": HBM_PEAK_GBPS, "frac": gbps / HBM_PEAK_GBPS}


def bank_form(args, hm, wl, torch, dev) -> dict:
    """Bank transfers at full size: 2^24 int64 accounts, U[2^20, 2^21]
    Zipf(0.9) transfers per round on the GPU, the host TM's 2^15 transfers
    on its 2^16 accounts per round producing the log."""
    n_acc, host_acc = 1 << 24, 1 << 16
    init = np.full(n_acc, 1000, dtype=np.int64)
    host = hm.pinned(n_acc * 8)
    hv = host.numpy().view(np.int64)
    hv[:] = init
    ctx = hm.Context(n_acc, 8, 64, init=init, max_ops=2, batch_capacity=1 << 21, log_capacity=1 << 16,
                     mode=hm.HETM_MODE_GRAPH, async_merge=True)
    tm = hm.HostTM(hv, ts_start=0)
    rows = []
    for r in range(args.bank_rounds):
        d = wl.c3(round_no=r)
        t1 = time.perf_counter()
        ts, hlog = tm.transfers(d["host"].src, d["host"].dst, d["host"].amt, threads=8)
        host_s = time.perf_counter() - t1
        b = hm.Batch(hm.HETM_PROG_TRANSFER, d["batch"], dev)
        log_t = hm.to_device(hlog, dev) if hlog.shape[0] else torch.zeros(24, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rr = ctx.round(b, log_t, hlog.shape[0], host)
        ctx.sync()
        el = time.perf_counter() - t1
        rows.append({"n": d["batch"].n, "s": el, "committed": rr.n_committed, "retries": rr.n_local_retries,
                     "conflict": rr.conflict, "host_s": host_s, "host_n": d["host"].n})
        log(f"bank round {r}: {d['batch'].n} transfers in {1e3 * el:.1f} ms, retries {rr.n_local_retries}")
    tm.close()
    total = float(ctx.read_state(hm.HETM_STATE_STMR).sum())
    ctx.close()
    timed = rows[1:] if len(rows) > 1 else rows
    committed = sum(x["committed"] for x in timed)
    rate = committed / sum(x["s"] for x in timed)
    return {"value": rate, "unit": "txn/s",
            "roofline": {**small_roofline(rate * TRANSFER_BYTES), "alg_bytes_per_txn": TRANSFER_BYTES},
            "ms_per_round": 1e3 * float(np.mean([x["s"] for x in timed])),
            "transfers_per_round": float(np.mean([x["n"] for x in timed])),
            "retries_per_commit": sum(x["retries"] for x in timed) / max(committed, 1),
            "conflict_rounds": sum(x["conflict"] for x in rows),
            "host_tm_txn_s": sum(x["host_n"] for x in rows) / sum(x["host_s"] for x in rows),
            "balance_conserved": total == 1000.0 * n_acc, "rounds_timed": len(timed),
            "workload": "2^24 int64 accounts = 1000, U[2^20, 2^21] Zipf(0.9) transfers per round, host TM "
                        "2^15 transfers on 2^16 accounts (8 threads), granule 64, first round untimed"}


def cache_form(args, hm, wl, torch, dev) -> dict:
    """The object cache at full size: 2^22 sets x 8 ways warmed to 95% by
    host PUTs, 2^20 GPU requests per round (95% GET / 5% PUT, Zipf 0.99 over
    2^26 keys, even keys), 2^14 host PUTs on odd keys per round."""
    nsets = 1 << 22
    N = nsets * 128
    g0 = wl.rng("c4", 0, 2)
    host = hm.pinned(N * 4)
    hv = host.numpy().view(np.uint32)
    hv[:] = 0
    tm = hm.HostTM(hv, stripe=128)
    keys = g0.permutation(np.arange(1, (1 << 26) + 1, dtype=np.uint64))[: int(nsets * 8 * 0.95)]
    t1 = time.perf_counter()
    for k0 in range(0, keys.shape[0], 1 << 21):
        tm.cache_puts(keys[k0:k0 + (1 << 21)], threads=8)
    warm_s = time.perf_counter() - t1
    log(f"cache: table warmed in {warm_s:.1f} s")
    ctx = hm.Context(N, 4, 128, init=hv.copy(), max_ops=2, batch_capacity=1 << 20, log_capacity=12 << 14,
                     mode=hm.HETM_MODE_GRAPH, async_merge=True)
    rows = []
    for r in range(args.cache_rounds):
        b = wl.c4_requests(g0, 1 << 20, 1 << 26, theta=0.99, put_frac=0.05, parity=0, tid0=(r + 1) << 24)
        hk = wl.c4_requests(g0, 1 << 14, 1 << 26, theta=0.99, put_frac=1.0, parity=1).key
        _, hlog = tm.cache_puts(hk, threads=8)
        bb = hm.Batch(hm.HETM_PROG_CACHE, b, dev)
        log_t = hm.to_device(hlog, dev)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rr = ctx.round(bb, log_t, hlog.shape[0], host)
        ctx.sync()
        el = time.perf_counter() - t1
        n_put = int((b.op == wl.CACHE_PUT).sum())
        rows.append({"s": el, "committed": rr.n_committed, "retries": rr.n_local_retries, "conflict": rr.conflict,
                     "bytes": rr.n_committed * CACHE_BYTES + (b.n - n_put) * CACHE_GET_BYTES + n_put * CACHE_PUT_BYTES})
        log(f"cache round {r}: {1e3 * el:.1f} ms, retries {rr.n_local_retries}")
    tm.close()
    ctx.close()
    timed = rows[1:] if len(rows) > 1 else rows
    committed = sum(x["committed"] for x in timed)
    secs = sum(x["s"] for x in timed)
    return {"value": committed / secs, "unit": "txn/s",
            "roofline": {**small_roofline(sum(x["bytes"] for x in timed) / secs),
                         "alg_bytes_per_txn": sum(x["bytes"] for x in timed) / max(committed, 1)},
            "ms_per_round": 1e3 * float(np.mean([x["s"] for x in timed])),
            "retries_per_commit": sum(x["retries"] for x in timed) / max(committed, 1),
            "conflict_rounds": sum(x["conflict"] for x in rows), "warmup_s": warm_s, "rounds_timed": len(timed),
            "host_tm_puts_s": keys.shape[0] / warm_s, "host_tm_threads": 8,
            "workload": "2^22 sets x 8 ways (2 GiB) warmed to 95%, 2^20 requests per round (95% GET / 5% PUT, "
                        "Zipf 0.99 over 2^26 keys, even keys), 2^14 host PUTs on odd keys, granule 128, "
                        "first round untimed"}


def serve_sweep(args, hm, wl, torch) -> dict:
    """The serving configuration swept over arrival rates: open-loop Poisson
    arrivals of lognormal (median 4, capped at 64 ops) transactions over a
    2^27-word STMR with 5% hot words; rounds admitted under a 2 GiB budget;
    the pipelined form (continuous batching, double-buffered merge), the same
    with streamed rounds whose host writes are shipped in 48 KB pieces and
    validated early, the same with a round period (requests that arrive
    while a round is open join it as further batches), and one round at a
    time.  Each form serves a warm-up
    stream first on its context; every call's host log follows the previous
    call's."""
    N = 1 << 27
    host_lo = N - N // 16
    g = wl.rng("c5", 0, 3)
    init = g.integers(0, 2 ** 32, size=N, dtype=np.uint64).astype(np.uint32)
    per_round = 1 << 16
    hlog = wl.host_log_uniform(np.random.default_rng(5), 1 << 23, host_lo, N, 0, shuffle_ts=False)
    rates = [float(x) for x in args.serve_rates.split(",")]
    bound_ms = args.serve_p99_bound_ms
    out = {"workload": f"2^27 u32 words, Poisson arrivals, lognormal lengths (median 4, max 64), 5% hot words, "
                       f"host log {per_round}/round, budget 2 GiB, granule 64; requests per point: rate x "
                       f"{args.serve_seconds} s (at least 2^17, at most 2^23)",
           "p99_bound_ms": bound_ms, "points": {}}
    period = args.serve_period_us
    out["round_period_us"] = period
    forms = (("pipelined", True, dict(mode=1, async_merge=True), False, 0.0),
             ("pipelined_early", True, dict(mode=1, async_merge=True), True, 0.0),
             ("pipelined_period", True, dict(mode=1, async_merge=True), False, period),
             ("plain", False, dict(mode=0), False, 0.0))
    call = [0]

    def serve(ctx, host, req, pipelined, early, period_us):
        call[0] += 1
        later = hlog.copy()
        later["ts"] += np.uint64(call[0] << 40)
        return ctx.serve(req["arrival_s"], req["batch"], host, later, per_round, 1 << 20, 2 << 30, pipelined,
                         early_validation=early, round_period_us=period_us)

    for name, pipelined, kw, early, period_us in forms:
        ctx = hm.Context(N, 4, 64, init=init, max_ops=64, batch_capacity=1 << 20, log_capacity=per_round, **kw)
        host = hm.pinned(N * 4)
        host.numpy()[:] = init.view(np.uint8)
        warm = wl.c5_requests(g, 1 << 17, 1e7, n_words=N, host_lo=host_lo)
        serve(ctx, host, warm, pipelined, early, period_us)
        ctx.sync()
        pts = {}
        for rate in rates:
            n = int(min(max(rate * args.serve_seconds, 1 << 17), 1 << 23))
            req = wl.c5_requests(g, n, rate, n_words=N, host_lo=host_lo)
            log(f"served {name}: {n} requests at {rate:g}/s ...")
            o = serve(ctx, host, req, pipelined, early, period_us)
            ctx.sync()
            pts[f"{rate:g}"] = {"offered_txn_s": rate, "throughput_txn_s": o["throughput"],
                                "p50_latency_us": o["p50_latency_us"], "p99_latency_us": o["p99_latency_us"],
                                "rounds": int(o["rounds"]), "batches": int(o["batches"]), "requests": n,
                                "serving_thread_ms": {k: round(o["us_" + k] / 1e3, 2) for k in
                                                      ("pack", "wait_round", "settle", "host_commit", "wait_merge",
                                                       "idle")}}
        ctx.close()
        ok = [p for p in pts.values() if p["p99_latency_us"] <= bound_ms * 1e3]
        out["points"][name] = pts
        out[f"{name}_best_txn_s_within_p99_bound"] = max((p["throughput_txn_s"] for p in ok), default=None)
    return out


def cpu_baseline(args, orc, ri, tickets) -> dict:
    """The C oracle replaying whole large rounds (in the GPU's commit order)
    on one host core for about 10 s."""
    info = cpu_info()
    keep = os.sched_getaffinity(0)
    core = max(keep)
    os.sched_setaffinity(0, {core})
    try:
        order = orc.order_from_tickets(tickets, even_ties=True)
        el, n_rounds, committed = 0.0, 0, 0
        N, G = ri.n_words, ri.granule
        while el < args.cpu_seconds and n_rounds < 40:
            S, H = ri.init.copy(), ri.init.copy()
            TS = np.zeros(N, np.uint64)
            t1 = time.perf_counter()
            o = orc.round_oplist(S, H, TS, G, ri.batch, order, ri.log, 0)
            el += time.perf_counter() - t1
            n_rounds += 1
            committed += 0 if o["conflict"] else ri.batch.n
            del S, H, TS
    finally:
        os.sched_setaffinity(0, keep)
    return {"value": committed / el, "unit": "txn/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_rounds} whole rounds of the large configuration ({ri.batch.n} txns, {ri.log.shape[0]} log "
                      f"entries each, replayed in the GPU's commit order) by the single-threaded C oracle pinned to "
                      f"core {core}: {el:.1f} s",
            "host": info}


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
    ap.add_argument("--exec-wg", type=int, default=0, help="transaction-kernel workgroups (0 = one per CU)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the workgroup tuner (one workgroup per CU unless --exec-wg is given)")
    ap.add_argument("--tune-cache", default=os.path.join(os.path.expanduser("~"), ".cache", "hetm", "tuned.json"),
                    help="JSON file of tuned workgroup counts by workload signature")
    ap.add_argument("--legs", default="ingest,small,conflict,early,bank,cache,served,cpu",
                    help="comma list of legs beside the headline (ingest, small, conflict, early, bank, cache, "
                         "served, cpu; also sweep, not run by default)")
    ap.add_argument("--sweep-rounds", type=int, default=20)
    ap.add_argument("--early-rounds", type=int, default=20)
    ap.add_argument("--early-fracs", type=lambda v: [float(x) for x in v.split(",")], default="0,0.25,0.5,1",
                    help="fractions of conflicting rounds swept by the early-validation leg")
    ap.add_argument("--early-exec-ms", type=float, default=0.6,
                    help="execution time over which the early-validation leg paces its pushes")
    ap.add_argument("--small-rounds", type=int, default=200)
    ap.add_argument("--bank-rounds", type=int, default=3)
    ap.add_argument("--cache-rounds", type=int, default=3)
    ap.add_argument("--conflict-rates", default="0.01,0.1",
                    help="fractions of rounds with an injected inter-device conflict (conflict leg)")
    ap.add_argument("--serve-rates", default="1e6,1e7,3e7,1e8,2e8,3e8")
    ap.add_argument("--serve-seconds", type=float, default=0.25)
    ap.add_argument("--serve-p99-bound-ms", type=float, default=5.0)
    ap.add_argument("--serve-period-us", type=float, default=500.0,
                    help="round period of the served form that admits arrivals into the running round")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--calibrate", action="store_true",
                    help="first run a plain 1 GiB device copy, the known-size reference for HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs a round on one GPU; there is no multi-GPU path, so --gpus must be 1"}))
        sys.exit(2)
    legs = set(x for x in args.legs.split(",") if x)

    import torch

    from paper_1905_00661_amd import hetm as hm
    from paper_1905_00661_amd import workloads as wl

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

    tuned = None
    if args.exec_wg == 0 and not args.no_tune:
        log("tuning the transaction kernel's workgroups ...")
        tuned = tune_exec(args, hm, torch, ri, dev)
        args.exec_wg = int(tuned["exec_workgroups"])
        log(f"  {args.exec_wg} workgroups ({'cached' if tuned['cached'] else 'measured'})")
    large = large_forms(args, hm, wl, torch, ri, dev)
    bat, plain = large["queued"], large["plain"]
    out = {
        "metric": METRIC, "value": bat["value"], "unit": "txn/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": bat["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "device": device_info(torch),
        "config": {"workload": f"large synthetic STMR: 2^{args.log2_words} u32 words, 2^{args.log2_txns} txns/batch "
                               f"(90% RO x16 reads, 10% 4RMW), hot 1% at p={args.p_hot}, host log "
                               f"2^{args.log2_log}, granule {G}, lock stripe {args.stripe}",
                   "form": "batched and queued: hipGraph rounds submitted one round ahead (hetm_round_submit / "
                           "hetm_round_collect), persistent transaction kernel, double-buffered merge; inputs "
                           "resident in HBM"},
        **{k: v for k, v in bat.items() if k not in ("value", "ms_per_step")},
        "batched_per_call": large["batched"], "graph_sync_merge": large["graph_sync_merge"], "plain": plain,
        "autotune": ({"signature": tuned["signature"], "exec_workgroups": tuned["exec_workgroups"],
                      "cached": tuned["cached"],
                      "table_ms": {str(r["exec_workgroups"]): round(1e3 * r["median_s"], 4) for r in tuned["table"]}}
                     if tuned else {"exec_workgroups": args.exec_wg, "tuned": False}),
        "batched_vs_plain": bat["value"] / plain["value"],
    }
    va = n_log * VALIDATE_APPLY_BYTES_PER_ENTRY / (plain["us_validate"] * 1e-6) / 1e9
    vs = n_log * VALIDATE_APPLY_STREAM_BYTES_PER_ENTRY / (plain["us_validate"] * 1e-6) / 1e9
    out["validate_apply"] = {"us_per_chunk": plain["us_validate"], "entries": n_log,
                             "alg_GBps": va, "alg_frac_of_hbm_peak": va / HBM_PEAK_GBPS,
                             "alg_bytes_per_entry": VALIDATE_APPLY_BYTES_PER_ENTRY,
                             "streamed_GBps": vs, "streamed_frac_of_hbm_peak": vs / HBM_PEAK_GBPS,
                             "streamed_bytes_per_entry": VALIDATE_APPLY_STREAM_BYTES_PER_ENTRY}
    vt = load_traffic("validate_apply") if n_log == 1 << 20 else None
    out["validate_apply"]["counter_bytes_per_chunk"] = vt
    out["validate_apply"]["counter_frac_of_hbm_peak"] = (
        vt / (plain["us_validate"] * 1e-6) / 1e9 / HBM_PEAK_GBPS if vt else None)
    # roofline of the dominant kernel: the transaction kernel, timed alone by
    # events on its stream just before and after it in the plain form
    alg = exec_alg_bytes(ri.batch)
    ach = alg / (plain["us_exec_kernel"] * 1e-6) / 1e9
    scope = exec_scope_bytes(ri.batch)
    out["roofline"] = {"bound": "hbm", "kernel": "k_exec_oplist", "achieved": ach, "peak": HBM_PEAK_GBPS,
                       "unit": "GB/s", "frac": ach / HBM_PEAK_GBPS, "traffic": load_traffic("k_exec_oplist"),
                       "alg_bytes_per_launch": alg, "avg_launch_us": plain["us_exec_kernel"],
                       "scope_bytes_per_launch": scope,
                       "scope_frac": scope / (plain["us_exec_kernel"] * 1e-6) / 1e9 / HBM_PEAK_GBPS}

    if "ingest" in legs:
        log("ingest: inputs from pinned host memory, results fetched ...")
        out["ingest"] = ingest_form(args, hm, wl, torch, ri, dev)
    if "small" in legs:
        log("small round latency ...")
        out["small"] = small_round(args, hm, wl, torch, dev)
    if "conflict" in legs:
        log("conflicting rounds ...")
        by_rate = {}
        for rate in [float(x) for x in args.conflict_rates.split(",")]:
            log(f"conflicting rounds at r = {rate:g} ...")
            by_rate[f"{rate:g}"] = conflict_form(args, hm, wl, torch, ri, dev, rate)
        out["conflict"] = {**by_rate.get("0.1", next(iter(by_rate.values()))), "by_rate": by_rate}
    if "sweep" in legs:
        log("granule and hot-fraction sweep ...")
        out["sweep"] = sweep_form(args, hm, wl, torch, dev)
    if "early" in legs:
        log("early validation on and off ...")
        out["early"] = early_form(args, hm, wl, torch, ri, dev)
    if "bank" in legs:
        log("bank transfers ...")
        out["bank"] = bank_form(args, hm, wl, torch, dev)
    if "cache" in legs:
        log("object cache ...")
        out["cache"] = cache_form(args, hm, wl, torch, dev)
    if "served" in legs:
        out["served"] = serve_sweep(args, hm, wl, torch)
    tickets = large.pop("tickets")
    if "cpu" in legs:
        import oracle as orc
        log("cpu baseline (oracle, whole rounds for ~10 s, one pinned core) ...")
        out["cpu_baseline"] = cpu_baseline(args, orc, ri, tickets)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
