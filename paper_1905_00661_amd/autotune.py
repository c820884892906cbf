"""Autotuner for the SHeTM round on one GPU.

Picks, by measurement on a sample of the caller's workload, the three knobs
of the round that trade off against each other:

* workgroups of the transaction kernel -- more lanes hide more memory
  latency but overlap more transactions (more local aborts, more cache
  turnover between a transaction's first read and its revalidation);
* lock stripe S -- smaller lock tables, more false local conflicts;
* granule G -- larger granules shrink the bitmaps and their atomics but
  copy more bytes over the host link at merge time and raise false
  inter-device conflicts.

Each (G, S) pair gets its own scratch context (they are allocation-time
parameters); workgroup counts are swept on that context with
``hetm_set_exec_workgroups``.  The score is committed transactions per
second of whole double-buffered rounds.  Results are cached by a workload
signature in a JSON file next to this module.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np

from . import hetm as hm

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_configs.json")


def signature(n_words: int, word_bytes: int, program: int, batch, n_log: int) -> str:
    L = np.diff(batch.offsets.astype(np.int64)) if hasattr(batch, "offsets") else np.zeros(1)
    nw = batch.n_writes if hasattr(batch, "n_writes") else np.zeros(1)
    key = (n_words, word_bytes, program, batch.n, n_log, int(L.sum()), int(np.asarray(nw).sum()))
    return hashlib.sha256(repr(key).encode()).hexdigest()[:16]


def load(sig: str) -> dict | None:
    try:
        return json.load(open(CACHE)).get(sig)
    except (OSError, ValueError):
        return None


def _store(sig: str, entry: dict) -> None:
    try:
        d = json.load(open(CACHE))
    except (OSError, ValueError):
        d = {}
    d[sig] = entry
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def tune(init: np.ndarray, program: int, batch, log: np.ndarray, granules=(16, 64), stripes=(1, 2),
         workgroups=(256, 384, 512, 768, 1024, 2048), rounds: int = 3, max_ops: int = 16,
         store: bool = True, verbose: bool = False) -> dict:
    """Times `rounds` whole rounds for every candidate and returns the best
    configuration with the full table.  `log` is one round's host log; each
    timed round re-applies it with timestamps shifted past the previous."""
    import torch
    N, W = init.shape[0], init.itemsize
    n_log = log.shape[0]
    sig = signature(N, W, program, batch, n_log)
    dev = "cuda:0"
    host = hm.pinned(N * W)
    host.numpy()[:] = init.view(np.uint8)
    base = hm.to_device(log, dev)
    ts_col = 1 if W == 4 else 2
    table = []
    for G in granules:
        for S in stripes:
            ctx = hm.Context(N, W, G, init=init, stripe=S, max_ops=max_ops, batch_capacity=batch.n,
                             log_capacity=max(n_log, 1), mode=hm.HETM_MODE_GRAPH, async_merge=True)
            b = hm.Batch(program, batch, dev)
            shift = 0
            for wg in workgroups:
                ctx.set_exec_workgroups(wg)
                times, committed, retries = [], 0, 0
                for r in range(rounds + 1):
                    lg = base.clone()
                    lg.view(torch.int64).view(-1, ts_col + 1)[:, ts_col].add_(shift)
                    shift += n_log
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    res = ctx.round(b, lg, n_log, host)
                    ctx.sync()
                    if r:                      # the first round warms up (graph capture)
                        times.append(time.perf_counter() - t0)
                        committed += res.n_committed
                        retries += res.n_local_retries
                row = {"granule": G, "stripe": S, "workgroups": wg, "round_ms": 1e3 * float(np.mean(times)),
                       "txn_per_s": committed / float(np.sum(times)), "retries_per_round": retries / rounds}
                table.append(row)
                if verbose:
                    print(row, flush=True)
            ctx.close()
    best = max(table, key=lambda r: r["txn_per_s"])
    entry = {"best": best, "table": table}
    if store:
        _store(sig, entry)
    return entry
