"""Helpers for the GPU parity tests: run a round through libhetm (the C ABI
via the ctypes binding) and the same round through the CPU oracle, on the
same seeded inputs, in the GPU's recorded commit order."""
from __future__ import annotations

import sys

import numpy as np

import oracle as orc
from paper_1905_00661_amd import hetm as hm
from paper_1905_00661_amd import workloads as wl


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def bits(bm: np.ndarray, n: int) -> np.ndarray:
    return np.unpackbits(bm.view(np.uint8), bitorder="little")[:n].astype(bool)


def gpu_round(ri: wl.RoundInputs, mode=hm.HETM_MODE_PLAIN, stripe=1, host=None, ctx=None, exec_workgroups=0,
              flags=True, ids=True, keep=False, async_merge=False, policy=hm.HETM_POLICY_CPU_WINS):
    """One whole round (hetm_round) on the GPU.  Returns a dict of numpy
    results and the context (if keep)."""
    import torch
    program = ri.program
    if ctx is None:
        ctx = hm.Context(ri.n_words, ri.word_bytes, ri.granule, init=ri.init, stripe=stripe,
                         batch_capacity=max(ri.batch.n, 1), log_capacity=max(ri.log.shape[0], 1),
                         mode=mode, exec_workgroups=exec_workgroups, async_merge=async_merge)
    H0 = wl.host_replica(ri.init, ri.log) if host is None else host
    host_t = hm.pinned(H0.nbytes)
    host_t.numpy()[:] = H0.view(np.uint8)
    b = hm.Batch(program, ri.batch, ctx.dev)
    n_log = ri.log.shape[0]
    log_t = hm.to_device(ri.log, ctx.dev) if n_log else torch.zeros(16, dtype=torch.uint8, device=ctx.dev)
    flags_t = torch.zeros(max((n_log + 31) // 32, 1) * 4, dtype=torch.uint8, device=ctx.dev) if flags else None
    ids_t = torch.zeros(max(ctx.n_granules, 1) * 4, dtype=torch.uint8, device=ctx.dev) if ids else None
    torch.cuda.synchronize()
    res = ctx.round(b if ri.batch.n else None, log_t, n_log, host_t, flags_t, ids_t, policy=policy)
    ctx.sync()     # the merge copy of a double-buffered round may still be in flight
    out = {
        "res": res,
        "results": b.results_np(),
        "tickets": b.tickets_np(),
        "S": ctx.read_state(hm.HETM_STATE_STMR).copy(),
        "H": host_t.numpy().view(ri.init.dtype).copy(),
        "flags": hm.tensor_to_numpy(flags_t, np.uint32) if flags else None,
        "ids": hm.tensor_to_numpy(ids_t, np.uint32, int(res.n_dirty)) if ids else None,
        "H0": H0,
    }
    if keep:
        out["ctx"] = ctx
    else:
        ctx.close()
    return out


REPLAY = {wl.PROG_OPLIST: orc.replay_oplist, wl.PROG_TRANSFER: orc.replay_transfer, wl.PROG_CACHE: orc.replay_cache}


def oracle_round(ri: wl.RoundInputs, tickets: np.ndarray, H0: np.ndarray, S0=None, TS0=None, floor=0,
                 policy=orc.POLICY_CPU_WINS):
    order = orc.order_from_tickets(tickets, even_ties=True)
    S = (ri.init if S0 is None else S0).copy()
    TS = np.zeros(ri.n_words, np.uint64) if TS0 is None else TS0.copy()
    H = H0.copy()
    out = orc.round_generic(REPLAY[ri.program], S, H, TS, ri.granule, ri.batch, order, ri.log, floor, policy)
    out.update({"S": S, "H": H, "TS": TS, "order": order})
    # transactions sharing a ticket must be read-only (they commute)
    tied = orc.tied_tickets(tickets)
    if tied.size:
        if ri.program == wl.PROG_OPLIST:
            assert not ri.batch.n_writes[tied].any(), "an update transaction shares its ticket"
        elif ri.program == wl.PROG_CACHE:
            assert not out["results"].reshape(-1, 9)[tied, 0].any(), "a writing cache op shares its ticket"
        else:
            raise AssertionError("tickets of this program must be unique")
    return out


def assert_round_equal(g: dict, o: dict, ri: wl.RoundInputs):
    """Element-wise, bit-exact comparison of every output of the round."""
    n_log = ri.log.shape[0]
    r = g["res"]
    assert r.error == 0
    assert r.conflict == o["conflict"], (r.conflict, o["conflict"])
    assert np.array_equal(g["results"], o["results"]), "transaction results differ"
    if g["flags"] is not None:
        assert np.array_equal(bits(g["flags"], n_log), bits(o["flags"], n_log)), "validation flags differ"
    assert int(r.n_dirty) == o["ids"].shape[0]
    assert int(r.n_runs) == o["n_runs"]
    if g["ids"] is not None:
        assert np.array_equal(g["ids"], o["ids"]), "dirty granule ids differ"
    assert np.array_equal(g["S"], o["S"]), f"GPU replica differs at {np.flatnonzero(g['S'] != o['S'])[:8]}"
    assert np.array_equal(g["H"], o["H"]), "host replica differs"
    assert np.array_equal(g["S"], g["H"]), "replicas differ after the merge"
    if o["conflict"] == 0 or r.host_discarded:
        assert int(r.n_committed) == ri.batch.n


def split_batch(program: int, batch, cuts):
    """The batch as consecutive sub-batches [cuts[k], cuts[k+1])."""
    parts = []
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        if program == wl.PROG_OPLIST:
            o = batch.offsets
            parts.append(wl.OplistBatch(offsets=(o[lo:hi + 1] - o[lo]).astype(np.uint32),
                                        idx=batch.idx[o[lo]:o[hi]].copy(), n_writes=batch.n_writes[lo:hi].copy(),
                                        tid=batch.tid[lo:hi].copy()))
        else:
            parts.append(wl.TransferBatch(src=batch.src[lo:hi].copy(), dst=batch.dst[lo:hi].copy(),
                                          amt=batch.amt[lo:hi].copy()))
    return parts


def join_results(program: int, parts: list) -> np.ndarray:
    """Results of consecutive sub-batches in the whole batch's layout
    (OPLIST: per operation in order; TRANSFER: three arrays of n)."""
    if program == wl.PROG_OPLIST:
        return np.concatenate([b.results_np() for b in parts])
    return np.concatenate([b.results_np().reshape(3, -1) for b in parts], axis=1).reshape(-1)


def streamed_round(ri: wl.RoundInputs, chunks: int = 3, where: str = "device", sync_before_push: bool = False,
                   async_merge: bool = False, policy=hm.HETM_POLICY_CPU_WINS, host=None, ctx=None, keep=False,
                   batches: int = 1, interleave: bool = False):
    """One streamed round (hetm_round_begin / push / end, GRAPH mode), the log
    pushed in `chunks` consecutive pieces from `where` (device, pinned or
    pageable host memory).  With sync_before_push the pieces are pushed once
    the execution part has finished, so early validation sees the whole read
    set and every transaction has run.  With batches > 1 the batch is cut
    into that many consecutive pieces of uneven size: the first goes to
    hetm_round_begin, the others to hetm_round_add, all before the first
    push, or with interleave one before each push.  Returns what gpu_round
    returns (results and tickets joined in the whole batch's order)."""
    import torch
    if ctx is None:
        ctx = hm.Context(ri.n_words, ri.word_bytes, ri.granule, init=ri.init, batch_capacity=max(ri.batch.n, 1),
                         log_capacity=max(ri.log.shape[0], 1), mode=hm.HETM_MODE_GRAPH, async_merge=async_merge)
    H0 = wl.host_replica(ri.init, ri.log) if host is None else host
    host_t = hm.pinned(H0.nbytes)
    host_t.numpy()[:] = H0.view(np.uint8)
    n = ri.batch.n
    if batches > 1:
        # uneven pieces: a tiny one, then growing ones
        w = np.array([1] + [2 ** k for k in range(1, batches)], np.float64)
        cuts = np.concatenate([[0], np.round(np.cumsum(w) / w.sum() * n)]).astype(np.int64)
        bs = [hm.Batch(ri.program, sb, ctx.dev) for sb in split_batch(ri.program, ri.batch, cuts)]
    else:
        bs = [hm.Batch(ri.program, ri.batch, ctx.dev)]
    b = bs[0]
    n_log = ri.log.shape[0]
    raw = np.ascontiguousarray(ri.log).view(np.uint8).reshape(-1)
    if where == "device":
        log_t = hm.to_device(ri.log, ctx.dev)
    elif where == "pinned":
        log_t = hm.pinned(raw.nbytes)
        log_t.numpy()[:] = raw
    else:
        log_t = torch.from_numpy(raw.copy())
    eb = ri.log.dtype.itemsize
    flags_t = torch.zeros(max((n_log + 31) // 32, 1) * 4, dtype=torch.uint8, device=ctx.dev)
    ids_t = torch.zeros(max(ctx.n_granules, 1) * 4, dtype=torch.uint8, device=ctx.dev)
    torch.cuda.synchronize()
    ctx.round_begin(b if b.n else None, host_t, flags=flags_t, ids=ids_t, policy=policy)
    adds = list(bs[1:])
    if not interleave:
        for bk in adds:
            ctx.round_add(bk)
        adds = []
    if sync_before_push:
        torch.cuda.synchronize()
    cuts = np.linspace(0, n_log, chunks + 1).astype(np.int64)
    doomed = 0
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        if adds:
            ctx.round_add(adds.pop(0))
        if hi > lo:
            doomed = ctx.round_push(log_t[lo * eb:hi * eb], int(hi - lo), wait=sync_before_push) or doomed
    for bk in adds:
        ctx.round_add(bk)
    res = ctx.round_end()
    ctx.sync()
    out = {
        "res": res,
        "results": join_results(ri.program, bs),
        "tickets": np.concatenate([bk.tickets_np() for bk in bs]),
        "S": ctx.read_state(hm.HETM_STATE_STMR).copy(),
        "H": host_t.numpy().view(ri.init.dtype).copy(),
        "flags": hm.tensor_to_numpy(flags_t, np.uint32),
        "ids": hm.tensor_to_numpy(ids_t, np.uint32, int(res.n_dirty)),
        "H0": H0,
        "doomed_seen": doomed,
    }
    if keep:
        out["ctx"] = ctx
    else:
        ctx.close()
    return out
