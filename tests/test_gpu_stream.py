"""Streamed GRAPH rounds (hetm_round_begin / push / end): the host log is
shipped in chunks while the round executes (§IV-D, inter-device
synchronization) and each chunk is validated early against the read set
(§IV-D, early validation).  The round's outcome is that of the same round
through hetm_round: bit-exact oracle parity, chunks from device, pinned and
pageable memory, both merge forms, both policies, rounds fed several
batches (hetm_round_add).  A chunk that hits the read set while a large
batch still runs dooms the round, which then runs fewer transactions than
its batch."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as orc
from gpu_util import assert_round_equal, oracle_round, say, streamed_round

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_00661_amd import hetm
    hetm.lib()
    return hetm


@pytest.fixture(scope="module")
def wl():
    from paper_1905_00661_amd import workloads
    return workloads


@pytest.mark.parametrize("variant,chunks,where,async_merge", [
    ("p", 3, "device", False), ("p", 3, "pinned", True), ("p", 1, "pageable", False),
    ("", 3, "device", False), ("", 2, "pinned", True), ("w", 5, "device", True)])
def test_streamed_round_parity(hm, wl, variant, chunks, where, async_merge):
    """The small configuration's round, its log pushed in `chunks` pieces
    once execution has finished: every output equals the oracle's (the
    as-named variants conflict, and early validation dooms them after every
    transaction ran, which changes nothing)."""
    ri = wl.c1(variant)
    say(f"streamed round c1{variant}: {chunks} chunks from {where}, async merge {async_merge}")
    g = streamed_round(ri, chunks=chunks, where=where, sync_before_push=True, async_merge=async_merge)
    o = oracle_round(ri, g["tickets"], g["H0"])
    assert_round_equal(g, o, ri)
    assert g["res"].doomed == (1 if o["conflict"] else 0)
    assert g["doomed_seen"] == o["conflict"]


@pytest.mark.parametrize("variant,batches,async_merge,interleave", [
    ("p", 3, False, False), ("", 4, True, False), ("w", 3, False, False), ("p", 5, True, True)])
def test_streamed_round_batches(hm, wl, variant, batches, async_merge, interleave):
    """A streamed round fed several batches of uneven size, the first through
    hetm_round_begin and the others through hetm_round_add (all before the
    pushes, or one before each push while the earlier ones run): every
    output equals the oracle's replay of the whole batch in the recorded
    ticket order, and the round counts every batch's transactions."""
    ri = wl.c1(variant)
    say(f"streamed round c1{variant}: {batches} batches, async merge {async_merge}, interleave {interleave}")
    g = streamed_round(ri, chunks=4, where="device", sync_before_push=not interleave, async_merge=async_merge,
                       batches=batches, interleave=interleave)
    o = oracle_round(ri, g["tickets"], g["H0"])
    assert_round_equal(g, o, ri)
    if o["conflict"]:
        assert int(g["res"].n_aborted) == ri.batch.n


@pytest.mark.parametrize("steal", [0.0, 0.002])
def test_streamed_transfer_batches(hm, wl, steal):
    """Bank transfers (hot-account chains per batch) in a streamed round of
    five batches: oracle parity and conserved balances; with `steal` some
    transfers touch the host's accounts and the round conflicts."""
    d = wl.c3(n_accounts=1 << 16, host_accounts=1 << 10, n_txn=40000, n_host=2000, steal=steal)
    H = d["init"].copy()
    tm = hm.HostTM(H)
    _, log = tm.transfers(d["host"].src, d["host"].dst, d["host"].amt)
    tm.close()
    ri = wl.RoundInputs(cfg="c3", n_words=1 << 16, word_bytes=8, granule=16, program=wl.PROG_TRANSFER,
                        init=d["init"], batch=d["batch"], log=log)
    g = streamed_round(ri, chunks=2, sync_before_push=True, async_merge=True, host=H, batches=5)
    o = oracle_round(ri, g["tickets"], H)
    assert_round_equal(g, o, ri)
    assert int(g["S"].sum()) == int(d["init"].sum())
    assert o["conflict"] == (1 if steal else 0)


def test_round_add_errors(hm, wl):
    """hetm_round_add outside a streamed round is ESTATE; a batch of another
    program is EINVAL and one over the capacity ECAPACITY, and either leaves
    the round as it was: it ends equal to the oracle's round of the batches
    that were taken."""
    import torch
    ri = wl.c1("p")
    ctx = hm.Context(ri.n_words, 4, ri.granule, init=ri.init, batch_capacity=ri.batch.n, log_capacity=ri.log.shape[0],
                     mode=hm.HETM_MODE_GRAPH)
    host_t = hm.pinned(ri.init.nbytes)
    H0 = wl.host_replica(ri.init, ri.log)
    host_t.numpy()[:] = H0.view(np.uint8)
    from gpu_util import split_batch
    a, b = split_batch(ri.program, ri.batch, [0, 1000, ri.batch.n])
    ba, bb = hm.Batch(ri.program, a), hm.Batch(ri.program, b)
    with pytest.raises(hm.HetmError) as e:
        ctx.round_add(bb)
    assert e.value.code == hm.HETM_ESTATE
    ctx.round_begin(ba, host_t)
    other = wl.TransferBatch(src=np.zeros(4, np.uint32), dst=np.ones(4, np.uint32), amt=np.ones(4, np.uint32))
    with pytest.raises(hm.HetmError) as e:
        ctx.round_add(hm.Batch(hm.HETM_PROG_TRANSFER, other))
    assert e.value.code == hm.HETM_EINVAL
    big = wl.c1("p", n_txn=ri.batch.n + 1).batch
    with pytest.raises(hm.HetmError) as e:
        ctx.round_add(hm.Batch(ri.program, big))
    assert e.value.code == hm.HETM_ECAPACITY
    ctx.round_add(bb)
    ctx.round_push(hm.to_device(ri.log), ri.log.shape[0])
    res = ctx.round_end()
    ctx.sync()
    g = {"res": res, "results": np.concatenate([ba.results_np(), bb.results_np()]),
         "tickets": np.concatenate([ba.tickets_np(), bb.tickets_np()]), "flags": None, "ids": None,
         "S": ctx.read_state(hm.HETM_STATE_STMR).copy(), "H": host_t.numpy().view(np.uint32).copy()}
    o = oracle_round(ri, g["tickets"], H0)
    assert_round_equal(g, o, ri)
    ctx.close()


@pytest.mark.parametrize("variant", ["p", "w"])
def test_streamed_mixed_chunks(hm, wl, variant):
    """Chunks read in place (two consecutive slices of one device buffer),
    then one from another device buffer and one from pinned memory, which
    move the round's log into the context's buffer: the round equals the
    oracle's."""
    import torch
    ri = wl.c1(variant)
    n = ri.log.shape[0]
    cuts = [0, n // 5, n // 2, (3 * n) // 4, n]
    eb = ri.log.dtype.itemsize
    raw = np.ascontiguousarray(ri.log).view(np.uint8).reshape(-1)
    ctx = hm.Context(ri.n_words, 4, ri.granule, init=ri.init, batch_capacity=ri.batch.n, log_capacity=n,
                     mode=hm.HETM_MODE_GRAPH, async_merge=True)
    H0 = wl.host_replica(ri.init, ri.log)
    host_t = hm.pinned(H0.nbytes)
    host_t.numpy()[:] = H0.view(np.uint8)
    b = hm.Batch(ri.program, ri.batch, ctx.dev)
    a_dev = hm.to_device(ri.log, ctx.dev)                                    # parts 0 and 1, in place
    b_dev = torch.from_numpy(raw[cuts[2] * eb:cuts[3] * eb].copy()).to(ctx.dev)   # part 2, elsewhere
    c_pin = hm.pinned((cuts[4] - cuts[3]) * eb)                              # part 3, pinned
    c_pin.numpy()[:] = raw[cuts[3] * eb:]
    flags_t = torch.zeros(((n + 31) // 32) * 4, dtype=torch.uint8, device=ctx.dev)
    ids_t = torch.zeros(ctx.n_granules * 4, dtype=torch.uint8, device=ctx.dev)
    torch.cuda.synchronize()
    ctx.round_begin(b, host_t, flags=flags_t, ids=ids_t)
    torch.cuda.synchronize()
    ctx.round_push(a_dev[:cuts[1] * eb], cuts[1])
    ctx.round_push(a_dev[cuts[1] * eb:cuts[2] * eb], cuts[2] - cuts[1])
    ctx.round_push(b_dev, cuts[3] - cuts[2])
    ctx.round_push(c_pin, cuts[4] - cuts[3])
    res = ctx.round_end()
    ctx.sync()
    g = {"res": res, "results": b.results_np(), "tickets": b.tickets_np(),
         "S": ctx.read_state(hm.HETM_STATE_STMR).copy(), "H": host_t.numpy().view(np.uint32).copy(),
         "flags": hm.tensor_to_numpy(flags_t, np.uint32),
         "ids": hm.tensor_to_numpy(ids_t, np.uint32, int(res.n_dirty)), "H0": H0}
    o = oracle_round(ri, g["tickets"], H0)
    assert_round_equal(g, o, ri)
    ctx.close()


def test_streamed_gpu_wins(hm, wl):
    """GPU wins: pushed chunks are not early-validated (the GPU keeps its
    round); the conflicting host log is discarded as in hetm_round."""
    ri = wl.c1("w")
    g = streamed_round(ri, chunks=3, where="device", policy=hm.HETM_POLICY_GPU_WINS)
    o = oracle_round(ri, g["tickets"], g["H0"], policy=orc.POLICY_GPU_WINS)
    assert_round_equal(g, o, ri)
    assert g["res"].doomed == 0


def test_streamed_rounds_in_sequence(hm, wl):
    """Streamed and whole rounds in turn on one context with the double-
    buffered merge: each matches the oracle, starting from the replicas the
    last one left."""
    from gpu_util import gpu_round
    ri = wl.c1("p")
    ctx = None
    S, TS, floor = ri.init.copy(), np.zeros(ri.n_words, np.uint64), 0
    for k, streamed in enumerate([True, False, True, True]):
        g = np.random.default_rng(100 + k)
        batch = wl._oplist_from_lists(np.full(2048, 4, np.uint64), np.full(2048, 4), g.integers(
            0, ri.n_words // 2, size=4 * 2048, dtype=np.uint64), k * 4096)
        log = wl.host_log_uniform(g, 6000, ri.n_words // 2, ri.n_words, floor)
        rk = wl.RoundInputs(cfg="seq", n_words=ri.n_words, word_bytes=4, granule=ri.granule, program=wl.PROG_OPLIST,
                            init=S.copy(), batch=batch, log=log)
        H0 = wl.host_replica(S, log)
        if ctx is None:
            from paper_1905_00661_amd import hetm
            ctx = hetm.Context(ri.n_words, 4, ri.granule, init=S, batch_capacity=4096, log_capacity=8192,
                               mode=hetm.HETM_MODE_GRAPH, async_merge=True)
        if streamed:
            out = streamed_round(rk, chunks=4, where="pinned", ctx=ctx, host=H0, keep=True)
        else:
            out = gpu_round(rk, ctx=ctx, host=H0, keep=True)
        o = oracle_round(rk, out["tickets"], H0, S0=S, TS0=TS, floor=floor)
        assert_round_equal(out, o, rk)
        S, TS, floor = o["S"], o["TS"], int(out["res"].max_ts)
    ctx.close()


def test_doomed_round_ran_fewer(hm, wl):
    """A large batch whose transactions all read a hot word first; the host
    pushes one-entry chunks writing that word until one comes back doomed.
    The round is a conflict (CPU wins), it ran fewer transactions than its
    batch, and both replicas equal the host's."""
    import torch
    n_words, n = 1 << 22, 1 << 20
    g = np.random.default_rng(21)
    init = g.integers(0, 2 ** 32, size=n_words, dtype=np.uint64).astype(np.uint32)
    idx = g.integers(0, n_words // 2, size=8 * n, dtype=np.uint64)
    idx[::8] = g.integers(0, 64, size=n, dtype=np.uint64)
    batch = wl._oplist_from_lists(np.full(n, 8, np.uint64), np.full(n, 2), idx, 0)
    ctx = hm.Context(n_words, 4, 16, init=init, batch_capacity=n, log_capacity=256, mode=hm.HETM_MODE_GRAPH)
    b = hm.Batch(1, batch)
    pieces = wl.host_log_uniform(g, 256, n_words // 2, n_words, 0)
    pieces["word"] = 5                                  # every piece writes hot word 5,
    pieces["value"] = 12345                             # the same value: any prefix gives one replica
    H0 = wl.host_replica(init, pieces)
    host_t = hm.pinned(n_words * 4)
    host_t.numpy()[:] = H0.view(np.uint8)
    log_t = hm.to_device(pieces)
    eb = pieces.dtype.itemsize
    torch.cuda.synchronize()
    ctx.round_begin(b, host_t)
    pushed, d = 0, 0
    while not d and pushed < 256:
        d = ctx.round_push(log_t[pushed * eb:(pushed + 1) * eb], 1, wait=True)
        pushed += 1
    res = ctx.round_end()
    ctx.sync()
    ran = int(ctx.stats().txns_aborted)                # transactions executed, then aborted
    say(f"doomed after {pushed} pushed entries; transactions run: {ran} of {n}")
    assert d == 1 and res.doomed == 1 and res.conflict == 1
    assert int(res.n_aborted) == n and int(res.n_committed) == 0
    assert ran < n, "the doomed round ran its whole batch"
    H = wl.host_replica(init, pieces[:pushed])
    assert np.array_equal(H, H0)
    assert np.array_equal(ctx.read_state(hm.HETM_STATE_STMR), H)
    assert np.array_equal(host_t.numpy().view(np.uint32), H)
    # the next round on the context is not doomed by the last one
    g2 = np.random.default_rng(22)
    b2 = hm.Batch(1, wl._oplist_from_lists(np.full(4096, 4, np.uint64), np.full(4096, 2), g2.integers(
        0, n_words // 2, size=4 * 4096, dtype=np.uint64), 1 << 24))
    log2 = wl.host_log_uniform(g2, 200, n_words // 2, n_words, int(res.max_ts))
    host_t.numpy()[:] = wl.host_replica(H, log2).view(np.uint8)
    ctx.round_begin(b2, host_t)
    assert ctx.round_push(hm.to_device(log2), 200, wait=True) == 0
    r2 = ctx.round_end()
    assert r2.conflict == 0 and r2.doomed == 0 and int(r2.n_committed) == 4096
    ctx.close()


def test_doomed_round_with_added_batches(hm, wl):
    """A streamed round whose first batch reads a hot word everywhere; the
    host pushes one-entry chunks writing that word until one comes back
    doomed, then adds three more batches: the round is a conflict, every
    batch's transactions are reported aborted, the added batches leave at
    once (the round ran far fewer transactions than it was given), and both
    replicas equal the host's."""
    import torch
    n_words, n = 1 << 22, 1 << 18
    g = np.random.default_rng(23)
    init = g.integers(0, 2 ** 32, size=n_words, dtype=np.uint64).astype(np.uint32)
    batches = []
    for k in range(4):
        idx = g.integers(0, n_words // 2, size=8 * n, dtype=np.uint64)
        idx[::8] = g.integers(0, 64, size=n, dtype=np.uint64)
        batches.append(hm.Batch(1, wl._oplist_from_lists(np.full(n, 8, np.uint64), np.full(n, 2), idx, k * n)))
    ctx = hm.Context(n_words, 4, 16, init=init, batch_capacity=n, log_capacity=256, mode=hm.HETM_MODE_GRAPH)
    pieces = wl.host_log_uniform(g, 256, n_words // 2, n_words, 0)
    pieces["word"] = 5
    pieces["value"] = 777
    host_t = hm.pinned(n_words * 4)
    host_t.numpy()[:] = wl.host_replica(init, pieces).view(np.uint8)
    log_t = hm.to_device(pieces)
    eb = pieces.dtype.itemsize
    torch.cuda.synchronize()
    ctx.round_begin(batches[0], host_t)
    pushed, d = 0, 0
    while not d and pushed < 256:
        d = ctx.round_push(log_t[pushed * eb:(pushed + 1) * eb], 1, wait=True)
        pushed += 1
    for b in batches[1:]:
        ctx.round_add(b)
    res = ctx.round_end()
    ctx.sync()
    ran = int(ctx.stats().txns_aborted)
    say(f"doomed after {pushed} entries, then 3 batches added; transactions run: {ran} of {4 * n}")
    assert d == 1 and res.doomed == 1 and res.conflict == 1
    assert int(res.n_aborted) == 4 * n and int(res.n_committed) == 0
    assert ran < n, "the batches added to a doomed round ran"
    H = wl.host_replica(init, pieces[:pushed])
    assert np.array_equal(ctx.read_state(hm.HETM_STATE_STMR), H)
    assert np.array_equal(host_t.numpy().view(np.uint32), H)
    ctx.close()


def test_stream_errors(hm, wl):
    """Out-of-order calls give ESTATE; a push past the capacity gives
    ECAPACITY and appends nothing; a pushed entry outside the replica fails
    the round (EINVAL) and leaves the context usable."""
    N = 1 << 12
    init = np.arange(N, dtype=np.uint32)
    plain = hm.Context(N, 4, 16, init=init, batch_capacity=16, log_capacity=16, mode=hm.HETM_MODE_PLAIN)
    host_t = hm.pinned(N * 4)
    host_t.numpy()[:] = init.view(np.uint8)
    with pytest.raises(hm.HetmError) as e:
        plain.round_begin(None, host_t)
    assert e.value.code == hm.HETM_ESTATE
    plain.close()
    ctx = hm.Context(N, 4, 16, init=init, batch_capacity=16, log_capacity=16, mode=hm.HETM_MODE_GRAPH)
    log = wl.host_log_uniform(np.random.default_rng(1), 16, 0, N, 0)
    log_t = hm.to_device(log)
    for call in (lambda: ctx.round_push(log_t, 1), lambda: ctx.round_end()):
        with pytest.raises(hm.HetmError) as e:
            call()
        assert e.value.code == hm.HETM_ESTATE
    ctx.round_begin(None, host_t)
    with pytest.raises(hm.HetmError) as e:
        ctx.round_begin(None, host_t)
    assert e.value.code == hm.HETM_ESTATE
    with pytest.raises(hm.HetmError) as e:
        ctx.round(None, log_t, 0, host_t)
    assert e.value.code == hm.HETM_ESTATE
    ctx.round_push(log_t, 10)
    with pytest.raises(hm.HetmError) as e:
        ctx.round_push(log_t, 7)
    assert e.value.code == hm.HETM_ECAPACITY
    ctx.round_push(log_t[10 * 16:], 6)
    host_t.numpy()[:] = wl.host_replica(init, log).view(np.uint8)
    r = ctx.round_end()
    assert r.conflict == 0 and r.error == 0
    assert np.array_equal(ctx.read_state(hm.HETM_STATE_STMR), wl.host_replica(init, log))
    # a bad entry fails the round's validation: EINVAL, nothing applied
    S1 = ctx.read_state(hm.HETM_STATE_STMR).copy()
    bad = wl.host_log_uniform(np.random.default_rng(2), 4, 0, N, int(r.max_ts))
    bad["word"][2] = N + 3
    ctx.round_begin(None, host_t)
    ctx.round_push(hm.to_device(bad), 4)
    with pytest.raises(hm.HetmError) as e:
        ctx.round_end()
    assert e.value.code == hm.HETM_EINVAL
    assert np.array_equal(ctx.read_state(hm.HETM_STATE_STMR), S1)
    ok = wl.host_log_uniform(np.random.default_rng(3), 8, 0, N, int(r.max_ts))
    host_t.numpy()[:] = wl.host_replica(S1, ok).view(np.uint8)
    ctx.round_begin(None, host_t, hm.to_device(ok), 8)
    r3 = ctx.round_end()
    assert r3.error == 0
    assert np.array_equal(ctx.read_state(hm.HETM_STATE_STMR), wl.host_replica(S1, ok))
    ctx.close()
