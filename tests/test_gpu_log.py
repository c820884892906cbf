"""Validation and apply of the host log (§IV-C.2) on the GPU against the
oracle: rounds that take their log in several chunks (timestamps interleaved
across chunks, duplicates, winners superseded by a later chunk, entries older
than an earlier chunk's), buckets that need several resolve passes, and logs
that break a precondition sent through hetm_round in every form -- such a
round applies nothing, and the corrected log with the same timestamps
applies in the next round."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_util import assert_round_equal, bits, gpu_round, oracle_round, say

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


FORMS = {"plain": (0, False), "graph": (1, False), "graph_async": (1, True)}


def _chunks(wl, g, N, sizes, floor, lo=0, hi=None):
    """Chunks of one round's log over words [lo, hi): timestamps are a random
    permutation of floor+1 .. floor+total, dealt across the chunks, so chunk
    ts ranges interleave and a word's entries in a later chunk may be older
    than its entry in an earlier one."""
    hi = N if hi is None else hi
    total = int(sum(sizes))
    log = np.zeros(total, wl.LOG4_DTYPE)
    log["word"] = g.integers(lo, hi, size=total, dtype=np.uint64).astype(np.uint32)
    log["value"] = g.integers(0, 2 ** 32, size=total, dtype=np.uint64).astype(np.uint32)
    log["ts"] = g.permutation(np.arange(floor + 1, floor + total + 1, dtype=np.uint64))
    out, at = [], 0
    for s in sizes:
        out.append(log[at:at + s].copy())
        at += s
    return out


def _tie_below(log, g):
    """Adds ties below a word's winning ts: a second entry (other value)
    carrying the ts of a non-winning entry of the same word."""
    w = log["word"]
    o = np.lexsort((log["ts"], w))
    extra = []
    for i in range(1, o.shape[0]):
        a, b = o[i - 1], o[i]
        if w[a] == w[b] and len(extra) < 64:           # a is below b's ts for the same word
            e = log[a].copy()
            e["value"] ^= 0x5A5A5A5A
            extra.append(e)
    if not extra:
        return log
    out = np.concatenate([log, np.array(extra, dtype=log.dtype)])
    return out[g.permutation(out.shape[0])]


def test_multi_chunk_step_api(hm, wl, orc):
    """One round, five log chunks through hetm_validate_apply_log: flags,
    outcome and GPU replica match the oracle's chunk-by-chunk apply after every
    chunk; then the merge.  Chunks span several tiles and buckets and
    interleave in ts; the fourth is newer than everything before it, the
    fifth older than the fourth and newer than the rest."""
    import torch
    N, G = 1 << 12, 4
    g = np.random.default_rng(11)
    init = g.integers(0, 2 ** 32, size=N, dtype=np.uint64).astype(np.uint32)
    ctx = hm.Context(N, 4, G, init=init, batch_capacity=1024, log_capacity=9000)
    batch = wl.c2_batch(np.random.default_rng(12), N, 1024, 0.5)   # GPU reads the lower half
    b = hm.Batch(1, batch)
    ctx.submit(b)
    RS = ctx.read_state(hm.HETM_STATE_RS).copy()
    order = orc.order_from_tickets(b.tickets_np(), even_ties=True)
    S = init.copy()
    res, oRS, oWS = orc.replay_oplist(S, G, batch, order)
    assert np.array_equal(RS, oRS) and np.array_equal(b.results_np(), res)
    chunks = _chunks(wl, g, N, [5000, 7000, 3000], 0, lo=N // 4)      # a third of them hit the read set
    chunks[1] = _tie_below(chunks[1], g)
    top = _chunks(wl, g, N, [2000], 15000 + 64, lo=N // 4)[0]         # all newer than the round so far
    chunks.append(top)
    # then a chunk between: newer than the first three, older than the last
    mid = _chunks(wl, g, N, [64], 15000, lo=N // 4)[0]
    mid["word"][:32] = top["word"][:32]                                 # half of it loses to the fourth chunk
    chunks.append(mid)
    TS = np.zeros(N, np.uint64)
    conflict = 0
    H = init.copy()
    for i, ch in enumerate(chunks):
        say(f"multi-chunk: chunk {i} n={ch.shape[0]}")
        assert ch.shape[0] <= 9000
        log_t = hm.to_device(ch)
        flags = torch.zeros(((ch.shape[0] + 31) // 32) * 4, dtype=torch.uint8, device="cuda")
        c = ctx.validate_apply(log_t, ch.shape[0], flags)
        ofl, oc = orc.validate(ch, oRS, G, N)
        orc.apply(S, TS, ch, 0)
        conflict |= oc
        assert c == conflict
        assert np.array_equal(bits(hm.tensor_to_numpy(flags, np.uint32), ch.shape[0]), bits(ofl, ch.shape[0]))
        assert np.array_equal(ctx.read_state(hm.HETM_STATE_STMR), S), f"replica differs after chunk {i}"
    H = wl.host_replica(H, np.concatenate(chunks))
    host_t = hm.pinned(N * 4)
    host_t.numpy()[:] = H.view(np.uint8)
    nd = ctx.copyback(hm.HETM_OUTCOME_DEVICE, host_t)
    ids, _ = orc.merge(conflict, oWS, G, S, H)
    assert conflict == 1 and nd == ids.shape[0]
    assert np.array_equal(ctx.read_state(hm.HETM_STATE_STMR), S)
    assert np.array_equal(host_t.numpy().view(np.uint32), H)
    ctx.close()


def test_chunk_with_crowded_buckets(hm, wl, orc):
    """A chunk whose entries pile onto a few words (buckets far above one
    resolve pass and far above their regions, so they spill), beside a
    uniform part, then a chunk older than it on the same words: both match
    the oracle."""
    N = 1 << 16
    g = np.random.default_rng(21)
    init = g.integers(0, 2 ** 32, size=N, dtype=np.uint64).astype(np.uint32)
    ctx = hm.Context(N, 4, 16, init=init, batch_capacity=16, log_capacity=40000)
    hot = g.integers(0, N, size=6)
    n1, n2 = 30000, 6000
    ts = g.permutation(np.arange(1, n1 + n2 + 1, dtype=np.uint64))
    c1 = np.zeros(n1, wl.LOG4_DTYPE)
    c1["word"] = np.where(g.random(n1) < 0.8, hot[g.integers(0, 6, size=n1)], g.integers(0, N, size=n1))
    c1["value"] = g.integers(0, 2 ** 32, size=n1, dtype=np.uint64).astype(np.uint32)
    c1["ts"] = ts[:n1]
    c2 = np.zeros(n2, wl.LOG4_DTYPE)
    c2["word"] = hot[g.integers(0, 6, size=n2)]
    c2["value"] = g.integers(0, 2 ** 32, size=n2, dtype=np.uint64).astype(np.uint32)
    c2["ts"] = ts[n1:]
    S, TS = init.copy(), np.zeros(N, np.uint64)
    for i, ch in enumerate((c1, c2)):
        say(f"crowded buckets: chunk {i}")
        ctx.validate_apply(hm.to_device(ch), ch.shape[0])
        orc.apply(S, TS, ch, 0)
        assert np.array_equal(ctx.read_state(hm.HETM_STATE_STMR), S)
    ctx.close()


@pytest.mark.parametrize("n_hot,hot_frac", [(100, 1.0), (3, 0.5), (20, 0.9)])
def test_chunk_spilling_many_buckets(hm, wl, orc, n_hot, hot_frac):
    """A 2^18-entry chunk whose entries fall on few words (`hot_frac` of
    them on `n_hot` words, the rest uniform), so that many buckets, or a
    few by far, outgrow their regions and spill; then a second chunk of
    the same round on the same hot words, which meets the first chunk's
    winners through TS.  Both match the oracle."""
    N = 1 << 20
    g = np.random.default_rng(31 + n_hot)
    init = g.integers(0, 2 ** 32, size=N, dtype=np.uint64).astype(np.uint32)
    n1, n2 = 1 << 18, 1 << 16
    ctx = hm.Context(N, 4, 16, init=init, batch_capacity=16, log_capacity=n1)
    hot = g.choice(N, size=n_hot, replace=False)
    ts = g.permutation(np.arange(1, n1 + n2 + 1, dtype=np.uint64))
    chunks = []
    for n, tsk in ((n1, ts[:n1]), (n2, ts[n1:])):
        ch = np.zeros(n, wl.LOG4_DTYPE)
        ch["word"] = np.where(g.random(n) < hot_frac, hot[g.integers(0, n_hot, size=n)], g.integers(0, N, size=n))
        ch["value"] = g.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
        ch["ts"] = tsk
        chunks.append(ch)
    S, TS = init.copy(), np.zeros(N, np.uint64)
    for i, ch in enumerate(chunks):
        say(f"spilling chunk {i}: {ch.shape[0]} entries, {hot_frac:.0%} on {n_hot} words")
        ctx.validate_apply(hm.to_device(ch), ch.shape[0])
        orc.apply(S, TS, ch, 0)
        got = ctx.read_state(hm.HETM_STATE_STMR)
        bad = np.flatnonzero(got != S)
        if bad.size:
            say(f"  {bad.size} words differ, {np.isin(bad, hot).sum()} of them hot; first {bad[:8]}")
            for w in bad[:6]:
                k = np.flatnonzero(ch["word"] == w)
                say(f"  word {w}: got {got[w]} want {S[w]} init {init[w]} entries {list(zip(k, ch['value'][k], ch['ts'][k]))}")
        assert bad.size == 0
    ctx.close()


def test_tie_with_earlier_chunk(hm, wl, orc):
    """A chunk whose winning ts for a word equals the winner an earlier chunk
    of the round applied is EORDER and applies nothing; a tie below an
    earlier chunk's winner passes, and a chunk older than the earlier ones
    on every word applies nothing of those words."""
    N = 1024
    init = np.arange(N, dtype=np.uint32)
    ctx = hm.Context(N, 4, 4, init=init, batch_capacity=16, log_capacity=64)
    LOG = wl.LOG4_DTYPE

    def mk(entries):
        return np.array(entries, dtype=LOG)

    S, TS = init.copy(), np.zeros(N, np.uint64)
    first = mk([(5, 50, 40), (6, 60, 41), (7, 70, 42)])
    ctx.validate_apply(hm.to_device(first), 3)
    orc.apply(S, TS, first, 0)
    tied = mk([(9, 1, 43), (5, 51, 40), (8, 2, 44)])
    assert orc.apply_rc(S.copy(), TS.copy(), tied, 0) == orc.EORDER
    with pytest.raises(hm.HetmError) as e:
        ctx.validate_apply(hm.to_device(tied), 3)
    assert e.value.code == hm.HETM_EORDER
    assert np.array_equal(ctx.read_state(hm.HETM_STATE_STMR), S)
    below = mk([(6, 7, 30), (6, 8, 30), (10, 3, 45)])       # both below word 6's winner (41)
    ctx.validate_apply(hm.to_device(below), 3)
    orc.apply(S, TS, below, 0)
    assert np.array_equal(ctx.read_state(hm.HETM_STATE_STMR), S)
    # an older chunk: every entry loses to the round's earlier winners
    older = mk([(5, 9, 35), (6, 9, 36), (7, 9, 37)])
    ctx.validate_apply(hm.to_device(older), 3)
    orc.apply(S, TS, older, 0)
    assert np.array_equal(ctx.read_state(hm.HETM_STATE_STMR), S)
    ctx.close()


@pytest.mark.parametrize("fault", ["word_outside", "stale_ts", "tie_at_winner"])
@pytest.mark.parametrize("form", list(FORMS))
def test_bad_log_round(hm, wl, orc, fault, form):
    """A whole round whose log breaks a precondition returns the error and is
    discarded: the GPU replica and the watermark are as before the round.
    The corrected log, with the same timestamps, then applies in the next
    round, which matches the oracle continued from before the bad one."""
    import torch
    N, G = 1 << 14, 16
    mode, am = FORMS[form]
    g = np.random.default_rng(31)
    init = g.integers(0, 2 ** 32, size=N, dtype=np.uint64).astype(np.uint32)
    ctx = hm.Context(N, 4, G, init=init, batch_capacity=2048, log_capacity=3000, mode=mode, async_merge=am)
    host_t = hm.pinned(N * 4)
    host = host_t.numpy().view(np.uint32)
    host[:] = init
    S, TS, floor = init.copy(), np.zeros(N, np.uint64), 0
    keep = []
    for r in range(3):
        batch = wl.c2_batch(np.random.default_rng(40 + r), N // 2, 2048, 0.5, tid0=r << 11)
        log = wl.host_log_uniform(np.random.default_rng(50 + r), 2500, N // 2, N, floor)
        bad = log.copy()
        if r == 1:
            if fault == "word_outside":
                bad["word"][1700] = N
            elif fault == "stale_ts":
                bad["ts"][1700] = floor
            else:
                e = bad[np.argmax(bad["ts"])].copy()
                e["value"] ^= 1
                bad = np.concatenate([bad, np.array([e], dtype=bad.dtype)])
        host[:] = wl.host_replica(host.copy(), log)
        H = host.copy()
        b = hm.Batch(1, batch)
        say(f"bad log: form={form} fault={fault} round {r}")
        if r == 1:
            bad_t = hm.to_device(bad)
            torch.cuda.synchronize()
            with pytest.raises(hm.HetmError) as e:
                ctx.round(b, bad_t, bad.shape[0], host_t)
            want = hm.HETM_EINVAL if fault == "word_outside" else hm.HETM_EORDER
            assert e.value.code == want
            ctx.sync()
            assert np.array_equal(ctx.read_state(hm.HETM_STATE_STMR), S), "a discarded round changed the replica"
            assert ctx.stats().watermark == floor
            assert not ctx.read_state(hm.HETM_STATE_RS).any() and not ctx.read_state(hm.HETM_STATE_WS).any()
            keep.append((b, bad_t))
            b = hm.Batch(1, batch)                      # the same work again, with the corrected log
        log_t = hm.to_device(log)
        torch.cuda.synchronize()
        res = ctx.round(b, log_t, log.shape[0], host_t)
        keep.append((b, log_t))
        o = orc.round_oplist(S, H, TS, G, batch, orc.order_from_tickets(b.tickets_np(), even_ties=True), log, floor)
        assert res.conflict == o["conflict"] == 0
        assert np.array_equal(b.results_np(), o["results"])
        floor = int(o["max_ts"])
        assert int(res.max_ts) == floor
    ctx.sync()
    assert np.array_equal(ctx.read_state(hm.HETM_STATE_STMR), S)
    assert np.array_equal(host, S)
    ctx.close()


@pytest.mark.parametrize("form", list(FORMS))
def test_log_shapes(hm, wl, form):
    """Log sizes around the tile (4096 entries) and bucket boundaries, with
    and without a batch, in every round form."""
    N = 1 << 15
    mode, am = FORMS[form]
    for n_log in (1, 63, 4095, 4096, 4097, 12289):
        g = np.random.default_rng(n_log)
        ri = wl.RoundInputs(cfg="shapes", n_words=N, word_bytes=4, granule=8, program=1,
                            init=g.integers(0, 2 ** 32, size=N, dtype=np.uint64).astype(np.uint32),
                            batch=wl.c2_batch(g, N, 500, 0.5), log=wl.host_log_uniform(g, n_log, 0, N, 0))
        say(f"log shapes form={form} n_log={n_log}")
        gr = gpu_round(ri, mode=mode, async_merge=am)
        o = oracle_round(ri, gr["tickets"], gr["H0"])
        assert_round_equal(gr, o, ri)
