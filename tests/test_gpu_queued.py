"""Queued rounds (hetm_round_submit / hetm_round_collect): rounds launched
one ahead of the host's collection of the last outcome must give, round by
round, what the oracle gives for the same rounds run one after another --
also when a round holds the one behind it (a conflict the undo log cannot
roll back, a device error)."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu

NLOG = 1 << 12


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


class Queue:
    """A context with queued rounds beside the oracle continued round by
    round: each round is checked when it is collected."""

    def __init__(self, hm, wl, N, G, stripe, init):
        import oracle as orc
        self.hm, self.wl, self.orc, self.G = hm, wl, orc, G
        self.ctx = hm.Context(N, 4, G, init=init, stripe=stripe, batch_capacity=1 << 13, log_capacity=NLOG,
                              mode=hm.HETM_MODE_GRAPH, async_merge=True)
        self.host_t = hm.pinned(N * 4)
        self.host = self.host_t.numpy().view(np.uint32)
        self.host[:] = init
        self.S, self.H, self.TS = init.copy(), init.copy(), np.zeros(N, np.uint64)
        self.floor = 0
        self.pending, self.keep, self.outcomes = [], [], []

    def submit(self, batch, log, lo, policy=0):
        import torch
        # the host's transactions write its replica (from word lo up, where
        # no merge copy can be in flight)
        self.host[lo:] = self.wl.host_replica(self.host.copy(), log)[lo:]
        b = self.hm.Batch(1, batch)
        log_t = self.hm.to_device(log)
        torch.cuda.synchronize()
        self.ctx.round_submit(b, log_t, log.shape[0], self.host_t, policy=policy)
        self.keep.append((b, log_t))
        self.pending.append((b, batch, log, policy))

    def collect(self):
        b, batch, log, policy = self.pending.pop(0)
        res = self.ctx.round_collect()
        orc = self.orc
        self.H = self.wl.host_replica(self.H, log)
        o = orc.round_oplist(self.S, self.H, self.TS, self.G, batch, orc.order_from_tickets(b.tickets_np(),
                                                                                           even_ties=True),
                             log, self.floor, policy)
        say(f"collected: conflict {res.conflict}, dirty {res.n_dirty}")
        assert res.error == 0
        assert res.conflict == o["conflict"]
        assert np.array_equal(b.results_np(), o["results"]), "transaction results differ"
        assert int(res.n_dirty) == o["ids"].shape[0]
        gpu_won = bool(o["conflict"]) and policy == self.hm.HETM_POLICY_GPU_WINS
        assert int(res.n_committed) == (0 if o["conflict"] and not gpu_won else batch.n)
        assert res.host_discarded == int(gpu_won)
        self.floor = int(o["max_ts"])
        assert int(res.max_ts) == self.floor
        self.outcomes.append(int(res.conflict))
        return res

    def finish(self):
        while self.pending:
            self.collect()
        self.ctx.sync()
        assert np.array_equal(self.ctx.read_state(self.hm.HETM_STATE_STMR), self.S), "GPU replica differs"
        assert np.array_equal(self.host, self.H), "host replica differs"


def _inputs(wl, r, N, conflict, watermark=None):
    batch = wl.c2_batch(np.random.default_rng(500 + r), N, 1 << 13, 0.5, tid0=r << 13)
    lo = 0 if conflict else N // 2
    # every log applies (CPU wins), so round r's timestamps start above r * NLOG
    wm = r * NLOG if watermark is None else watermark
    log = wl.host_log_uniform(np.random.default_rng(600 + r), NLOG, lo, N, wm)
    return batch, log, lo


@pytest.mark.parametrize("stripe", [1, 2], ids=["undo-log", "no-undo-log"])
def test_queued_rounds_match_oracle(hm, wl, stripe):
    """Seven rounds, each submitted while the one before runs; the logs of
    rounds 3 and 6 hit the GPU's read set (CPU wins).  With the slot layout's
    undo log a conflicting round rolls back on the device and the round
    behind it runs at once; without one (lock stripes of two words) round 3
    holds round 4, which runs empty, and collect restores round 3's granules
    from the host replica and launches round 4 again; round 6, with nothing
    behind it, is restored alone.  Every round matches the oracle continued
    from the last; the replicas match at the end."""
    N, G = 1 << 18, 16
    init = np.random.default_rng(77).integers(0, 2 ** 32, size=N, dtype=np.uint64).astype(np.uint32)
    q = Queue(hm, wl, N, G, stripe, init)
    for r in range(7):
        conflict = r in (3, 6)
        if conflict:
            # the host writes into the GPU's half: no copy may be in flight there
            while q.pending:
                q.collect()
            q.ctx.sync()
        batch, log, lo = _inputs(wl, r, N, conflict)
        say(f"queued round {r}, stripe {stripe}")
        q.submit(batch, log, lo)
        if len(q.pending) == 2:
            q.collect()
    q.finish()
    assert q.outcomes == [0, 0, 0, 1, 0, 0, 1]
    st = q.ctx.stats()
    assert st.rounds == 7 and st.rounds_conflicted == 2
    assert (st.rollbacks_device, st.rollbacks_host) == ((2, 0) if stripe == 1 else (0, 2))
    q.ctx.close()


def test_queued_error_cancels_next(hm, wl):
    """A round whose log breaks a precondition (a timestamp at the
    watermark) is discarded when collected: its collect returns EORDER, the
    round queued behind it ran empty and is cancelled (ESTATE, its batch
    untouched), the GPU replica is back where it was before the failed
    round, and rounds submitted after that -- the first while the cancelled
    one is still queued -- run and continue from there."""
    N, G = 1 << 16, 16
    init = np.random.default_rng(78).integers(0, 2 ** 32, size=N, dtype=np.uint64).astype(np.uint32)
    q = Queue(hm, wl, N, G, 1, init)
    batch, log, lo = _inputs(wl, 0, N, False)
    q.submit(batch, log, lo)
    q.collect()
    bad_batch, bad_log, _ = _inputs(wl, 1, N, False)
    bad_log["ts"][17] = q.floor                    # not above the watermark
    next_batch, next_log, _ = _inputs(wl, 2, N, False)
    b1, b2 = hm.Batch(1, bad_batch), hm.Batch(1, next_batch)
    l1, l2 = hm.to_device(bad_log), hm.to_device(next_log)
    import torch
    torch.cuda.synchronize()
    say("queued: a failing round, then one behind it")
    q.ctx.round_submit(b1, l1, NLOG, q.host_t)
    q.ctx.round_submit(b2, l2, NLOG, q.host_t)
    with pytest.raises(hm.HetmError) as e:
        q.ctx.round_collect()
    assert e.value.code == hm.HETM_EORDER
    # a round submitted while the cancelled one is still queued runs for real
    # (the host never wrote the failed logs; the next rounds carry fresh ones)
    batch, log, lo = _inputs(wl, 3, N, False, watermark=q.floor)
    q.submit(batch, log, lo)
    with pytest.raises(hm.HetmError) as e:
        q.ctx.round_collect()
    assert e.value.code == hm.HETM_ESTATE
    assert not b2.tickets_np().any(), "the cancelled round ran"
    q.collect()
    q.ctx.sync()
    for k, r in enumerate((4, 5, 6)):
        batch, log, lo = _inputs(wl, r, N, False, watermark=q.floor + k * NLOG)
        q.submit(batch, log, lo)
        if len(q.pending) == 2:
            q.collect()
    q.finish()
    q.ctx.close()


def test_queued_state_errors(hm, wl):
    """Queued rounds need GRAPH mode with the double-buffered merge; at most
    two are queued; collect needs one; while rounds are queued every other
    call that queues work or reads the state is refused."""
    import torch
    N, G = 1 << 14, 16
    init = np.zeros(N, np.uint32)
    batch, log, lo = _inputs(wl, 0, N, False)
    host_t = hm.pinned(N * 4)
    for mode, am in ((hm.HETM_MODE_PLAIN, False), (hm.HETM_MODE_GRAPH, False)):
        ctx = hm.Context(N, 4, G, init=init, batch_capacity=1 << 13, log_capacity=NLOG, mode=mode, async_merge=am)
        b = hm.Batch(1, batch)
        with pytest.raises(hm.HetmError) as e:
            ctx.round_submit(b, hm.to_device(log), NLOG, host_t)
        assert e.value.code == hm.HETM_ESTATE
        ctx.close()
    ctx = hm.Context(N, 4, G, init=init, batch_capacity=1 << 13, log_capacity=NLOG, mode=hm.HETM_MODE_GRAPH,
                     async_merge=True)
    with pytest.raises(hm.HetmError) as e:
        ctx.round_collect()
    assert e.value.code == hm.HETM_ESTATE
    bs = [hm.Batch(1, batch) for _ in range(3)]
    log_t = hm.to_device(log)
    torch.cuda.synchronize()
    ctx.round_submit(bs[0], log_t, NLOG, host_t)
    ctx.round_submit(bs[1], log_t, 0, host_t)
    with pytest.raises(hm.HetmError) as e:
        ctx.round_submit(bs[2], log_t, 0, host_t)
    assert e.value.code == hm.HETM_ESTATE
    with pytest.raises(hm.HetmError) as e:
        ctx.round(bs[2], log_t, 0, host_t)
    assert e.value.code == hm.HETM_ESTATE
    with pytest.raises(hm.HetmError) as e:
        ctx.read_state(hm.HETM_STATE_STMR)
    assert e.value.code == hm.HETM_ESTATE
    r0, r1 = ctx.round_collect(), ctx.round_collect()
    assert r0.error == r1.error == 0 and int(r0.n_committed) == int(r1.n_committed) == batch.n
    ctx.sync()
    ctx.read_state(hm.HETM_STATE_STMR)           # allowed again
    ctx.close()


def test_queued_policies(hm, wl):
    """Queued rounds under both policies, one behind the other (each slot
    holds a graph per policy): the round at r = 2 conflicts under GPU wins,
    so the host's round is discarded and the granules either side wrote go
    to the host replica, and the CPU-wins round after it continues from
    there.  Every round matches the oracle under its policy."""
    N, G = 1 << 16, 16
    init = np.random.default_rng(79).integers(0, 2 ** 32, size=N, dtype=np.uint64).astype(np.uint32)
    q = Queue(hm, wl, N, G, 1, init)
    policies = [0, 1, 1, 0, 1]
    wm = 0
    for r, pol in enumerate(policies):
        conflict = r == 2
        if r in (2, 3):
            # the r = 2 log writes the GPU's half; and under GPU wins its merge
            # copies every granule that log wrote, so the host writes again
            # only once that merge has landed
            while q.pending:
                q.collect()
            q.ctx.sync()
            wm = max(wm, q.floor)
        batch, log, lo = _inputs(wl, r, N, conflict, watermark=wm)
        say(f"queued round {r}, policy {pol}")
        q.submit(batch, log, lo, policy=pol)
        # a discarded log does not raise the watermark: later logs start above
        # the last one submitted either way
        wm += NLOG
        if len(q.pending) == 2:
            q.collect()
    q.finish()
    assert q.outcomes == [0, 0, 1, 0, 0]
    q.ctx.close()
