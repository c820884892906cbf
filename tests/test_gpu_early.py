"""Early validation (§IV-D) through the step API: a chunk of the host log
validated while the batch still executes dooms the round, the transaction
kernel stops short, and the round ends as a conflict (CPU wins: the GPU
replica is restored from the host replica).  A doom never reaches into the
next round.  Oracle parity, bit-exact."""
import numpy as np
import pytest

import oracle as orc
from gpu_util import say

pytestmark = pytest.mark.gpu

N = 1 << 16
G = 64


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


def _batch(wl, seed, n, lo, hi, tid0):
    g = np.random.default_rng(seed)
    return wl._oplist_from_lists(np.full(n, 4, np.uint64), np.full(n, 2), g.integers(lo, hi, size=4 * n,
                                                                                   dtype=np.uint64), tid0)


def _close(hm, ctx, log_t, n_log, host_t):
    c = ctx.validate_apply(log_t, n_log)
    nd = ctx.copyback(hm.HETM_OUTCOME_DEVICE, host_t)
    return c, nd


def test_doom_stops_later_batches(hm, wl):
    """Batch A commits, a chunk hitting A's read set is early-validated
    (deterministic doom), batch B then executes nothing; the round is a
    conflict and both replicas equal the host's.  The next round on the same
    context, with a disjoint log, commits in full and matches the oracle."""
    import torch
    init = np.random.default_rng(7).integers(0, 2 ** 32, size=N, dtype=np.uint64).astype(np.uint32)
    ctx = hm.Context(N, 4, G, init=init, batch_capacity=8192, log_capacity=4096, mode=hm.HETM_MODE_PLAIN)
    A, B = _batch(wl, 1, 256, 0, N // 2, 0), _batch(wl, 2, 8192, 0, N // 2, 1000)
    bA, bB = hm.Batch(1, A), hm.Batch(1, B)
    ctx.submit(bA)
    torch.cuda.synchronize()
    RS = ctx.read_state(hm.HETM_STATE_RS)
    hit_g = int(np.flatnonzero(np.unpackbits(RS.view(np.uint8), bitorder="little"))[0])
    log = wl.host_log_uniform(np.random.default_rng(3), 1000, N // 2, N, 0)
    log["word"][500] = hit_g * G + 3                       # lands in a granule A read
    log_t = hm.to_device(log)
    say("early validation: deterministic doom")
    assert ctx.early_validate(log_t, 1000, wait=True) == 1
    ctx.submit(bB)
    H0 = wl.host_replica(init, log)
    host_t = hm.pinned(N * 4)
    host_t.numpy()[:] = H0.view(np.uint8)
    c, nd = _close(hm, ctx, log_t, 1000, host_t)
    st = ctx.stats()
    assert c == 1
    assert st.rounds_conflicted == 1
    assert st.txns_aborted == A.n, "batch B ran although the round was doomed"
    TS = np.zeros(N, np.uint64)
    S = init.copy()
    orc.apply(S, TS, log, 0)
    assert np.array_equal(ctx.read_state(hm.HETM_STATE_STMR), H0)
    assert np.array_equal(host_t.numpy().view(np.uint32), H0)
    assert not ctx.read_state(hm.HETM_STATE_RS).any()

    # next round: the doom of the last round must not stop this one
    C = _batch(wl, 4, 4096, 0, N // 2, 50000)
    bC = hm.Batch(1, C)
    log2 = wl.host_log_uniform(np.random.default_rng(5), 2000, N // 2, N, int(TS.max()))
    log2_t = hm.to_device(log2)
    assert ctx.early_validate(log2_t, 2000, wait=True) == 0
    ctx.submit(bC)
    H1 = wl.host_replica(H0, log2)
    host_t.numpy()[:] = H1.view(np.uint8)
    c, nd = _close(hm, ctx, log2_t, 2000, host_t)
    assert c == 0
    order = orc.order_from_tickets(bC.tickets_np(), even_ties=True)
    S = H0.copy()
    o = orc.round_generic(orc.replay_oplist, S, H1.copy(), TS, G, C, order, log2, int(TS.max()))
    assert np.array_equal(bC.results_np(), o["results"])
    assert np.array_equal(ctx.read_state(hm.HETM_STATE_STMR), S)
    assert np.array_equal(host_t.numpy().view(np.uint32), S)
    assert ctx.stats().txns_committed == C.n
    ctx.close()


@pytest.mark.parametrize("delay_us", [0, 300])
def test_doom_while_executing(hm, wl, delay_us):
    """A chunk with a write to a hot word, early-validated `delay_us` after a
    large batch is submitted: whatever the early kernel saw, the round is a
    conflict and the replicas equal the host's.  Reports how much of the
    batch ran before the kernel stopped."""
    import time
    n_words = 1 << 22
    n = 1 << 18
    g = np.random.default_rng(11)
    init = g.integers(0, 2 ** 32, size=n_words, dtype=np.uint64).astype(np.uint32)
    idx = g.integers(0, n_words // 2, size=8 * n, dtype=np.uint64)
    idx[::8] = g.integers(0, 64, size=n, dtype=np.uint64)          # every transaction reads a hot word first
    batch = wl._oplist_from_lists(np.full(n, 8, np.uint64), np.full(n, 2), idx, 0)
    ctx = hm.Context(n_words, 4, 16, init=init, batch_capacity=n, log_capacity=4096, mode=hm.HETM_MODE_PLAIN)
    b = hm.Batch(1, batch)
    log = wl.host_log_uniform(g, 4096, n_words // 2, n_words, 0)
    log["word"][0] = 5
    log_t = hm.to_device(log)
    H0 = wl.host_replica(init, log)
    host_t = hm.pinned(n_words * 4)
    host_t.numpy()[:] = H0.view(np.uint8)
    import torch
    torch.cuda.synchronize()
    ctx.submit(b)
    t_end = time.perf_counter() + delay_us * 1e-6
    while time.perf_counter() < t_end:
        pass
    d = ctx.early_validate(log_t, 4096, wait=True)
    c, nd = _close(hm, ctx, log_t, 4096, host_t)
    ran = ctx.stats().txns_aborted
    say(f"delay {delay_us} us: doomed={d} transactions run before the stop: {ran} of {n}")
    assert c == 1
    if d:
        assert ran <= n
    else:
        assert ran == n
    assert np.array_equal(ctx.read_state(hm.HETM_STATE_STMR), H0)
    assert np.array_equal(host_t.numpy().view(np.uint32), H0)
    ctx.close()


def test_early_validate_edges(hm, wl):
    """n = 0 is a no-op; an entry past the end is skipped (the final
    validation reports it); a GRAPH context refuses the call."""
    init = np.zeros(N, np.uint32)
    ctx = hm.Context(N, 4, G, init=init, batch_capacity=16, log_capacity=16, mode=hm.HETM_MODE_PLAIN)
    empty = hm.to_device(np.zeros(1, wl.LOG4_DTYPE))
    assert ctx.early_validate(empty, 0, wait=True) == 0
    bad = np.zeros(4, wl.LOG4_DTYPE)
    bad["word"] = [1, 2, N + 5, 3]
    bad["ts"] = [1, 2, 3, 4]
    assert ctx.early_validate(hm.to_device(bad), 4, wait=True) == 0
    ctx.close()
    gctx = hm.Context(N, 4, G, init=init, batch_capacity=16, log_capacity=16, mode=hm.HETM_MODE_GRAPH)
    with pytest.raises(hm.HetmError) as e:
        gctx.early_validate(empty, 0)
    assert e.value.code == hm.HETM_ESTATE
    gctx.close()
