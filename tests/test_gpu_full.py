"""Parity at the full sizes of the five named configurations, in the launch
configuration the benchmark times (hipGraph round with the double-buffered
merge, default transaction grid).  Every output is compared bit-exactly with
the oracle, which replays the whole round in the GPU's commit order."""
import numpy as np
import pytest

import oracle as orc
from gpu_util import assert_round_equal, gpu_round, oracle_round, say

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


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


def test_c2_full_size(hm, wl):
    """2^28 u32 words (1 GiB), 2^20 transactions (90% 16-read, 10% 4RMW,
    hot 1% at p = 0.5), 2^20-entry host log with one injected conflict,
    granule 16."""
    ri = wl.c2(p_hot=0.5, granule=16, conflict_rate=0.0)
    say("c2 full: GPU round")
    g = gpu_round(ri, mode=1, async_merge=True)
    say("c2 full: oracle round")
    o = oracle_round(ri, g["tickets"], g["H0"])
    assert_round_equal(g, o, ri)
    assert o["conflict"] == 0 and int(g["res"].n_committed) == 1 << 20


def test_c2_full_size_conflict(hm, wl):
    """The same at hot fraction 0.9 and granule 64 with a conflicting log:
    CPU wins, the round rolls back on the device from its undo log."""
    ri = wl.c2(p_hot=0.9, granule=64, conflict_rate=1.0, round_no=1)
    g = gpu_round(ri, mode=1, async_merge=True)
    o = oracle_round(ri, g["tickets"], g["H0"])
    assert_round_equal(g, o, ri)
    assert o["conflict"] == 1


def test_c2_full_size_queued(hm, wl):
    """Three large rounds as the benchmark's headline runs them: each
    submitted while the one before runs (hetm_round_submit), collected in
    order.  Every collected round equals the oracle continued from the last
    in every output it reports, and both replicas equal the oracle's at the
    end."""
    import torch
    N, n, G = 1 << 28, 1 << 20, 16
    rounds = [wl.c2(p_hot=0.5, granule=G, round_no=3)]
    rounds += [wl.c2(p_hot=0.5, granule=G, round_no=4 + k, watermark=(k + 1) * n, init=False) for k in range(2)]
    init = rounds[0].init
    ctx = hm.Context(N, 4, G, init=init, max_ops=16, batch_capacity=n, log_capacity=n, mode=hm.HETM_MODE_GRAPH,
                     async_merge=True)
    host_t = hm.pinned(N * 4)
    host = host_t.numpy().view(np.uint32)
    host[:] = init
    S, H, TS, floor = init.copy(), init.copy(), np.zeros(N, np.uint64), 0
    keep, pending = [], []

    def collect():
        nonlocal H, floor
        b, ri = pending.pop(0)
        res = ctx.round_collect()
        say(f"c2 full queued: oracle round {len(keep) - len(pending) - 1}")
        H = wl.host_replica(H, ri.log)
        o = orc.round_oplist(S, H, TS, G, ri.batch, orc.order_from_tickets(b.tickets_np(), even_ties=True), ri.log,
                             floor)
        assert res.error == 0 and res.conflict == o["conflict"] == 0
        assert np.array_equal(b.results_np(), o["results"]), "transaction results differ"
        assert int(res.n_dirty) == o["ids"].shape[0] and int(res.n_runs) == o["n_runs"]
        assert int(res.n_committed) == n
        floor = int(o["max_ts"])
        assert int(res.max_ts) == floor

    for r, ri in enumerate(rounds):
        # the host's writes land in its half, where no merge copy is in flight
        host[N // 2:] = wl.host_replica(host.copy(), ri.log)[N // 2:]
        b = hm.Batch(hm.HETM_PROG_OPLIST, ri.batch)
        log_t = hm.to_device(ri.log)
        torch.cuda.synchronize()
        say(f"c2 full queued: submit round {r}")
        ctx.round_submit(b, log_t, n, host_t)
        keep.append((b, log_t))
        pending.append((b, ri))
        if len(pending) == 2:
            collect()
    while pending:
        collect()
    ctx.sync()
    assert np.array_equal(ctx.read_state(hm.HETM_STATE_STMR), S), "GPU replica differs"
    assert np.array_equal(host, H), "host replica differs"
    ctx.close()


@pytest.mark.parametrize("conflict_rate", [0.0, 1.0])
def test_c2_full_size_streamed(hm, wl, conflict_rate):
    """The large round as a streamed round: its 2^20-entry log pushed in 16
    chunks once execution has finished (early validation sees the whole read
    set), then the tail.  Equal to the oracle in every output."""
    from gpu_util import streamed_round
    ri = wl.c2(p_hot=0.5, granule=16, conflict_rate=conflict_rate, round_no=2)
    say(f"c2 full streamed, conflict rate {conflict_rate}: GPU round")
    g = streamed_round(ri, chunks=16, where="device", sync_before_push=True, async_merge=True)
    say("c2 full streamed: oracle round")
    o = oracle_round(ri, g["tickets"], g["H0"])
    assert_round_equal(g, o, ri)
    assert o["conflict"] == int(conflict_rate) and g["res"].doomed == o["conflict"]


def test_c3_full_size(hm, wl):
    """2^24 int64 accounts = 1000, a batch of U[2^20, 2^21] Zipf(0.9)
    transfers, the host's 2^15 transfers on its 2^16 accounts by the host TM
    threads; balance conserved exactly."""
    d = wl.c3()
    H = d["init"].copy()
    tm = hm.HostTM(H, ts_start=0)
    ts, log = tm.transfers(d["host"].src, d["host"].dst, d["host"].amt, threads=8)
    tm.close()
    ri = wl.RoundInputs(cfg="c3", n_words=1 << 24, word_bytes=8, granule=64, program=wl.PROG_TRANSFER,
                        init=d["init"], batch=d["batch"], log=log)
    say(f"c3 full: {d['batch'].n} transfers")
    g = gpu_round(ri, host=H, mode=1, async_merge=True)
    say(f"c3 full: retries={g['res'].n_local_retries}")
    o = oracle_round(ri, g["tickets"], H)
    assert_round_equal(g, o, ri)
    assert int(g["S"].sum()) == 1000 * (1 << 24) and g["S"].min() >= 0


def test_c4_full_size(hm, wl):
    """2^22 sets x 8 ways (2 GiB of words) warmed to 95% by host PUTs, 2^20
    GPU requests (95% GET / 5% PUT, Zipf 0.99 over 2^26 keys, even keys),
    2^14 host PUTs on odd keys; no torn entries."""
    nsets = 1 << 22
    N = nsets * 128
    g0 = wl.rng("c4", 0, 2)
    warm = np.zeros(N, np.uint32)
    tm = hm.HostTM(warm, stripe=128)
    keys = g0.permutation(np.arange(1, (1 << 26) + 1, dtype=np.uint64))[: int(nsets * 8 * 0.95)]
    tm.cache_puts(keys, threads=8)
    clock = tm.clock
    tm.close()
    b = wl.c4_requests(g0, 1 << 20, 1 << 26, theta=0.99, put_frac=0.05, parity=0, tid0=clock + 10 ** 7)
    H = warm.copy()
    tm = hm.HostTM(H, stripe=128, ts_start=clock)
    hk = wl.c4_requests(g0, 1 << 14, 1 << 26, theta=0.99, put_frac=1.0, parity=1).key
    _, log = tm.cache_puts(hk, threads=8)
    tm.close()
    ri = wl.RoundInputs(cfg="c4", n_words=N, word_bytes=4, granule=128, program=wl.PROG_CACHE, init=warm, batch=b,
                        log=log)
    say("c4 full: GPU round")
    g = gpu_round(ri, host=H, mode=1, async_merge=True, stripe=1)
    o = oracle_round(ri, g["tickets"], H)
    assert_round_equal(g, o, ri)
    sets = g["S"].reshape(nsets, 128)
    k = sets[:, 0:16].reshape(nsets, 8, 2).astype(np.uint64)
    k = k[:, :, 0] | (k[:, :, 1] << np.uint64(32))
    full = k != 0
    v = sets[:, 32:96].reshape(nsets, 8, 8)[full]
    z = k[full]
    chk = (z ^ (z >> np.uint64(30))) * np.uint64(0xbf58476d1ce4e5b9)
    chk = (chk ^ (chk >> np.uint64(27))) * np.uint64(0x94d049bb133111eb)
    chk = (chk ^ (chk >> np.uint64(31))).astype(np.uint32)
    assert np.array_equal(np.bitwise_xor.reduce(v[:, :7], axis=1) ^ chk, v[:, 7]), "torn cache entry"


def test_c5_full_size_served(hm, wl):
    """The served configuration: 2^27 u32 words, 2^21 requests arriving
    Poisson at 3e7/s, lognormal lengths (median 4, max 64), 5% hot words,
    2 GiB admission budget, continuous batching; the whole run replays on
    the oracle round by round."""
    from test_gpu_serve import replay_served
    N = 1 << 27
    host_lo = N - N // 16
    g = wl.rng("c5", 0, 3)
    init = g.integers(0, 2 ** 32, size=N, dtype=np.uint64).astype(np.uint32)
    req = wl.c5_requests(g, 1 << 21, 3e7, n_words=N, host_lo=host_lo)
    hlog = wl.host_log_uniform(np.random.default_rng(5), 1 << 22, host_lo, N, 0, shuffle_ts=False)
    ctx = hm.Context(N, 4, 64, init=init, max_ops=64, batch_capacity=1 << 20, log_capacity=1 << 16, mode=1,
                     async_merge=True)
    host_t = hm.pinned(N * 4)
    host_t.numpy()[:] = init.view(np.uint8)
    out = ctx.serve(req["arrival_s"], req["batch"], host_t, hlog, 1 << 16, 1 << 20, 2 << 30, True)
    say(f"c5 full: rounds={out['rounds']} p50={out['p50_latency_us']:.0f}us p99={out['p99_latency_us']:.0f}us")
    assert out["served"] == 1 << 21
    S, res = replay_served(init, req["batch"], out, hlog, 1 << 16, 64)
    assert np.array_equal(out["results"], res)
    assert np.array_equal(ctx.read_state(hm.HETM_STATE_STMR), S)
    assert np.array_equal(host_t.numpy().view(np.uint32), S)
    ctx.close()
