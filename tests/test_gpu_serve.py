"""Serving (hetm_serve): open-loop arrivals, continuous batching over the
double-buffered round, admission into the running round (round period),
re-queue on conflict.  Oracle parity of a whole
served run, and probe requests whose results are the same alone and in the
mix (tolerance 0)."""
import numpy as np
import pytest

import oracle as orc
from gpu_util import say

pytestmark = pytest.mark.gpu

N = 1 << 20
HOST_LO = N - N // 16


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


def host_stream(wl, seed, n, lo, hi, inject_every=0, gpu_hi=HOST_LO):
    """The host's log stream: uniform words in [lo, hi), increasing ts; with
    inject_every > 0 every inject_every-th entry lands in the GPU range."""
    log = wl.host_log_uniform(np.random.default_rng(seed), n, lo, hi, 0, shuffle_ts=False)
    if inject_every:
        k = np.arange(0, n, inject_every)      # one write into the GPU's hot words every few rounds
        log["word"][k] = np.random.default_rng(seed + 1).integers(0, 1000, size=k.shape[0]).astype(np.uint32)
    return log


def replay_served(init, batch, out, log, per_round, G):
    """Oracle: round by round, the committed requests of the round in ticket
    order, then the round's host log chunk (serialized before the GPU's
    transactions by validation; the sets are disjoint when the round
    commits, so the order inside the round does not change any result)."""
    S = init.copy()
    TS = np.zeros(S.shape[0], np.uint64)
    res_all = np.zeros_like(out["results"])
    seq = out["commit_seq"]
    rnd = (seq >> np.uint64(32)).astype(np.int64)
    start = 0
    for r in range(int(out["rounds"])):
        end = int(out["round_log_end"][r])
        if not out["round_conflict"][r]:
            ids = np.flatnonzero(rnd == r)
            ids = ids[np.argsort(seq[ids] & np.uint64(0xFFFFFFFF), kind="stable")]
            sub = _subset(batch, ids)
            res, _, _ = orc.replay_oplist(S, G, sub, np.arange(ids.shape[0]))
            o = 0
            for k, i in enumerate(ids):
                L = int(batch.offsets[i + 1] - batch.offsets[i])
                res_all[batch.offsets[i]:batch.offsets[i] + L] = res[o:o + L]
                o += L
        else:
            assert not np.any(rnd == r)
        if end > start:
            orc.apply(S, TS, log[start:end], 0)
        start = end
    return S, res_all


def _subset(b, ids):
    from paper_1905_00661_amd import workloads as wl
    lens = (b.offsets[ids + 1] - b.offsets[ids]).astype(np.uint64)
    idx = np.concatenate([b.idx[b.offsets[i]:b.offsets[i + 1]] for i in ids]) if len(ids) else np.zeros(0, np.uint32)
    off = np.zeros(len(ids) + 1, np.uint32)
    off[1:] = np.cumsum(lens)
    return wl.OplistBatch(offsets=off, idx=idx.astype(np.uint32), n_writes=b.n_writes[ids].copy(), tid=b.tid[ids].copy())


def make_ctx(hm, init, pipelined, G=64, max_batch=8192):
    if pipelined:
        return hm.Context(N, 4, G, init=init, max_ops=64, batch_capacity=max_batch, log_capacity=4096, mode=1,
                          async_merge=True)
    return hm.Context(N, 4, G, init=init, max_ops=64, batch_capacity=max_batch, log_capacity=4096, mode=0)


@pytest.mark.parametrize("pipelined,rate,inject,early,period", [
    (True, 2e6, 0, False, 0), (False, 2e6, 0, False, 0), (False, 5e5, 3 * 4096, False, 0), (True, 2e7, 0, False, 0),
    (True, 5e5, 3 * 4096, False, 0), (True, 2e6, 0, True, 0), (True, 5e5, 3 * 4096, True, 0),
    (True, 2e7, 997, True, 0), (True, 2e6, 0, False, 400), (True, 2e7, 0, False, 1000),
    (True, 5e5, 3 * 4096, False, 600), (True, 2e7, 997, True, 500)])
def test_serve_matches_oracle(hm, wl, pipelined, rate, inject, early, period):
    """20,000 lognormal-length requests (median 4, capped at 64) arriving
    Poisson at `rate`, 5% hot words, host log stream of 4096 entries per
    round in the host's region (plus injected inter-device conflicts).  With
    `early` the rounds are streamed: the host ships its writes in pieces
    (1000 entries) while the GPU runs, each early-validated.  With a round
    `period` (µs) the requests that arrive while a round is open join it as
    further batches."""
    g = wl.rng("c5", 0, 3)
    init = g.integers(0, 2 ** 32, size=N, dtype=np.uint64).astype(np.uint32)
    req = wl.c5_requests(g, 20000, rate, n_words=N, host_lo=HOST_LO)
    log = host_stream(wl, 5, 1 << 20, HOST_LO, N, inject_every=inject)
    ctx = make_ctx(hm, init, pipelined)
    host_t = hm.pinned(N * 4)
    host_t.numpy()[:] = init.view(np.uint8)
    out = ctx.serve(req["arrival_s"], req["batch"], host_t, log, 4096, 8192, 64 << 20, pipelined,
                    early_validation=early, push_entries=1000 if early else 0, round_period_us=period)
    say(f"serve pipelined={pipelined} early={early} period={period} rate={rate:g}: rounds={out['rounds']} "
        f"batches={out['batches']} conflicted={out['conflicted_rounds']} "
        f"p50={out['p50_latency_us']:.0f}us p99={out['p99_latency_us']:.0f}us thr={out['throughput']:.3g}/s")
    assert out["served"] == 20000
    if period:
        assert out["batches"] > out["rounds"], "no round took a second batch"
    else:
        assert out["batches"] == out["rounds"]
    if inject:
        assert out["conflicted_rounds"] > 0 and out["requeued"] > 0
    S, res = replay_served(init, req["batch"], out, log, 4096, 64)
    assert np.array_equal(out["results"], res), "request results differ from the oracle replay"
    assert np.array_equal(ctx.read_state(hm.HETM_STATE_STMR), S)
    assert np.array_equal(host_t.numpy().view(np.uint32), S)
    assert np.all(out["latency_us"] > 0)
    ctx.close()


@pytest.mark.parametrize("pipelined", [True, False])
def test_serve_twice_on_one_context(hm, wl, pipelined):
    """Two serve calls on one context, the second with the host log moved
    later in time: each call matches the oracle replay continued from the
    state the previous call left, and both replicas agree after each."""
    g = wl.rng("c5", 0, 3)
    init = g.integers(0, 2 ** 32, size=N, dtype=np.uint64).astype(np.uint32)
    req = wl.c5_requests(g, 20000, 2e7, n_words=N, host_lo=HOST_LO)
    log = host_stream(wl, 5, 1 << 20, HOST_LO, N)
    ctx = make_ctx(hm, init, pipelined)
    host_t = hm.pinned(N * 4)
    host_t.numpy()[:] = init.view(np.uint8)
    S = init
    for call in range(2):
        lg = log.copy()
        lg["ts"] += np.uint64(call << 40)
        out = ctx.serve(req["arrival_s"], req["batch"], host_t, lg, 4096, 8192, 64 << 20, pipelined)
        say(f"serve call {call} pipelined={pipelined}: rounds={out['rounds']} p99={out['p99_latency_us']:.0f}us")
        assert out["served"] == 20000
        S, res = replay_served(S, req["batch"], out, lg, 4096, 64)
        assert np.array_equal(out["results"], res), f"call {call}: request results differ from the oracle replay"
        assert np.array_equal(ctx.read_state(hm.HETM_STATE_STMR), S)
        assert np.array_equal(host_t.numpy().view(np.uint32), S)
    ctx.close()


@pytest.mark.parametrize("pipelined,period", [(False, 0), (True, 0), (True, 800)])
def test_serve_starvation_guard(hm, wl, pipelined, period):
    """Every host log chunk writes a hot GPU word, so every round with host
    writes aborts; with a starvation limit of 2 the guard runs a round
    without host writes after two losses in a row, the GPU makes progress,
    and the whole run still matches the oracle replay."""
    g = wl.rng("c5", 2, 3)
    init = g.integers(0, 2 ** 32, size=N, dtype=np.uint64).astype(np.uint32)
    req = wl.c5_requests(g, 6000, 1e6, n_words=N, host_lo=HOST_LO)
    log = host_stream(wl, 21, 1 << 18, HOST_LO, N, inject_every=64)
    ctx = make_ctx(hm, init, pipelined)
    host_t = hm.pinned(N * 4)
    host_t.numpy()[:] = init.view(np.uint8)
    out = ctx.serve(req["arrival_s"], req["batch"], host_t, log, 4096, 8192, 64 << 20, pipelined, starvation_limit=2,
                    round_period_us=period)
    say(f"starvation guard pipelined={pipelined}: rounds={out['rounds']} conflicted={out['conflicted_rounds']} "
        f"starved={out['starved_rounds']}")
    assert out["served"] == 6000
    assert out["starved_rounds"] > 0 and out["conflicted_rounds"] > 0
    S, res = replay_served(init, req["batch"], out, log, 4096, 64)
    assert np.array_equal(out["results"], res)
    assert np.array_equal(ctx.read_state(hm.HETM_STATE_STMR), S)
    assert np.array_equal(host_t.numpy().view(np.uint32), S)
    ctx.close()


@pytest.mark.parametrize("period", [0, 500])
def test_serve_alone_vs_mix(hm, wl, period):
    """Probe requests each touch 4 private words no other request touches:
    their results and final words are identical served alone and served
    inside a 20,000-request mix (tolerance 0), also when the mix's rounds
    take requests that arrive while they run (a round period)."""
    P0 = HOST_LO - 4096
    n_probe = 512
    g = wl.rng("c5", 1, 3)
    init = g.integers(0, 2 ** 32, size=N, dtype=np.uint64).astype(np.uint32)
    probe_idx = (P0 + np.arange(n_probe * 4)).astype(np.uint64)
    probes = wl._oplist_from_lists(np.full(n_probe, 4, np.uint64), np.full(n_probe, 2), probe_idx, 10 ** 6)
    mix = wl.c5_requests(g, 20000, 4e6, n_words=N, host_lo=P0)     # the mix stays below the probes
    log = host_stream(wl, 9, 1 << 20, HOST_LO, N)

    def run(arr, batch, period=0):
        ctx = make_ctx(hm, init, True)
        host_t = hm.pinned(N * 4)
        host_t.numpy()[:] = init.view(np.uint8)
        out = ctx.serve(arr, batch, host_t, log, 1024, 4096, 32 << 20, True, round_period_us=period)
        S = ctx.read_state(hm.HETM_STATE_STMR).copy()
        ctx.close()
        return out, S

    t_probe = np.sort(np.random.default_rng(3).uniform(0, 0.004, n_probe))
    alone, S_alone = run(t_probe, probes)
    # interleave probes with the mix by arrival time
    arr = np.concatenate([mix["arrival_s"], t_probe])
    order = np.argsort(arr, kind="stable")
    mb = mix["batch"]
    allb = wl.OplistBatch(offsets=np.concatenate([mb.offsets, mb.offsets[-1] + probes.offsets[1:]]).astype(np.uint32),
                          idx=np.concatenate([mb.idx, probes.idx]), n_writes=np.concatenate([mb.n_writes, probes.n_writes]),
                          tid=np.concatenate([mb.tid, probes.tid]))
    sub = _subset(allb, order)
    mixed, S_mixed = run(arr[order], sub, period)
    if period:
        assert mixed["batches"] > mixed["rounds"]
    pos = np.flatnonzero(order >= mix["arrival_s"].shape[0])            # probes inside the mixed request list
    assert pos.shape[0] == n_probe
    got = np.concatenate([mixed["results"][sub.offsets[p]:sub.offsets[p + 1]] for p in pos])
    assert np.array_equal(got, alone["results"])
    assert np.array_equal(S_mixed[P0:P0 + 4 * n_probe], S_alone[P0:P0 + 4 * n_probe])
    say(f"alone p99={alone['p99_latency_us']:.0f}us  mixed p99={mixed['p99_latency_us']:.0f}us rounds={mixed['rounds']}")
