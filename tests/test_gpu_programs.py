"""GPU parity for the TRANSFER (bank accounts, int64 words) and CACHE (object
cache) programs, with host logs produced by the host TM threads, and
workload invariants: total balance conserved, no torn cache entries."""
import numpy as np
import pytest

import oracle as orc
from gpu_util import assert_round_equal, gpu_round, oracle_round, say

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


def transfer_round(hm, wl, n_accounts, host_accounts, n_txn, n_host, steal, G, stripe=1, mode=0, seed_round=0):
    d = wl.c3(n_accounts=n_accounts, host_accounts=host_accounts, n_txn=n_txn, n_host=n_host, steal=steal,
              round_no=seed_round)
    H = d["init"].copy()
    tm = hm.HostTM(H, stripe=1, ts_start=0)
    ts, log = tm.transfers(d["host"].src, d["host"].dst, d["host"].amt, threads=4)
    tm.close()
    ri = wl.RoundInputs(cfg="c3", n_words=n_accounts, word_bytes=8, granule=G, program=wl.PROG_TRANSFER,
                        init=d["init"], batch=d["batch"], log=log)
    g = gpu_round(ri, host=H, stripe=stripe, mode=mode)
    o = oracle_round(ri, g["tickets"], H)
    return ri, g, o


@pytest.mark.parametrize("steal,G,stripe,mode", [(0.0, 16, 1, 0), (0.0, 1, 1, 1), (0.001, 64, 4, 0),
                                                 (0.0, 4096, 1, 1)])
def test_transfer_round(hm, wl, steal, G, stripe, mode):
    """Bank transfers, Zipf(0.9) accounts: 2^18 accounts, 2^16 GPU transfers,
    the host's 2^13 transfers over its own 2^12 accounts; 'steal' sends a
    fraction of GPU transfers into the host's accounts (inter-device
    conflicts, CPU wins)."""
    say(f"transfer steal={steal} G={G} S={stripe} mode={mode}")
    ri, g, o = transfer_round(hm, wl, 1 << 18, 1 << 12, 1 << 16, 1 << 13, steal, G, stripe, mode)
    assert_round_equal(g, o, ri)
    assert int(g["S"].sum()) == 1000 * (1 << 18), "total balance not conserved"
    assert g["S"].min() >= 0
    if steal:
        assert o["conflict"] == 1
    say(f"  retries={g['res'].n_local_retries} dirty={g['res'].n_dirty}")


def test_transfer_hot_accounts(hm, wl):
    """Every transfer among 64 accounts: extreme local contention."""
    g0 = np.random.default_rng(8)
    n = 8192
    src = g0.integers(0, 64, size=n, dtype=np.uint64)
    dst = (src + g0.integers(1, 64, size=n, dtype=np.uint64)) % 64
    b = wl.TransferBatch(src=src.astype(np.uint32), dst=dst.astype(np.uint32),
                         amt=g0.integers(1, 101, size=n, dtype=np.uint64).astype(np.uint32))
    log = np.zeros(0, wl.LOG8_DTYPE)
    ri = wl.RoundInputs(cfg="c3hot", n_words=1024, word_bytes=8, granule=1, program=wl.PROG_TRANSFER,
                        init=np.full(1024, 1000, np.int64), batch=b, log=log)
    g = gpu_round(ri, host=ri.init.copy())
    o = oracle_round(ri, g["tickets"], ri.init.copy())
    assert_round_equal(g, o, ri)
    assert int(g["S"].sum()) == 1000 * 1024
    say(f"hot accounts: retries={g['res'].n_local_retries}")


def test_transfer_uneven_batches(hm, wl):
    """One round fed by several batches of uneven size (the device queue is
    refilled per batch); tickets continue across batches."""
    import torch
    d = wl.c3(n_accounts=1 << 16, host_accounts=1 << 10, n_txn=50000, n_host=2000)
    H = d["init"].copy()
    tm = hm.HostTM(H)
    _, log = tm.transfers(d["host"].src, d["host"].dst, d["host"].amt)
    tm.close()
    N = 1 << 16
    ctx = hm.Context(N, 8, 8, init=d["init"], batch_capacity=50000, log_capacity=log.shape[0])
    cuts = [0, 1, 77, 4096, 4097, 20000, 50000]
    parts, tickets, results = [], [], []
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        sub = wl.TransferBatch(src=d["batch"].src[lo:hi].copy(), dst=d["batch"].dst[lo:hi].copy(),
                               amt=d["batch"].amt[lo:hi].copy())
        bt = hm.Batch(hm.HETM_PROG_TRANSFER, sub)
        ctx.submit(bt)
        parts.append(bt)
    for bt in parts:
        tickets.append(bt.tickets_np())
        r = bt.results_np().reshape(3, -1)
        results.append(r)
    log_t = hm.to_device(log)
    c = ctx.validate_apply(log_t, log.shape[0])
    host_t = hm.pinned(H.nbytes)
    host_t.numpy()[:] = H.view(np.uint8)
    ctx.copyback(hm.HETM_OUTCOME_DEVICE, host_t)
    order = orc.order_from_tickets(np.concatenate(tickets))
    S, Ho, TS = d["init"].copy(), H.copy(), np.zeros(N, np.uint64)
    out = orc.round_generic(orc.replay_transfer, S, Ho, TS, 8, d["batch"], order, log, 0)
    assert c == out["conflict"] == 0
    assert np.array_equal(np.concatenate(results, axis=1).reshape(-1), out["results"])
    assert np.array_equal(ctx.read_state(hm.HETM_STATE_STMR), S)
    assert np.array_equal(host_t.numpy().view(np.int64), Ho)
    ctx.close()


def _cache_invariants(S, nsets):
    sets = S.reshape(nsets, 128)
    keys = sets[:, 0:16].reshape(nsets, 8, 2).astype(np.uint64)
    keys = keys[:, :, 0] | (keys[:, :, 1] << np.uint64(32))
    vals = sets[:, 32:96].reshape(nsets, 8, 8)
    full = keys != 0
    chk = np.array([orc.mix64(int(k)) & 0xFFFFFFFF for k in keys[full]], dtype=np.uint32)
    x = np.bitwise_xor.reduce(vals[full][:, :7], axis=1) ^ chk
    assert np.array_equal(x, vals[full][:, 7]), "torn cache entry"
    ks = np.sort(np.where(full, keys, 0), axis=1)
    dup = (ks[:, 1:] == ks[:, :-1]) & (ks[:, 1:] != 0)
    assert not dup.any(), "duplicate key in a set"
    return int(full.sum())


@pytest.mark.parametrize("steal,stripe,G,mode", [(False, 1, 128, 0), (False, 128, 16, 1), (True, 1, 128, 0)])
def test_cache_round(hm, wl, steal, stripe, G, mode):
    """The object cache: 2^12 sets x 8 ways warmed by host PUTs, then 2^15
    GPU GET/PUT requests (95/5, Zipf 0.99 over 2^16 keys, even keys) while
    the host PUTs odd keys; 'steal' lets the GPU touch odd keys too."""
    nsets = 1 << 12
    N = nsets * 128
    g0 = wl.rng("c4", 0, 2)
    warm = np.zeros(N, np.uint32)
    tm = hm.HostTM(warm, stripe=128)
    wk = g0.permutation(np.arange(1, 1 << 16, dtype=np.uint64))[: int(nsets * 8 * 0.95)]
    tm.cache_puts(wk, threads=4)
    clock = tm.clock
    tm.close()
    b = wl.c4_requests(g0, 1 << 15, 1 << 16, theta=0.99, put_frac=0.05, parity=None if steal else 0,
                       tid0=clock + 100000)
    H = warm.copy()
    tm = hm.HostTM(H, stripe=128, ts_start=clock)
    hk = wl.c4_requests(g0, 1 << 11, 1 << 16, theta=0.99, put_frac=1.0, parity=1).key
    _, log = tm.cache_puts(hk, threads=4)
    tm.close()
    ri = wl.RoundInputs(cfg="c4", n_words=N, word_bytes=4, granule=G, program=wl.PROG_CACHE, init=warm, batch=b,
                        log=log)
    say(f"cache steal={steal} S={stripe} G={G} mode={mode}")
    g = gpu_round(ri, host=H, stripe=stripe, mode=mode)
    o = oracle_round(ri, g["tickets"], H)
    assert_round_equal(g, o, ri)
    assert _cache_invariants(g["S"], nsets) > 0
    r = g["results"].reshape(-1, 9)
    say(f"  hits={(r[:, 0] & 0x100).astype(bool).sum()} conflict={o['conflict']} retries={g['res'].n_local_retries}")
    if steal:
        assert o["conflict"] == 1
