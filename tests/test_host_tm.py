"""The host TM threads (libhetm, C++): their concurrent result and log equal
a serial replay of the same transactions in commit-timestamp order by the
oracle, and the log satisfies the paper's instrumentation contract
(timestamps totally order the updates of each word).  CPU only."""
import numpy as np
import pytest

import oracle as orc
from paper_1905_00661_amd import workloads as wl


@pytest.fixture(scope="module")
def hm():
    from paper_1905_00661_amd import hetm
    hetm.lib()
    return hetm


def _sorted(log):
    return log[np.lexsort((log["word"], log["ts"]))]


@pytest.mark.parametrize("threads,stripe", [(1, 1), (4, 1), (8, 4)])
def test_host_transfers_equal_serial_replay(hm, threads, stripe):
    d = wl.c3(n_accounts=1 << 12, host_accounts=1 << 6, n_txn=10, n_host=20000)
    H = d["init"].copy()
    tm = hm.HostTM(H, stripe=stripe, ts_start=777)
    b = d["host"]
    ts, log = tm.transfers(b.src, b.dst, b.amt, threads=threads)
    assert sorted(ts.tolist()) == list(range(778, 778 + b.n))
    assert tm.clock == 777 + b.n
    assert int(H.sum()) == 1000 * (1 << 12) and H.min() >= 0
    o = np.argsort(ts)
    R = d["init"].copy()
    sb = wl.TransferBatch(src=b.src[o].copy(), dst=b.dst[o].copy(), amt=b.amt[o].copy())
    olog = orc.host_transfers(R, sb, ts[o])
    assert np.array_equal(R, H)
    assert np.array_equal(_sorted(log), _sorted(olog))
    # the log applied to the initial replica reproduces the host replica
    S = d["init"].copy()
    orc.apply(S, np.zeros(S.shape[0], np.uint64), log, 777)
    assert np.array_equal(S, H)
    tm.close()


def test_host_cache_puts_equal_serial_replay(hm):
    nsets = 64
    H = np.zeros(nsets * 128, np.uint32)
    keys = (np.random.default_rng(3).integers(1, 500, size=3000, dtype=np.uint64) * 2 + 1)
    tm = hm.HostTM(H, stripe=128, ts_start=10)
    ts, log = tm.cache_puts(keys, threads=4)
    assert log.shape[0] == 12 * keys.shape[0]
    o = np.argsort(ts)
    R = np.zeros_like(H)
    olog = orc.host_cache_puts(R, keys[o], ts[o])
    assert np.array_equal(R, H)
    assert np.array_equal(_sorted(log), _sorted(olog))
    tm.close()


def test_host_tm_rejects_bad_input(hm):
    H = np.zeros(16, np.int64)
    tm = hm.HostTM(H)
    with pytest.raises(hm.HetmError):
        tm.transfers([0], [99], [1])
    tm.close()
