"""The OPLIST batch split into read-only and update lists: batches of one
kind only, kinds clustered across several partition tiles (4096
transactions each), and malformed transactions, against the oracle."""
from __future__ import annotations

import numpy as np
import pytest

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


FORMS = {"plain": (0, False), "graph": (1, False), "graph_async": (1, True)}


def _batch_inputs(wl, case: str, seed: int):
    """A round whose batch has the kind layout named by `case`; hot words
    make lanes of both kinds meet on the same slots.  The GPU's words are
    the low half, the host log's the high half: no inter-device conflict,
    so every transaction must commit."""
    N, G = 1 << 14, 16
    g = np.random.default_rng(seed)
    init = g.integers(0, 2 ** 32, size=N, dtype=np.uint64).astype(np.uint32)
    if case == "all_read_only":
        kinds = np.zeros(5000, bool)
    elif case == "all_update":
        kinds = np.ones(5000, bool)
    else:   # read-only, then updates, then read-only again: tiles of skewed kinds
        kinds = np.concatenate([np.zeros(6000, bool), np.ones(3000, bool), np.zeros(500, bool)])
    n = kinds.shape[0]
    lens = g.integers(1, 17, size=n).astype(np.uint64)
    nws = np.where(kinds, [g.integers(1, min(int(L), 8) + 1) for L in lens], 0).astype(np.int64)
    hot = g.integers(0, N // 2, size=64)
    idx = g.integers(0, N // 2, size=int(lens.sum()), dtype=np.uint64)
    pick = g.random(idx.shape[0]) < 0.3
    idx[pick] = hot[g.integers(0, hot.shape[0], size=int(pick.sum()))]
    batch = wl._oplist_from_lists(lens, nws, idx, 0)
    log = wl.host_log_uniform(g, 3000, N // 2, N, 0)
    return wl.RoundInputs(cfg=case, n_words=N, word_bytes=4, granule=G, program=1, init=init, batch=batch, log=log)


@pytest.mark.parametrize("case", ["all_read_only", "all_update", "clustered"])
@pytest.mark.parametrize("form", list(FORMS))
def test_kind_layouts(hm, wl, case, form):
    """Every transaction commits exactly once whichever lists hold it, and the
    round matches the oracle replayed in the GPU's commit order."""
    ri = _batch_inputs(wl, case, seed=len(case) * 7 + len(form))
    mode, am = FORMS[form]
    say(f"kinds case={case} form={form} n={ri.batch.n}")
    g = gpu_round(ri, mode=mode, async_merge=am)
    assert g["res"].conflict == 0 and int(g["res"].n_committed) == ri.batch.n
    o = oracle_round(ri, g["tickets"], g["H0"])
    assert_round_equal(g, o, ri)


@pytest.mark.parametrize("fault", ["writes_over_length", "writes_over_buffer", "length_over_max_ops",
                                   "word_outside"])
@pytest.mark.parametrize("form", list(FORMS))
def test_malformed_transaction(hm, wl, fault, form):
    """A malformed transaction makes the round fail with HETM_EINVAL and its
    index; the round is discarded (the transactions that committed on the
    GPU are undone: the GPU replica equals the host replica again), and the
    context serves a good round after."""
    import torch
    N, G, n, bad = 4096, 16, 300, 211
    g = np.random.default_rng(5)
    init = g.integers(0, 2 ** 32, size=N, dtype=np.uint64).astype(np.uint32)
    lens = g.integers(1, 9, size=n).astype(np.uint64)
    nws = np.array([g.integers(0, min(int(L), 8) + 1) for L in lens], dtype=np.int64)
    if fault == "writes_over_length":
        lens[bad], nws[bad] = 2, 3
    elif fault == "writes_over_buffer":
        lens[bad], nws[bad] = 12, 9
    elif fault == "length_over_max_ops":
        lens[bad], nws[bad] = 17, 1
    idx = g.integers(0, N, size=int(lens.sum()), dtype=np.uint64)
    if fault == "word_outside":
        idx[int(lens[:bad].sum())] = N
    batch = wl._oplist_from_lists(lens, nws, idx, 0)
    say(f"malformed fault={fault} at {bad}")
    mode, am = FORMS[form]
    ctx = hm.Context(N, 4, G, init=init, max_ops=16, batch_capacity=n, log_capacity=16, mode=mode, async_merge=am)
    b = hm.Batch(hm.HETM_PROG_OPLIST, batch, ctx.dev)
    host_t = hm.pinned(N * 4)
    host_t.numpy()[:] = init.view(np.uint8)
    empty_log = torch.zeros(16, dtype=torch.uint8, device=ctx.dev)
    with pytest.raises(hm.HetmError) as e:
        ctx.round(b, empty_log, 0, host_t)
    assert e.value.code == hm.HETM_EINVAL
    assert f"index {bad}" in str(e.value)
    assert np.array_equal(ctx.read_state(hm.HETM_STATE_STMR), init)
    assert not ctx.read_state(hm.HETM_STATE_RS).any() and not ctx.read_state(hm.HETM_STATE_WS).any()
    # a good round on the same context afterwards
    ok_lens = np.full(64, 4, np.uint64)
    ok = wl._oplist_from_lists(ok_lens, np.full(64, 1, np.int64), g.integers(0, N, size=256, dtype=np.uint64), 0)
    b2 = hm.Batch(hm.HETM_PROG_OPLIST, ok, ctx.dev)
    r = ctx.round(b2, empty_log, 0, host_t)
    assert int(r.n_committed) == 64 and r.error == 0 and r.conflict == 0
    ctx.sync()
    assert np.array_equal(ctx.read_state(hm.HETM_STATE_STMR), host_t.numpy().view(np.uint32))
    ctx.close()
