"""The workgroup tuner on the GPU: it times whole rounds of the small
configuration at widths around one workgroup per compute unit, leaves the
context at a width among them, and a round at that width still matches
the oracle bit for bit."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_util import assert_round_equal, gpu_round, oracle_round, say

pytestmark = pytest.mark.gpu


def test_tuned_width_is_valid_and_correct(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_00661_amd import autotune
    from paper_1905_00661_amd import hetm as hm
    from paper_1905_00661_amd import workloads as wl
    ri = wl.c1("p")
    ctx = hm.Context(ri.n_words, 4, ri.granule, init=ri.init, batch_capacity=ri.batch.n, log_capacity=ri.log.shape[0],
                     mode=hm.HETM_MODE_GRAPH, async_merge=True)
    b = hm.Batch(ri.program, ri.batch, ctx.dev)
    base = hm.to_device(ri.log, ctx.dev)
    log_t = base.clone()
    n_log = ri.log.shape[0]
    host = hm.pinned(ri.n_words * 4)
    S = ri.init.copy()
    shift = [0]

    def run_round():
        # the host replica tracks the GPU's after every round (no conflicts:
        # GPU words in the lower half, log in the upper)
        lg = ri.log.copy()
        lg["ts"] += np.uint64(shift[0])
        host.numpy()[:] = wl.host_replica(ctx.read_state(hm.HETM_STATE_STMR), lg).view(np.uint8)
        log_t.copy_(base)
        log_t.view(torch.int64).view(-1, 2)[:, 1].add_(shift[0])
        shift[0] += n_log
        r = ctx.round(b, log_t, n_log, host)
        assert r.conflict == 0 and r.error == 0

    cache = autotune.TuneCache(str(tmp_path / "t.json"))
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    res = autotune.tune_exec_workgroups(ctx.set_exec_workgroups, run_round, cus, sig="c1p", cache=cache, repeats=1,
                                        sync=lambda: (ctx.sync(), torch.cuda.synchronize()))
    say(f"tuned: {res['exec_workgroups']} workgroups; table {[(r['exec_workgroups'], r['median_s']) for r in res['table']]}")
    assert res["exec_workgroups"] in autotune.candidates_for(cus)
    assert cache.get("c1p")["exec_workgroups"] == res["exec_workgroups"]
    # one more round at the tuned width, checked against the oracle
    ctx.sync()
    S = ctx.read_state(hm.HETM_STATE_STMR).copy()
    lg = ri.log.copy()
    lg["ts"] += np.uint64(shift[0])
    rk = wl.RoundInputs(cfg="tuned", n_words=ri.n_words, word_bytes=4, granule=ri.granule, program=ri.program,
                        init=S, batch=ri.batch, log=lg)
    H0 = wl.host_replica(S, lg)
    out = gpu_round(rk, ctx=ctx, host=H0, keep=True)
    o = oracle_round(rk, out["tickets"], H0, S0=S, floor=shift[0])
    assert_round_equal(out, o, rk)
    ctx.close()
