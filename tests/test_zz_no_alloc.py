"""hetm_read_words_noalloc, the read of the replica's values that allocates
nothing, against hetm_read_state(STMR) on the same context: two calls in a
row (the second over a smaller range at another offset, so what the first
left in the shared device array would show if it were read back), every
layout, the largest range one call takes, and the limits it rejects."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

from gpu_util import gpu_round, say

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


def _read(hm, ctx, first, n, where):
    """Reads n words from `first` into a fresh buffer of kind `where`."""
    import torch
    W = ctx.word_bytes
    dt = np.uint32 if W == 4 else np.int64
    if where == "device":
        t = torch.full((max(n * W, 1),), 0xAB, dtype=torch.uint8, device="cuda")
        hm.hetm_read_words_noalloc(ctx.ctx, first, n, t.data_ptr())
        return t.cpu().numpy()[: n * W].view(dt)
    if where == "pinned":
        t = hm.pinned(n * W)
        t.numpy()[:] = 0xAB
        hm.hetm_read_words_noalloc(ctx.ctx, first, n, t.data_ptr())
        return t.numpy()[: n * W].view(dt).copy()
    buf = np.full(max(n * W, 1), 0xAB, np.uint8)
    hm.hetm_read_words_noalloc(ctx.ctx, first, n, buf.ctypes.data)
    return buf[: n * W].view(dt)


@pytest.mark.parametrize("stripe", [1, 4])
def test_matches_read_state_after_a_round(hm, wl, stripe):
    """After a whole round (values and versions changed; stripe 1 is the slot
    layout, stripe 4 a value array plus lock table): a full read, then a
    smaller one at an offset, each equal to hetm_read_state's values."""
    ri = wl.c1("", n_words=(1 << 16) + 37)
    say(f"noalloc: c1 round, stripe {stripe}, N {ri.n_words}")
    out = gpu_round(ri, stripe=stripe, keep=True)
    ctx = out["ctx"]
    ref = ctx.read_state(hm.HETM_STATE_STMR)
    assert not np.array_equal(ref, ri.init)          # the round changed the replica
    assert np.array_equal(ref, out["H"])             # and the replicas agree
    a = _read(hm, ctx, 0, ri.n_words, "device")
    assert np.array_equal(a, ref)
    first, n = 1001, ri.n_words // 3 + 7
    b = _read(hm, ctx, first, n, "pinned")
    assert np.array_equal(b, ref[first:first + n])
    c = _read(hm, ctx, ri.n_words - 5, 5, "host")
    assert np.array_equal(c, ref[-5:])
    ctx.close()


def test_u64_words(hm):
    """u64 words (a value array): two reads in a row against read_state."""
    N = 50_003
    init = np.random.default_rng(3).integers(-2 ** 62, 2 ** 62, size=N, dtype=np.int64)
    ctx = hm.Context(N, 8, 16, init=init, batch_capacity=16, log_capacity=16)
    ref = ctx.read_state(hm.HETM_STATE_STMR)
    assert np.array_equal(ref, init)
    assert np.array_equal(_read(hm, ctx, 0, N, "device"), ref)
    assert np.array_equal(_read(hm, ctx, 77, 1000, "host"), ref[77:1077])
    ctx.close()


def test_largest_range_then_smaller(hm):
    """The largest range one call takes (2^24 words, slot layout, at an
    offset into a replica a little larger), then a smaller one."""
    M = 1 << 24
    N = M + 37
    init = np.random.default_rng(4).integers(0, 2 ** 32, size=N, dtype=np.uint64).astype(np.uint32)
    say(f"noalloc: largest range, N {N}")
    ctx = hm.Context(N, 4, 64, init=init, batch_capacity=16, log_capacity=16)
    ref = ctx.read_state(hm.HETM_STATE_STMR)
    assert np.array_equal(ref, init)
    assert np.array_equal(_read(hm, ctx, 37, M, "device"), ref[37:])
    assert np.array_equal(_read(hm, ctx, 5, 4099, "pinned"), ref[5:5 + 4099])
    ctx.close()


def test_limits_rejected(hm):
    """A range over the limit (ECAPACITY) or past the replica's end (EINVAL)
    copies nothing; an empty range is a no-op."""
    N = 4096
    init = np.arange(N, dtype=np.uint32)
    ctx = hm.Context(N, 4, 1, init=init, batch_capacity=16, log_capacity=16)
    L = hm.lib()
    buf = np.full(64, 0xCD, np.uint8)
    p = ctypes.c_void_p(buf.ctypes.data)
    assert L.hetm_read_words_noalloc(ctx.ctx, 0, (1 << 24) + 1, p) == hm.HETM_ECAPACITY
    assert b"limit" in L.hetm_last_error(ctx.ctx)
    assert L.hetm_read_words_noalloc(ctx.ctx, N - 3, 4, p) == hm.HETM_EINVAL
    assert L.hetm_read_words_noalloc(ctx.ctx, N + 1, 0, p) == hm.HETM_EINVAL
    assert L.hetm_read_words_noalloc(ctx.ctx, 0, 0, None) == hm.HETM_OK
    assert (buf == 0xCD).all()
    assert L.hetm_read_words_noalloc(ctx.ctx, N - 16, 16, p) == hm.HETM_OK
    assert np.array_equal(buf.view(np.uint32), init[-16:])
    ctx.close()
