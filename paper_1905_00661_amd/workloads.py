"""Seeded synthetic inputs for one SHeTM round.

This module only draws inputs: initial STMR images, GPU transaction
descriptors and host write logs.  It computes nothing the method computes
(no transaction execution, validation, apply or merge), so both the HIP path
and the CPU oracle can consume its output without sharing any arithmetic.

Workload shapes follow the paper's synthetic benchmarks (uniform W1/W2-style
read/update transactions, §V-A/§V-B), its contention injection into the CPU
write stream (§V-C) and its object-cache application (§V-D), at the sizes
of the five named configurations:

* ``c1``  plain single round, 2^16 u32 words, 4096 4R/4W transactions,
          10,000-entry host log, granule 64 words (variants ``w``: granule 1,
          ``p``: GPU and host touch disjoint halves).
* ``c2``  2^28 u32 words, 2^20 transactions (90% 16-read read-only, 10% 4R/4W
          update), 1% hot set drawing 0/50/90% of accesses, 2^20-entry host
          log with an injected inter-device conflict per round at rate r.
* ``c3``  bank transfers over 2^24 int64 accounts, Zipf(0.9) account draws.
* ``c4``  set-associative object cache, 2^22 sets x 8 ways, Zipf(0.99) keys.
* ``c5``  open-loop Poisson arrivals, lognormal lengths capped at 64 ops.

Every array is produced by ``numpy.random.Generator(PCG64)`` seeded from a
``SeedSequence`` over (base seed, config, round, stream), so any input can be
regenerated exactly from its coordinates.
"""
from __future__ import annotations

import dataclasses
import functools

import numpy as np

BASE_SEED = 0x190500661

# stream ids
_S_STMR, _S_TXN, _S_LOG, _S_ARRIVAL, _S_LEN, _S_HOST = range(6)
_CFG_IDS = {"c1": 1, "c1w": 1, "c1p": 11, "c2": 2, "c3": 3, "c4": 4, "c5": 5, "tiny": 9}

LOG4_DTYPE = np.dtype([("word", "<u4"), ("value", "<u4"), ("ts", "<u8")])
LOG8_DTYPE = np.dtype([("word", "<u4"), ("pad", "<u4"), ("value", "<u8"), ("ts", "<u8")])

PROG_OPLIST = 1
PROG_TRANSFER = 2
PROG_CACHE = 3

CACHE_GET = 0
CACHE_PUT = 1


def rng(cfg: str, round_no: int, stream: int, seed: int = BASE_SEED) -> np.random.Generator:
    ss = np.random.SeedSequence([seed & 0xFFFFFFFF, seed >> 32, _CFG_IDS.get(cfg, 99), round_no, stream])
    return np.random.Generator(np.random.PCG64(ss))


@dataclasses.dataclass
class OplistBatch:
    """A batch of OPLIST transactions in CSR form.

    ``offsets[i]..offsets[i+1]`` index ``idx`` for transaction i; its first
    ``n_writes[i]`` indices are also written (value read + ``tid[i]``)."""
    offsets: np.ndarray   # uint32 [n+1]
    idx: np.ndarray       # uint32 [offsets[-1]]
    n_writes: np.ndarray  # uint8  [n]
    tid: np.ndarray       # uint32 [n]

    @property
    def n(self) -> int:
        return int(self.n_writes.shape[0])

    def subset(self, lo: int, hi: int) -> "OplistBatch":
        o = self.offsets[lo:hi + 1]
        return OplistBatch(offsets=(o - o[0]).astype(np.uint32),
                           idx=self.idx[o[0]:o[-1]].copy(),
                           n_writes=self.n_writes[lo:hi].copy(), tid=self.tid[lo:hi].copy())


@dataclasses.dataclass
class TransferBatch:
    src: np.ndarray  # uint32 [n]
    dst: np.ndarray  # uint32 [n]
    amt: np.ndarray  # uint32 [n], in [1, 100]

    @property
    def n(self) -> int:
        return int(self.src.shape[0])


@dataclasses.dataclass
class CacheBatch:
    key: np.ndarray  # uint64 [n], nonzero
    op: np.ndarray   # uint8 [n], CACHE_GET / CACHE_PUT
    tid: np.ndarray  # uint32 [n]

    @property
    def n(self) -> int:
        return int(self.key.shape[0])


@dataclasses.dataclass
class RoundInputs:
    cfg: str
    n_words: int
    word_bytes: int
    granule: int
    program: int
    init: np.ndarray            # STMR image (uint32 or int64 words)
    batch: object               # OplistBatch / TransferBatch / CacheBatch
    log: np.ndarray             # LOG4_DTYPE or LOG8_DTYPE
    watermark: int = 0          # max host ts applied before this round
    meta: dict = dataclasses.field(default_factory=dict)


def _oplist_from_lists(lens: np.ndarray, nws: np.ndarray, flat_idx: np.ndarray, tid0: int) -> OplistBatch:
    n = lens.shape[0]
    offsets = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(lens, out=offsets[1:])
    assert offsets[-1] < 2 ** 32
    return OplistBatch(offsets=offsets.astype(np.uint32), idx=flat_idx.astype(np.uint32),
                       n_writes=nws.astype(np.uint8),
                       tid=(np.arange(n, dtype=np.uint64) + tid0 + 1).astype(np.uint32))


def host_log_uniform(g: np.random.Generator, n: int, lo: int, hi: int, watermark: int,
                     shuffle_ts: bool = True) -> np.ndarray:
    """Host write log of ``n`` entries at uniform words in [lo, hi).

    Timestamps are the distinct values watermark+1 .. watermark+n, handed out
    in a random order so the log arrives in arbitrary order (§IV-C.2)."""
    log = np.zeros(n, dtype=LOG4_DTYPE)
    log["word"] = g.integers(lo, hi, size=n, dtype=np.uint64).astype(np.uint32)
    log["value"] = g.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
    ts = np.arange(1, n + 1, dtype=np.uint64) + np.uint64(watermark)
    if shuffle_ts:
        g.shuffle(ts)
    log["ts"] = ts
    return log


def host_replica(init: np.ndarray, log: np.ndarray) -> np.ndarray:
    """The host replica at the round cut: the host executed the logged writes
    itself, one after the other in timestamp order, so each word holds the
    value of its last write.  (This is the CPU side of the round, which
    produces the log; it is an input of the GPU round.)"""
    H = init.copy()
    o = np.argsort(log["ts"], kind="stable")[::-1]      # latest write first
    w = log["word"][o].astype(np.int64)
    uniq, first = np.unique(w, return_index=True)
    H[uniq] = log["value"][o][first]
    return H


# ----------------------------------------------------------------------------
# C1: plain single round, small
# ----------------------------------------------------------------------------

def c1(variant: str = "", seed: int = BASE_SEED, n_words: int = 1 << 16, n_txn: int = 4096,
       n_log: int = 10000, ops: int = 4) -> RoundInputs:
    """2^16 u32 words, 4096 transactions of 4 reads + 4 writes (write = read +
    tid), 10,000-entry host log, granule 64 words.  ``variant``: '' as named,
    'w' granule 1, 'p' GPU indices in the lower half and log in the upper."""
    cfg = "c1p" if variant == "p" else "c1"
    gs, gt, gl = rng(cfg, 0, _S_STMR, seed), rng(cfg, 0, _S_TXN, seed), rng(cfg, 0, _S_LOG, seed)
    init = gs.integers(0, 2 ** 32, size=n_words, dtype=np.uint64).astype(np.uint32)
    half = n_words // 2
    gpu_hi = half if variant == "p" else n_words
    flat = gt.integers(0, gpu_hi, size=n_txn * ops, dtype=np.uint64)
    lens = np.full(n_txn, ops, dtype=np.uint64)
    batch = _oplist_from_lists(lens, np.full(n_txn, ops), flat, 0)
    lo = half if variant == "p" else 0
    log = host_log_uniform(gl, n_log, lo, n_words, 0, shuffle_ts=True)
    granule = 1 if variant == "w" else 64
    return RoundInputs(cfg="c1" + variant, n_words=n_words, word_bytes=4, granule=granule,
                       program=PROG_OPLIST, init=init, batch=batch, log=log)


# ----------------------------------------------------------------------------
# C2: large synthetic STMR
# ----------------------------------------------------------------------------

def c2_batch(g: np.random.Generator, n_words: int, n_txn: int, p_hot: float,
             update_frac: float = 0.1, ro_reads: int = 16, upd_ops: int = 4,
             tid0: int = 0) -> OplistBatch:
    """90% read-only (16 reads) / 10% update (4 RMW) transactions over the GPU
    half [0, N/2) of the STMR; the hot set is the first 1% of the words and
    each access falls in it with probability ``p_hot``."""
    half = n_words // 2
    hot = max(1, int(0.01 * n_words))
    is_upd = g.random(n_txn) < update_frac
    lens = np.where(is_upd, upd_ops, ro_reads).astype(np.uint64)
    nws = np.where(is_upd, upd_ops, 0)
    total = int(lens.sum())
    hot_draw = g.random(total) < p_hot
    idx = np.where(hot_draw,
                   g.integers(0, hot, size=total, dtype=np.uint64),
                   g.integers(hot, half, size=total, dtype=np.uint64))
    return _oplist_from_lists(lens, nws, idx, tid0)


def c2(seed: int = BASE_SEED, n_words: int = 1 << 28, n_txn: int = 1 << 20, n_log: int = 1 << 20,
       p_hot: float = 0.5, conflict_rate: float = 0.0, granule: int = 64, round_no: int = 0,
       watermark: int = 0, batch: OplistBatch | None = None, init: bool = True,
       per_entry: bool = False) -> RoundInputs:
    """One round of the large synthetic configuration (sizes overridable for
    scaled-down tests).  Non-conflicting host writes land uniformly in the
    host half [N/2, N).  With probability ``conflict_rate`` per round one log
    entry is redirected to a word the batch reads (``per_entry``: every entry
    independently with that probability)."""
    gs, gt, gl = rng("c2", 0, _S_STMR, seed), rng("c2", round_no, _S_TXN, seed), rng("c2", round_no, _S_LOG, seed)
    img = gs.integers(0, 2 ** 32, size=n_words, dtype=np.uint64).astype(np.uint32) if init else None
    if batch is None:
        batch = c2_batch(gt, n_words, n_txn, p_hot, tid0=round_no * n_txn)
    log = host_log_uniform(gl, n_log, n_words // 2, n_words, watermark)
    injected = []
    if per_entry:
        hit = np.flatnonzero(gl.random(n_log) < conflict_rate)
    else:
        hit = np.array([int(gl.integers(0, n_log))]) if gl.random() < conflict_rate else np.zeros(0, np.int64)
    if hit.size:
        src = gl.integers(0, batch.idx.shape[0], size=hit.size)
        log["word"][hit] = batch.idx[src]
        injected = hit.tolist()
    return RoundInputs(cfg="c2", n_words=n_words, word_bytes=4, granule=granule, program=PROG_OPLIST,
                       init=img, batch=batch, log=log, watermark=watermark,
                       meta={"p_hot": p_hot, "conflict_rate": conflict_rate, "injected": injected})


# ----------------------------------------------------------------------------
# Zipf draws (exact inversion of the finite Zipf CDF)
# ----------------------------------------------------------------------------

@functools.lru_cache(maxsize=4)
def _zipf_cdf(n: int, theta: float) -> np.ndarray:
    w = np.arange(1, n + 1, dtype=np.float64) ** (-theta)
    c = np.cumsum(w)
    c /= c[-1]
    return c


def zipf_ranks(g: np.random.Generator, n: int, theta: float, size: int) -> np.ndarray:
    """0-based ranks with P(rank = r) proportional to (r+1)^-theta over [0, n)."""
    u = g.random(size)
    return np.minimum(np.searchsorted(_zipf_cdf(n, theta), u, side="left"), n - 1).astype(np.uint64)


# ----------------------------------------------------------------------------
# C3: bank transfers
# ----------------------------------------------------------------------------

def c3_batch(g: np.random.Generator, n_accounts: int, host_accounts: int, n_txn: int,
             theta: float = 0.9, steal: float = 0.0) -> TransferBatch:
    """Transfers between two Zipf(theta)-drawn accounts of the GPU range
    [host_accounts, n_accounts); rank r maps to account host_accounts + r.
    dst is redrawn until it differs from src.  With probability ``steal`` a
    transfer draws its accounts in the host range instead."""
    span = n_accounts - host_accounts
    src = zipf_ranks(g, span, theta, n_txn)
    dst = zipf_ranks(g, span, theta, n_txn)
    same = src == dst
    while same.any():
        dst[same] = zipf_ranks(g, span, theta, int(same.sum()))
        same = src == dst
    src += host_accounts
    dst += host_accounts
    if steal > 0:
        st = g.random(n_txn) < steal
        k = int(st.sum())
        s2 = g.integers(0, host_accounts, size=k, dtype=np.uint64)
        d2 = g.integers(0, host_accounts - 1, size=k, dtype=np.uint64)
        d2 = d2 + (d2 >= s2)
        src[st], dst[st] = s2, d2
    amt = g.integers(1, 101, size=n_txn, dtype=np.uint64)
    return TransferBatch(src=src.astype(np.uint32), dst=dst.astype(np.uint32), amt=amt.astype(np.uint32))


def c3_host_transfers(g: np.random.Generator, host_accounts: int, n: int) -> TransferBatch:
    s = g.integers(0, host_accounts, size=n, dtype=np.uint64)
    d = g.integers(0, host_accounts - 1, size=n, dtype=np.uint64)
    d = d + (d >= s)
    a = g.integers(1, 101, size=n, dtype=np.uint64)
    return TransferBatch(src=s.astype(np.uint32), dst=d.astype(np.uint32), amt=a.astype(np.uint32))


def c3(seed: int = BASE_SEED, n_accounts: int = 1 << 24, host_accounts: int = 1 << 16,
       n_txn: int | None = None, n_host: int = 1 << 15, theta: float = 0.9, round_no: int = 0,
       steal: float = 0.0) -> dict:
    """Bank-transfer inputs: accounts start at 1000; the GPU batch size is
    drawn uniformly in [2^20, 2^21] unless given; the host runs ``n_host``
    transfers over its own accounts [0, host_accounts)."""
    gt, gh = rng("c3", round_no, _S_TXN, seed), rng("c3", round_no, _S_HOST, seed)
    if n_txn is None:
        n_txn = int(gt.integers(1 << 20, (1 << 21) + 1))
    return {"init": np.full(n_accounts, 1000, dtype=np.int64),
            "batch": c3_batch(gt, n_accounts, host_accounts, n_txn, theta, steal),
            "host": c3_host_transfers(gh, host_accounts, n_host)}


# ----------------------------------------------------------------------------
# C4: object cache
# ----------------------------------------------------------------------------

def c4_requests(g: np.random.Generator, n: int, n_keys: int, theta: float = 0.99,
                put_frac: float = 0.05, parity: int | None = 0, tid0: int = 0) -> CacheBatch:
    """GET/PUT requests over keys 1..n_keys drawn Zipf(theta); ``parity``
    keeps only keys whose low bit equals it (the key-bit split between the
    devices described for the cache experiment): rank r maps to key 2r+2-parity."""
    r = zipf_ranks(g, n_keys if parity is None else n_keys // 2, theta, n)
    if parity is None:
        key = r + 1
    else:
        key = 2 * r + 2 - parity   # parity 0 -> even keys 2,4,..; parity 1 -> odd keys 1,3,..
    op = (g.random(n) < put_frac).astype(np.uint8)
    return CacheBatch(key=key.astype(np.uint64), op=op,
                      tid=(np.arange(n, dtype=np.uint64) + tid0 + 1).astype(np.uint32))


# ----------------------------------------------------------------------------
# C5: serving
# ----------------------------------------------------------------------------

def c5_requests(g: np.random.Generator, n: int, rate: float, n_words: int = 1 << 27,
                hot_frac: float = 0.05, p_hot: float = 0.5, update_frac: float = 0.1,
                median_len: float = 4.0, sigma: float = 1.0, max_len: int = 64,
                host_lo: int | None = None, tid0: int = 0) -> dict:
    """Open-loop Poisson arrivals at ``rate`` txn/s; lengths lognormal
    (median 4, sigma 1) clamped to [1, 64]; update transactions write their
    first min(L, 4) words.  Accesses fall in the hot 5% of the GPU range
    with probability ``p_hot``.  The GPU range is [0, host_lo)."""
    if host_lo is None:
        host_lo = n_words - n_words // 16
    gaps = g.exponential(1.0 / rate, size=n)
    arrival = np.cumsum(gaps)
    L = np.clip(np.rint(np.exp(np.log(median_len) + sigma * g.standard_normal(n))), 1, max_len).astype(np.uint64)
    upd = g.random(n) < update_frac
    nw = np.where(upd, np.minimum(L, 4), 0)
    total = int(L.sum())
    hot = max(1, int(hot_frac * host_lo))
    hd = g.random(total) < p_hot
    idx = np.where(hd, g.integers(0, hot, size=total, dtype=np.uint64),
                   g.integers(hot, host_lo, size=total, dtype=np.uint64))
    return {"arrival_s": arrival, "batch": _oplist_from_lists(L, nw, idx, tid0)}


# ----------------------------------------------------------------------------
# tiny brute-force cases
# ----------------------------------------------------------------------------

def tiny(seed: int, n_words: int = 16, n_txn: int = 5, max_ops: int = 3) -> RoundInputs:
    g = rng("tiny", seed, _S_TXN)
    init = g.integers(0, 1000, size=n_words, dtype=np.uint64).astype(np.uint32)
    lens = g.integers(1, max_ops + 1, size=n_txn, dtype=np.uint64)
    nws = np.array([g.integers(0, int(l) + 1) for l in lens])
    idx = g.integers(0, n_words, size=int(lens.sum()), dtype=np.uint64)
    batch = _oplist_from_lists(lens, nws, idx, 0)
    log = host_log_uniform(g, 3, 0, n_words, 0)
    return RoundInputs(cfg="tiny", n_words=n_words, word_bytes=4, granule=int(g.choice([1, 2, 4])),
                       program=PROG_OPLIST, init=init, batch=batch, log=log)
