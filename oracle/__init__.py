"""CPU oracle for one SHeTM round -- TEST INFRASTRUCTURE, not the product.

Thin numpy wrappers over ``hetm_oracle.c`` (plain single-threaded C built
with gcc).  Only ``tests/``, the smoke check and the CPU-baseline leg of the
benchmark may import this package; the product library never does, and the
two share no code.  Every function follows a step of the paper's basic
algorithm (§IV-C): execution replay in a given commit order, validation,
apply and merge.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hetm_oracle.c")
_LIB = os.path.join(_HERE, "libhetm_oracle.so")

OK, EINVAL, EORDER = 0, -1, -3

LOG4 = np.dtype([("word", "<u4"), ("value", "<u4"), ("ts", "<u8")])
LOG8 = np.dtype([("word", "<u4"), ("pad", "<u4"), ("value", "<u8"), ("ts", "<u8")])

CACHE_SET_WORDS = 128


def build() -> str:
    """Compile the oracle with gcc (always rebuilds)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                           "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P, U64, I = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
        sig = {
            "orc_replay_oplist": [P, U64, U64, P, P, P, P, U64, P, P, P, P],
            "orc_replay_transfer": [P, U64, U64, P, P, P, U64, P, P, P, P],
            "orc_replay_cache": [P, U64, U64, P, P, P, U64, P, P, P, P],
            "orc_validate": [P, I, U64, P, U64, U64, P, P],
            "orc_apply": [P, I, P, U64, P, U64, U64, P],
            "orc_merge": [ctypes.c_uint32, P, U64, U64, I, P, P, P, P, P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes, f.restype = args, I
        L.orc_mix64.argtypes, L.orc_mix64.restype = [U64], U64
        L.orc_cache_set.argtypes, L.orc_cache_set.restype = [U64, U64], U64
        L.orc_cache_value.argtypes, L.orc_cache_value.restype = [U64, ctypes.c_uint32, P], None
        L.orc_host_transfers.argtypes, L.orc_host_transfers.restype = [P, U64, P, P, P, P, U64, P], U64
        L.orc_host_cache_puts.argtypes, L.orc_host_cache_puts.restype = [P, U64, P, P, U64, P], U64
        _lib = L
    return _lib


def _p(a: np.ndarray | None):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be contiguous"
    return a.ctypes.data


def n_granules(n_words: int, G: int) -> int:
    return (n_words + G - 1) // G


def bitmap_words(nbits: int) -> int:
    return (nbits + 31) // 32


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle returned {code}")
        self.code = code


def _check(rc: int, what: str):
    if rc != OK:
        raise OracleError(rc, what)


# ---------------------------------------------------------------- execution

def replay_oplist(S: np.ndarray, G: int, batch, order: np.ndarray, RS=None, WS=None):
    """Replays an OPLIST batch in commit ``order`` on S (modified in place).
    Returns (results, RS, WS)."""
    N = S.shape[0]
    ng = bitmap_words(n_granules(N, G))
    RS = np.zeros(ng, np.uint32) if RS is None else RS
    WS = np.zeros(ng, np.uint32) if WS is None else WS
    res = np.zeros(int(batch.offsets[-1]), np.uint32)
    order = np.ascontiguousarray(order, dtype=np.uint32)
    assert S.dtype == np.uint32
    _check(lib().orc_replay_oplist(_p(S), N, G, _p(batch.offsets), _p(batch.idx), _p(batch.n_writes),
                                   _p(batch.tid), batch.n, _p(order), _p(res), _p(RS), _p(WS)),
           "replay_oplist")
    return res, RS, WS


def replay_transfer(S: np.ndarray, G: int, batch, order: np.ndarray, RS=None, WS=None):
    N = S.shape[0]
    ng = bitmap_words(n_granules(N, G))
    RS = np.zeros(ng, np.uint32) if RS is None else RS
    WS = np.zeros(ng, np.uint32) if WS is None else WS
    res = np.zeros(3 * batch.n, np.int64)
    order = np.ascontiguousarray(order, dtype=np.uint32)
    assert S.dtype == np.int64
    _check(lib().orc_replay_transfer(_p(S), N, G, _p(batch.src), _p(batch.dst), _p(batch.amt),
                                     batch.n, _p(order), _p(res), _p(RS), _p(WS)), "replay_transfer")
    return res, RS, WS


def replay_cache(S: np.ndarray, G: int, batch, order: np.ndarray, RS=None, WS=None):
    N = S.shape[0]
    ng = bitmap_words(n_granules(N, G))
    RS = np.zeros(ng, np.uint32) if RS is None else RS
    WS = np.zeros(ng, np.uint32) if WS is None else WS
    res = np.zeros(9 * batch.n, np.uint32)
    order = np.ascontiguousarray(order, dtype=np.uint32)
    assert S.dtype == np.uint32
    _check(lib().orc_replay_cache(_p(S), N, G, _p(batch.key), _p(batch.op), _p(batch.tid),
                                  batch.n, _p(order), _p(res), _p(RS), _p(WS)), "replay_cache")
    return res, RS, WS


# ---------------------------------------------------------------- validate / apply / merge

def validate(log: np.ndarray, RS: np.ndarray, G: int, N: int):
    """Returns (flags bit-array as uint32 words, conflict)."""
    W = 4 if log.dtype == LOG4 else 8
    flags = np.zeros(bitmap_words(log.shape[0]), np.uint32)
    c = ctypes.c_uint32(0)
    _check(lib().orc_validate(_p(log), W, log.shape[0], _p(RS), G, N, _p(flags), ctypes.byref(c)),
           "validate")
    return flags, int(c.value)


def apply(S: np.ndarray, TS: np.ndarray, log: np.ndarray, floor: int) -> int:
    """Applies log to S / TS in place; returns the largest timestamp seen.
    Raises OracleError(-1 / -3) on a precondition violation."""
    W = 4 if log.dtype == LOG4 else 8
    assert S.itemsize == W and TS.dtype == np.uint64
    mx = ctypes.c_uint64(0)
    _check(lib().orc_apply(_p(S), W, _p(TS), S.shape[0], _p(log), log.shape[0], floor, ctypes.byref(mx)),
           "apply")
    return int(mx.value)


def apply_rc(S, TS, log, floor) -> int:
    W = 4 if log.dtype == LOG4 else 8
    mx = ctypes.c_uint64(0)
    return lib().orc_apply(_p(S), W, _p(TS), S.shape[0], _p(log), log.shape[0], floor, ctypes.byref(mx))


def merge(conflict: int, WS: np.ndarray, G: int, S: np.ndarray, H: np.ndarray):
    """Merges in place; returns (ids, n_runs)."""
    N = S.shape[0]
    ids = np.zeros(n_granules(N, G), np.uint32)
    nd, nr = ctypes.c_uint64(0), ctypes.c_uint64(0)
    _check(lib().orc_merge(conflict, _p(WS), G, N, S.itemsize, _p(S), _p(H), _p(ids),
                           ctypes.byref(nd), ctypes.byref(nr)), "merge")
    return ids[:nd.value].copy(), int(nr.value)


# ---------------------------------------------------------------- cache helpers

def mix64(z: int) -> int:
    return int(lib().orc_mix64(z))


def cache_set(key: int, nsets: int) -> int:
    return int(lib().orc_cache_set(key, nsets))


def cache_value(key: int, tid: int) -> np.ndarray:
    v = np.zeros(8, np.uint32)
    lib().orc_cache_value(key, tid, _p(v))
    return v


def host_transfers(H: np.ndarray, batch, ts: np.ndarray) -> np.ndarray:
    """Replays host transfers serially in the given order with the given
    commit timestamps; returns the log."""
    ts = np.ascontiguousarray(ts, dtype=np.uint64)
    log = np.zeros(max(2 * batch.n, 1), LOG8)
    m = lib().orc_host_transfers(_p(H), H.shape[0], _p(batch.src), _p(batch.dst), _p(batch.amt), _p(ts),
                                 batch.n, _p(log))
    return log[:m].copy()


def host_cache_puts(H: np.ndarray, keys: np.ndarray, ts: np.ndarray) -> np.ndarray:
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    ts = np.ascontiguousarray(ts, dtype=np.uint64)
    log = np.zeros(max(12 * keys.shape[0], 1), LOG4)
    m = lib().orc_host_cache_puts(_p(H), H.shape[0], _p(keys), _p(ts), keys.shape[0], _p(log))
    return log[:m].copy()


# ---------------------------------------------------------------- whole round

POLICY_CPU_WINS, POLICY_GPU_WINS = 0, 1


def log_granules(log: np.ndarray, G: int, N: int) -> np.ndarray:
    """Bitmap (uint32 words, bit g of word g/32) of the granules the host log
    writes: the host's write set at granule resolution (§IV-B)."""
    bm = np.zeros(bitmap_words(n_granules(N, G)), np.uint32)
    g = log["word"].astype(np.int64) // G
    np.bitwise_or.at(bm, g >> 5, np.left_shift(np.uint32(1), (g & 31).astype(np.uint32)))
    return bm


def round_generic(replay, S: np.ndarray, H: np.ndarray, TS: np.ndarray, G: int, batch, order, log,
                  floor: int, policy: int = POLICY_CPU_WINS) -> dict:
    """One full round (§IV-C): replay the batch in commit order, validate the
    host log, apply it, merge.  H is the host replica holding the host's own
    writes of the round.  S, H, TS are updated in place.

    policy (§IV-E): CPU_WINS applies the log always and, on a conflict,
    restores the GPU's written granules from H.  GPU_WINS applies the log
    only when validation found no conflict; on a conflict the host's round is
    discarded -- nothing of its log is applied, the watermark stays -- and the
    granules written by either side go from S to H."""
    res, RS, WS = replay(S, G, batch, order)
    flags, conflict = validate(log, RS, G, S.shape[0])
    if policy == POLICY_GPU_WINS and conflict:
        mx = floor
        ids, runs = merge(0, WS | log_granules(log, G, S.shape[0]), G, S, H)
    else:
        mx = apply(S, TS, log, floor)
        ids, runs = merge(conflict, WS, G, S, H)
    return {"results": res, "RS": RS, "WS": WS, "flags": flags, "conflict": conflict,
            "ids": ids, "n_runs": runs, "max_ts": mx}


def round_oplist(S, H, TS, G, batch, order, log, floor, policy: int = POLICY_CPU_WINS) -> dict:
    return round_generic(replay_oplist, S, H, TS, G, batch, order, log, floor, policy)


def order_from_tickets(tickets: np.ndarray, even_ties: bool = False) -> np.ndarray:
    """Commit order pi from per-transaction tickets (gaps allowed).  Tickets
    are unique, except with even_ties, where transactions may share an even
    ticket (read-only transactions serialized at the same snapshot, which
    commute; the caller checks that they read only); ties replay in index
    order."""
    order = np.argsort(tickets, kind="stable").astype(np.uint32)
    t = tickets[order]
    if t.shape[0] > 1:
        tie = t[1:] == t[:-1]
        if tie.any() and not (even_ties and np.all(t[1:][tie] % 2 == 0)):
            raise ValueError("tickets are not unique")
    return order


def tied_tickets(tickets: np.ndarray) -> np.ndarray:
    """Indices of the transactions whose ticket another one shares."""
    vals, counts = np.unique(tickets, return_counts=True)
    return np.flatnonzero(np.isin(tickets, vals[counts > 1]))
