"""Python binding of libhetm (ctypes), with the C ABI's names.

Argument marshalling only: every step of a round runs in the HIP kernels of
``libhetm.so``.  PyTorch supplies device memory, pinned host memory and the
stream; the functions take and return plain pointers and integers, and
:class:`Context` wraps one ``hetm_ctx`` with torch buffers.

The library must have been built (``python -m paper_1905_00661_amd.build`` or
``__graft_entry__.build()``); loading fails loudly otherwise -- there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhetm.so")

# error codes
HETM_OK, HETM_EINVAL, HETM_ENOMEM, HETM_EORDER = 0, -1, -2, -3
HETM_ECAPACITY, HETM_EDEVICE, HETM_ERETRY, HETM_ESTATE = -4, -5, -6, -7
# programs / modes / state selectors
HETM_PROG_OPLIST, HETM_PROG_TRANSFER, HETM_PROG_CACHE = 1, 2, 3
HETM_MODE_PLAIN, HETM_MODE_GRAPH = 0, 1
HETM_OUTCOME_DEVICE = 0xFFFFFFFF
HETM_POLICY_CPU_WINS, HETM_POLICY_GPU_WINS = 0, 1
HETM_STATE_STMR, HETM_STATE_RS, HETM_STATE_WS, HETM_STATE_LOCKS = 0, 2, 3, 4

EXPORTS = ["hetm_alloc_stmr", "hetm_free", "hetm_submit_batch", "hetm_validate_apply_log",
           "hetm_copyback_dirty", "hetm_round", "hetm_strerror", "hetm_last_error", "hetm_sync",
           "hetm_stats_get", "hetm_read_state", "hetm_state_bytes", "hetm_host_tm_create",
           "hetm_host_tm_free", "hetm_host_tm_clock", "hetm_host_run_transfers", "hetm_host_run_cache_puts",
           "hetm_serve", "hetm_set_exec_workgroups", "hetm_early_validate", "hetm_set_version_clock",
           "hetm_read_words_noalloc", "hetm_round_begin", "hetm_round_push", "hetm_round_add", "hetm_round_end",
           "hetm_round_submit", "hetm_round_collect"]

P = ctypes.c_void_p
U32, U64, I32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32


class hetm_config(ctypes.Structure):
    _fields_ = [("n_words", U64), ("word_bytes", U32), ("granule_words", U32),
                ("lock_stripe_words", U32), ("max_txn_ops", U32), ("batch_capacity", U64),
                ("log_capacity", U64), ("mode", U32), ("device", I32), ("stream", P),
                ("exec_workgroups", U32), ("retry_cap", U32), ("async_merge", U32)]


class hetm_oplist_desc(ctypes.Structure):
    _fields_ = [("offsets", P), ("idx", P), ("n_writes", P), ("tid", P)]


class hetm_transfer_desc(ctypes.Structure):
    _fields_ = [("src", P), ("dst", P), ("amt", P)]


class hetm_cache_desc(ctypes.Structure):
    _fields_ = [("key", P), ("op", P), ("tid", P)]


class hetm_round_args(ctypes.Structure):
    _fields_ = [("program", U32), ("descs", P), ("n_txns", U64), ("results", P), ("tickets", P),
                ("log", P), ("n_log", U64), ("flags_bits", P), ("host_replica", P), ("ids_out", P),
                ("policy", U32), ("pad_", U32)]


class hetm_round_result(ctypes.Structure):
    _fields_ = [("conflict", U32), ("error", I32), ("n_committed", U64), ("n_aborted", U64),
                ("n_local_retries", U64), ("n_dirty", U64), ("n_runs", U64), ("max_ts", U64),
                ("merge_pending", U32), ("doomed", U32), ("us_exec", ctypes.c_double), ("us_validate", ctypes.c_double),
                ("us_merge", ctypes.c_double), ("us_total", ctypes.c_double),
                ("host_discarded", U32), ("gpu_losses", U32), ("us_exec_kernel", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class hetm_serve_spec(ctypes.Structure):
    _fields_ = [("n_requests", U64), ("arrival_s", P), ("offsets", P), ("idx", P), ("n_writes", P), ("tid", P),
                ("host_log", P), ("host_log_len", U64), ("host_log_per_round", U64), ("max_batch", U64),
                ("mem_budget_bytes", U64), ("pipelined", U32), ("starvation_limit", U32),
                ("early_validation", U32), ("push_entries", U32), ("round_period_us", ctypes.c_double)]


class hetm_serve_report(ctypes.Structure):
    _fields_ = [("served", U64), ("rounds", U64), ("conflicted_rounds", U64), ("requeued", U64),
                ("wall_s", ctypes.c_double), ("throughput", ctypes.c_double), ("p50_latency_us", ctypes.c_double),
                ("p99_latency_us", ctypes.c_double), ("mean_latency_us", ctypes.c_double),
                ("max_latency_us", ctypes.c_double), ("latency_us", P), ("results", P), ("commit_seq", P),
                ("round_conflict", P), ("max_rounds", U64), ("round_log_end", P),
                ("us_pack", ctypes.c_double), ("us_wait_round", ctypes.c_double), ("us_settle", ctypes.c_double),
                ("us_host_commit", ctypes.c_double), ("us_wait_merge", ctypes.c_double), ("us_idle", ctypes.c_double),
                ("starved_rounds", U64), ("batches", U64)]


class hetm_stats(ctypes.Structure):
    _fields_ = [("rounds", U64), ("rounds_conflicted", U64), ("txns_committed", U64),
                ("txns_aborted", U64), ("local_retries", U64), ("log_entries", U64),
                ("dirty_granules", U64), ("watermark", U64), ("device_bytes", U64),
                ("us_host_scatter", ctypes.c_double), ("us_merge_wait", ctypes.c_double),
                ("version_resets", U64), ("rollbacks_device", U64), ("rollbacks_host", U64)]


class HetmError(RuntimeError):
    def __init__(self, code: int, what: str, detail: str = ""):
        super().__init__(f"{what} failed: {code} ({_strerror(code)}) {detail}".strip())
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """Loads libhetm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(hipcc, gfx950); there is no non-HIP implementation")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "hetm_alloc_stmr": ([ctypes.POINTER(hetm_config), P, ctypes.POINTER(P)], ctypes.c_int),
            "hetm_free": ([P], ctypes.c_int),
            "hetm_submit_batch": ([P, U32, P, U64, P, P], ctypes.c_int),
            "hetm_validate_apply_log": ([P, P, U64, P, P], ctypes.c_int),
            "hetm_copyback_dirty": ([P, U32, P, P, P], ctypes.c_int),
            "hetm_round": ([P, ctypes.POINTER(hetm_round_args), ctypes.POINTER(hetm_round_result)], ctypes.c_int),
            "hetm_strerror": ([ctypes.c_int], ctypes.c_char_p),
            "hetm_last_error": ([P], ctypes.c_char_p),
            "hetm_sync": ([P], ctypes.c_int),
            "hetm_stats_get": ([P, ctypes.POINTER(hetm_stats)], ctypes.c_int),
            "hetm_read_state": ([P, U32, P, U64], ctypes.c_int),
            "hetm_state_bytes": ([P, U32], U64),
            "hetm_read_words_noalloc": ([P, U64, U64, P], ctypes.c_int),
            "hetm_round_begin": ([P, ctypes.POINTER(hetm_round_args)], ctypes.c_int),
            "hetm_round_push": ([P, P, U64, P], ctypes.c_int),
            "hetm_round_add": ([P, U32, P, U64, P, P], ctypes.c_int),
            "hetm_round_end": ([P, ctypes.POINTER(hetm_round_result)], ctypes.c_int),
            "hetm_round_submit": ([P, ctypes.POINTER(hetm_round_args)], ctypes.c_int),
            "hetm_round_collect": ([P, ctypes.POINTER(hetm_round_result)], ctypes.c_int),
            "hetm_host_tm_create": ([P, U64, U32, U32, U64, ctypes.POINTER(P)], ctypes.c_int),
            "hetm_host_tm_free": ([P], ctypes.c_int),
            "hetm_host_tm_clock": ([P], U64),
            "hetm_host_run_transfers": ([P, P, P, P, U64, U32, P, P, U64, ctypes.POINTER(U64)], ctypes.c_int),
            "hetm_host_run_cache_puts": ([P, P, U64, U32, P, P, U64, ctypes.POINTER(U64)], ctypes.c_int),
            "hetm_set_exec_workgroups": ([P, U32], ctypes.c_int),
            "hetm_early_validate": ([P, P, U64, P], ctypes.c_int),
            "hetm_set_version_clock": ([P, U32], ctypes.c_int),
            "hetm_serve": ([P, ctypes.POINTER(hetm_serve_spec), P, ctypes.POINTER(hetm_serve_report)], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes, f.restype = args, res
        _lib = L
    return _lib


def _strerror(code: int) -> str:
    try:
        return lib().hetm_strerror(code).decode()
    except Exception:   # noqa: BLE001 - message formatting only
        return "?"


def _check(rc: int, what: str, ctx=None):
    if rc != HETM_OK:
        detail = lib().hetm_last_error(ctx).decode() if ctx else ""
        raise HetmError(rc, what, detail)


# ------------------------------------------------------------- C-ABI mirrors

def hetm_alloc_stmr(cfg: hetm_config, init_image: int | None) -> int:
    out = P()
    rc = lib().hetm_alloc_stmr(ctypes.byref(cfg), init_image, ctypes.byref(out))
    if rc != HETM_OK:
        raise HetmError(rc, "hetm_alloc_stmr", lib().hetm_last_error(None).decode())
    return out.value


def hetm_free(ctx: int) -> None:
    _check(lib().hetm_free(ctx), "hetm_free")


def hetm_submit_batch(ctx: int, program: int, descs, n_txns: int, results: int, tickets: int) -> None:
    _check(lib().hetm_submit_batch(ctx, program, ctypes.byref(descs), n_txns, results, tickets),
           "hetm_submit_batch", ctx)


def hetm_validate_apply_log(ctx: int, log: int, n: int, flags_bits: int | None, want_conflict: bool = True):
    c = U32(0)
    _check(lib().hetm_validate_apply_log(ctx, log, n, flags_bits, ctypes.byref(c) if want_conflict else None),
           "hetm_validate_apply_log", ctx)
    return int(c.value) if want_conflict else None


def hetm_copyback_dirty(ctx: int, conflict: int, host_replica: int, ids_out: int | None = None) -> int:
    nd = U64(0)
    _check(lib().hetm_copyback_dirty(ctx, conflict, host_replica, ctypes.byref(nd), ids_out),
           "hetm_copyback_dirty", ctx)
    return int(nd.value)


def hetm_round(ctx: int, args: hetm_round_args) -> hetm_round_result:
    res = hetm_round_result()
    _check(lib().hetm_round(ctx, ctypes.byref(args), ctypes.byref(res)), "hetm_round", ctx)
    return res


def hetm_sync(ctx: int) -> None:
    _check(lib().hetm_sync(ctx), "hetm_sync", ctx)


def hetm_stats_get(ctx: int) -> hetm_stats:
    s = hetm_stats()
    _check(lib().hetm_stats_get(ctx, ctypes.byref(s)), "hetm_stats_get", ctx)
    return s


def hetm_read_state(ctx: int, what: int, dst: int, nbytes: int) -> None:
    _check(lib().hetm_read_state(ctx, what, dst, nbytes), "hetm_read_state", ctx)


def hetm_read_words_noalloc(ctx: int, first_word: int, n_words: int, dst: int) -> None:
    _check(lib().hetm_read_words_noalloc(ctx, first_word, n_words, dst), "hetm_read_words_noalloc", ctx)


def hetm_state_bytes(ctx: int, what: int) -> int:
    return int(lib().hetm_state_bytes(ctx, what))


# ------------------------------------------------------------- host side

class HostTM:
    """The host's TM threads over a host replica (numpy array, borrowed)."""

    LOG4 = np.dtype([("word", "<u4"), ("value", "<u4"), ("ts", "<u8")])
    LOG8 = np.dtype([("word", "<u4"), ("pad", "<u4"), ("value", "<u8"), ("ts", "<u8")])

    def __init__(self, replica: np.ndarray, stripe: int = 1, ts_start: int = 0):
        assert replica.flags["C_CONTIGUOUS"] and replica.itemsize in (4, 8)
        self.replica = replica
        h = P()
        _check(lib().hetm_host_tm_create(replica.ctypes.data, replica.shape[0], replica.itemsize, stripe, ts_start,
                                         ctypes.byref(h)), "hetm_host_tm_create")
        self.h = h.value

    def close(self):
        if self.h:
            lib().hetm_host_tm_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # noqa: BLE001
            pass

    @property
    def clock(self) -> int:
        return int(lib().hetm_host_tm_clock(self.h))

    def transfers(self, src, dst, amt, threads: int = 4):
        n = len(src)
        src, dst, amt = (np.ascontiguousarray(x, dtype=np.uint32) for x in (src, dst, amt))
        ts = np.zeros(max(n, 1), np.uint64)
        log = np.zeros(max(2 * n, 1), self.LOG8)
        m = U64(0)
        _check(lib().hetm_host_run_transfers(self.h, src.ctypes.data, dst.ctypes.data, amt.ctypes.data, n, threads,
                                             ts.ctypes.data, log.ctypes.data, log.shape[0], ctypes.byref(m)),
               "hetm_host_run_transfers")
        return ts[:n], log[:m.value]

    def cache_puts(self, keys, threads: int = 4):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        n = keys.shape[0]
        ts = np.zeros(max(n, 1), np.uint64)
        log = np.zeros(max(12 * n, 1), self.LOG4)
        m = U64(0)
        _check(lib().hetm_host_run_cache_puts(self.h, keys.ctypes.data, n, threads, ts.ctypes.data,
                                              log.ctypes.data, log.shape[0], ctypes.byref(m)),
               "hetm_host_run_cache_puts")
        return ts[:n], log[:m.value]


# ------------------------------------------------------------- torch helpers

def _torch():
    import torch
    return torch


def to_device(a: np.ndarray, device: str = "cuda"):
    """Copies a numpy array to a flat device tensor of the same bytes."""
    torch = _torch()
    a = np.ascontiguousarray(a)
    t = torch.from_numpy(a.view(np.uint8).reshape(-1).copy())
    return t.to(device)


def pinned(nbytes: int):
    torch = _torch()
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, pin_memory=True)


def tensor_to_numpy(t, dtype, count: int | None = None) -> np.ndarray:
    a = t.cpu().numpy().view(dtype)
    return a if count is None else a[:count]


class Batch:
    """Device copies of a batch's descriptors plus its results / tickets."""

    def __init__(self, program: int, batch, device: str = "cuda"):
        torch = _torch()
        self.program, self.src = program, batch
        self.n = batch.n
        if program == HETM_PROG_OPLIST:
            self.bufs = [to_device(batch.offsets), to_device(batch.idx), to_device(batch.n_writes),
                         to_device(batch.tid)]
            self.desc = hetm_oplist_desc(*[b.data_ptr() for b in self.bufs])
            self.n_results, self.res_dtype = int(batch.offsets[-1]), np.uint32
        elif program == HETM_PROG_TRANSFER:
            self.bufs = [to_device(batch.src), to_device(batch.dst), to_device(batch.amt)]
            self.desc = hetm_transfer_desc(*[b.data_ptr() for b in self.bufs])
            self.n_results, self.res_dtype = 3 * self.n, np.int64
        else:
            self.bufs = [to_device(batch.key), to_device(batch.op), to_device(batch.tid)]
            self.desc = hetm_cache_desc(*[b.data_ptr() for b in self.bufs])
            self.n_results, self.res_dtype = 9 * self.n, np.uint32
        self.results = torch.zeros(max(self.n_results, 1) * np.dtype(self.res_dtype).itemsize,
                                   dtype=torch.uint8, device=device)
        self.tickets = torch.zeros(max(self.n, 1) * 4, dtype=torch.uint8, device=device)

    def results_np(self) -> np.ndarray:
        return tensor_to_numpy(self.results, self.res_dtype, self.n_results)

    def tickets_np(self) -> np.ndarray:
        return tensor_to_numpy(self.tickets, np.uint32, self.n)


class Context:
    """One hetm_ctx: the GPU replica and its metadata, on torch's stream."""

    def __init__(self, n_words: int, word_bytes: int, granule: int, init: np.ndarray | None = None,
                 stripe: int = 1, max_ops: int = 64, batch_capacity: int = 1 << 20,
                 log_capacity: int = 1 << 20, mode: int = HETM_MODE_PLAIN, exec_workgroups: int = 0,
                 retry_cap: int = 0, device: int = 0, async_merge: bool = False):
        torch = _torch()
        self.torch = torch
        self.dev = f"cuda:{device}"
        torch.cuda.set_device(device)
        self.stream = torch.cuda.current_stream(device)
        self.n_words, self.word_bytes, self.granule = n_words, word_bytes, granule
        self.n_granules = (n_words + granule - 1) // granule
        self.cfg = hetm_config(n_words=n_words, word_bytes=word_bytes, granule_words=granule,
                               lock_stripe_words=stripe, max_txn_ops=max_ops, batch_capacity=batch_capacity,
                               log_capacity=log_capacity, mode=mode, device=device,
                               stream=self.stream.cuda_stream, exec_workgroups=exec_workgroups,
                               retry_cap=retry_cap, async_merge=int(async_merge))
        init_t = None
        if init is not None:
            assert init.nbytes == n_words * word_bytes
            init_t = to_device(init, self.dev)
            torch.cuda.synchronize()
        self.ctx = hetm_alloc_stmr(self.cfg, init_t.data_ptr() if init_t is not None else None)
        del init_t

    def close(self):
        if getattr(self, "ctx", None):
            hetm_free(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # noqa: BLE001 - interpreter shutdown
            pass

    # -- state
    def read_state(self, what: int) -> np.ndarray:
        nb = hetm_state_bytes(self.ctx, what)
        buf = np.empty(nb, np.uint8)
        hetm_read_state(self.ctx, what, buf.ctypes.data, nb)
        if what == HETM_STATE_STMR:
            return buf.view(np.uint32 if self.word_bytes == 4 else np.int64)
        if what == HETM_STATE_LOCKS:
            return buf.view(np.uint64)
        return buf.view(np.uint32)

    def stats(self) -> hetm_stats:
        return hetm_stats_get(self.ctx)

    def sync(self) -> None:
        hetm_sync(self.ctx)

    def early_validate(self, log_dev, n: int, wait: bool = False):
        d = U32(0)
        _check(lib().hetm_early_validate(self.ctx, log_dev.data_ptr() if n else None, n,
                                         ctypes.byref(d) if wait else None), "hetm_early_validate", self.ctx)
        return int(d.value) if wait else None

    def set_version_clock(self, value: int) -> None:
        _check(lib().hetm_set_version_clock(self.ctx, value), "hetm_set_version_clock", self.ctx)

    def set_exec_workgroups(self, wg: int) -> None:
        _check(lib().hetm_set_exec_workgroups(self.ctx, wg), "hetm_set_exec_workgroups", self.ctx)

    # -- round steps
    def submit(self, b: Batch) -> None:
        hetm_submit_batch(self.ctx, b.program, b.desc, b.n, b.results.data_ptr(), b.tickets.data_ptr())

    def validate_apply(self, log_dev, n: int, flags=None) -> int:
        return hetm_validate_apply_log(self.ctx, log_dev.data_ptr() if n else None, n,
                                       flags.data_ptr() if flags is not None else None)

    def copyback(self, conflict: int, host, ids=None) -> int:
        return hetm_copyback_dirty(self.ctx, conflict, host.data_ptr(), ids.data_ptr() if ids is not None else None)

    def serve(self, arrival_s: np.ndarray, batch, host, host_log: np.ndarray, host_log_per_round: int,
              max_batch: int, mem_budget_bytes: int, pipelined: bool, max_rounds: int = 1 << 16,
              starvation_limit: int = 0, early_validation: bool = False, push_entries: int = 0,
              round_period_us: float = 0.0) -> dict:
        """Runs the request loop (hetm_serve) over OPLIST requests; returns the
        report and per-request latencies, results and commit positions."""
        arrival_s = np.ascontiguousarray(arrival_s, dtype=np.float64)
        n = arrival_s.shape[0]
        host_log = np.ascontiguousarray(host_log)
        lat = np.zeros(max(n, 1), np.float64)
        res = np.zeros(max(int(batch.offsets[-1]), 1), np.uint32)
        seq = np.zeros(max(n, 1), np.uint64)
        rconf = np.zeros(max_rounds, np.uint8)
        rlog = np.zeros(max_rounds, np.uint64)
        spec = hetm_serve_spec(n_requests=n, arrival_s=arrival_s.ctypes.data, offsets=batch.offsets.ctypes.data,
                               idx=batch.idx.ctypes.data, n_writes=batch.n_writes.ctypes.data,
                               tid=batch.tid.ctypes.data, host_log=host_log.ctypes.data if host_log.size else None,
                               host_log_len=host_log.shape[0], host_log_per_round=host_log_per_round,
                               max_batch=max_batch, mem_budget_bytes=mem_budget_bytes, pipelined=int(pipelined),
                               starvation_limit=starvation_limit, early_validation=int(early_validation),
                               push_entries=push_entries, round_period_us=float(round_period_us))
        rep = hetm_serve_report(latency_us=lat.ctypes.data, results=res.ctypes.data, commit_seq=seq.ctypes.data,
                                round_conflict=rconf.ctypes.data, max_rounds=max_rounds,
                                round_log_end=rlog.ctypes.data)
        _check(lib().hetm_serve(self.ctx, ctypes.byref(spec), host.data_ptr(), ctypes.byref(rep)), "hetm_serve",
               self.ctx)
        out = {f: getattr(rep, f) for f, _ in hetm_serve_report._fields_ if f not in
               ("latency_us", "results", "commit_seq", "round_conflict", "round_log_end", "max_rounds")}
        R = int(rep.rounds)
        out.update(latency_us=lat[:n], results=res[:int(batch.offsets[-1])], commit_seq=seq[:n],
                   round_conflict=rconf[:R], round_log_end=rlog[:R])
        return out

    def _round_args(self, b, log_dev, n_log, host, flags, ids, policy) -> hetm_round_args:
        return hetm_round_args(program=b.program if b else 0, descs=ctypes.addressof(b.desc) if b else None,
                               n_txns=b.n if b else 0, results=b.results.data_ptr() if b else None,
                               tickets=b.tickets.data_ptr() if b else None,
                               log=log_dev.data_ptr() if n_log else None, n_log=n_log, policy=policy,
                               flags_bits=flags.data_ptr() if flags is not None else None,
                               host_replica=host.data_ptr(), ids_out=ids.data_ptr() if ids is not None else None)

    def round(self, b: Batch | None, log_dev, n_log: int, host, flags=None, ids=None,
              policy: int = HETM_POLICY_CPU_WINS) -> hetm_round_result:
        return hetm_round(self.ctx, self._round_args(b, log_dev, n_log, host, flags, ids, policy))

    # -- streamed round (GRAPH mode)
    def round_begin(self, b: Batch | None, host, log_dev=None, n_log: int = 0, flags=None, ids=None,
                    policy: int = HETM_POLICY_CPU_WINS) -> None:
        self._streamed = self._round_args(b, log_dev, n_log, host, flags, ids, policy)   # kept alive
        _check(lib().hetm_round_begin(self.ctx, ctypes.byref(self._streamed)), "hetm_round_begin", self.ctx)

    def round_push(self, log, n: int, wait: bool = False):
        """Pushes n entries of `log` (a tensor, host or device); with wait,
        returns 1 if the open round is doomed."""
        d = U32(0)
        _check(lib().hetm_round_push(self.ctx, log.data_ptr() if n else None, n, ctypes.byref(d) if wait else None),
               "hetm_round_push", self.ctx)
        return int(d.value) if wait else None

    def round_add(self, b: "Batch") -> None:
        """Adds batch b to the open streamed round (after its earlier
        batches, before its tail); b's buffers must live until round_end."""
        _check(lib().hetm_round_add(self.ctx, b.program, ctypes.addressof(b.desc), b.n, b.results.data_ptr(),
                                    b.tickets.data_ptr()), "hetm_round_add", self.ctx)

    def round_end(self) -> hetm_round_result:
        r = hetm_round_result()
        _check(lib().hetm_round_end(self.ctx, ctypes.byref(r)), "hetm_round_end", self.ctx)
        return r

    # -- queued rounds (GRAPH mode, async_merge)
    def round_submit(self, b: Batch | None, log_dev, n_log: int, host, flags=None, ids=None,
                     policy: int = HETM_POLICY_CPU_WINS) -> None:
        """Queues a whole round behind those already queued (up to two);
        b, the log, flags and ids must live until the round is collected."""
        a = self._round_args(b, log_dev, n_log, host, flags, ids, policy)
        _check(lib().hetm_round_submit(self.ctx, ctypes.byref(a)), "hetm_round_submit", self.ctx)

    def round_collect(self) -> hetm_round_result:
        """Waits for the oldest queued round and returns its result."""
        r = hetm_round_result()
        _check(lib().hetm_round_collect(self.ctx, ctypes.byref(r)), "hetm_round_collect", self.ctx)
        return r
