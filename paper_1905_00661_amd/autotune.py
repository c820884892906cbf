"""Launch-width tuner for the transaction kernel, cached per workload.

The persistent transaction kernel's grid (workgroups of 4 waves) trades
memory-level parallelism against local conflicts: more waves keep more slot
reads in flight but overlap more transactions, which raises local retries
and the line-request load on the L2.  Which width wins depends on the
workload (words, batch size, hot fraction, operations per transaction) and on
the library's own kernels, so it is measured: runs of back-to-back rounds of
the caller's workload (the steady state, where a round's merge overlaps the
next round) are timed at a few widths around one workgroup per compute unit.
The fastest is kept only if it beats one workgroup per compute unit by a
margin; differences below it are noise between runs, not a property of the
width.

Results are cached by a signature of the workload's shape, the device name
and a hash of the library's sources, so a changed kernel never reuses a
stale choice.  The granule and the lock stripe are not tuned: the granule
sets how precisely inter-device conflicts are detected and the stripe how
many false local conflicts arise, so both belong to the workload.
"""
from __future__ import annotations

import glob
import hashlib
import json
import os
import statistics
import time
from typing import Callable, Iterable

PKG = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "hetm", "tuned.json")


def library_hash() -> str:
    """Hash of the library's HIP and host sources and its public header."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(PKG, "csrc", "*")))
    files.append(os.path.join(os.path.dirname(PKG), "include", "hetm.h"))
    for f in files:
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def signature(workload: dict, device: str, sources: str) -> str:
    """A key for one workload shape on one device with one build of the
    library; independent of the dict's insertion order."""
    blob = json.dumps({"workload": workload, "device": device, "sources": sources}, sort_keys=True)
    return hashlib.sha256(blob.encode()).hexdigest()[:16]


class TuneCache:
    """A JSON file of signature -> tuned entry.  A missing or unreadable
    file reads as empty; writes replace the file atomically."""

    def __init__(self, path: str = DEFAULT_CACHE):
        self.path = path

    def _load(self) -> dict:
        try:
            with open(self.path) as f:
                d = json.load(f)
            return d if isinstance(d, dict) else {}
        except (OSError, ValueError):
            return {}

    def get(self, sig: str) -> dict | None:
        return self._load().get(sig)

    def put(self, sig: str, entry: dict) -> None:
        d = self._load()
        d[sig] = entry
        os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
        tmp = f"{self.path}.{os.getpid()}.tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def pick(candidates: Iterable[int], measure: Callable[[int], float], repeats: int = 3,
         default: int | None = None, margin: float = 0.0) -> tuple[int, list[dict]]:
    """Measures each candidate `repeats` times (seconds per round) and returns
    the one with the lowest median, the smaller on a tie, with the table.
    If `default` is a candidate and its median is within `margin` (a
    fraction) of the best, the default is returned instead."""
    table = []
    for c in candidates:
        times = [measure(c) for _ in range(repeats)]
        table.append({"exec_workgroups": c, "median_s": statistics.median(times), "min_s": min(times)})
    best = min(table, key=lambda r: (r["median_s"], r["exec_workgroups"]))
    for r in table:
        if r["exec_workgroups"] == default and r["median_s"] <= best["median_s"] * (1.0 + margin):
            return default, table
    return best["exec_workgroups"], table


def candidates_for(cus: int, fractions: Iterable[float] = (0.5, 0.75, 1.0, 1.5, 2.0)) -> list[int]:
    return sorted({max(1, int(round(f * cus))) for f in fractions})


def tune_exec_workgroups(set_workgroups: Callable[[int], None], run_round: Callable[[], None], cus: int,
                         sig: str | None = None, cache: TuneCache | None = None, repeats: int = 3,
                         fractions: Iterable[float] = (0.5, 0.75, 1.0, 1.5, 2.0),
                         sync: Callable[[], None] = lambda: None,
                         timer: Callable[[], float] = time.perf_counter,
                         rounds: int = 8, warm: int = 2, margin: float = 0.02) -> dict:
    """Returns {"exec_workgroups", "table", "cached"} and leaves the context
    set to the chosen width.  run_round runs one whole round of the workload
    (returning when the host has its outcome; work it leaves in flight, such
    as an overlapped merge, may run on into the next round); sync waits for
    all of it.  One measurement is `rounds` rounds back to back after `warm`
    untimed ones, in seconds per round.  One workgroup per compute unit is
    kept unless another width is faster by more than `margin`.  A cached
    entry for `sig` is used without measuring."""
    if cache is not None and sig is not None:
        hit = cache.get(sig)
        if hit is not None and "exec_workgroups" in hit:
            set_workgroups(int(hit["exec_workgroups"]))
            return {**hit, "cached": True}

    def measure(wg: int) -> float:
        set_workgroups(wg)
        for _ in range(warm):        # rounds at a new width warm it up and fill the pipeline
            run_round()
        t0 = timer()
        for _ in range(rounds):
            run_round()
        sync()
        return (timer() - t0) / rounds

    best, table = pick(candidates_for(cus, fractions), measure, repeats, default=cus, margin=margin)
    set_workgroups(best)
    entry = {"exec_workgroups": best, "table": table}
    if cache is not None and sig is not None:
        cache.put(sig, entry)
    return {**entry, "cached": False}
