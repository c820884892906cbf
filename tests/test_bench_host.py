"""Host-side logic of bench.py: the transaction kernel's algorithmic bytes,
the committed traffic summary it reads, and the one-GPU contract."""
from __future__ import annotations

import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1905_00661_amd import workloads as wl  # noqa: E402


def test_exec_alg_bytes_by_hand():
    """Two read-only transactions (16 and 3 reads) and one update (4 reads,
    2 writes): 21 B per transaction, 17 B per read, 8 B per read of an
    update, 28 B per write."""
    batch = wl._oplist_from_lists(np.array([16, 3, 4], np.uint64), np.array([0, 0, 2], np.int64),
                                  np.arange(23, dtype=np.uint64), 0)
    expect = 3 * 21 + (16 + 3 + 4) * 17 + 4 * 8 + 2 * 28
    assert bench.exec_alg_bytes(batch) == expect


def test_exec_alg_bytes_large_mix():
    """The large mix (90% read-only with 16 reads, 10% with 4 read-modify-
    writes) averages 287 B per transaction."""
    n_ro, n_up = 900, 100
    lens = np.concatenate([np.full(n_ro, 16), np.full(n_up, 4)]).astype(np.uint64)
    nws = np.concatenate([np.zeros(n_ro), np.full(n_up, 4)]).astype(np.int64)
    batch = wl._oplist_from_lists(lens, nws, np.zeros(int(lens.sum()), np.uint64), 0)
    assert abs(bench.exec_alg_bytes(batch) / 1000 - 287.0) < 1e-9


import pytest  # noqa: E402


@pytest.mark.parametrize("kernel", sorted(bench.TRAFFIC_FILES))
def test_traffic_summary_matches_sources(kernel):
    """Each committed counter summary is read only while its kernels' sources
    hash to the value it records, and then gives a positive byte count."""
    text = open(os.path.join(ROOT, "profiles", bench.TRAFFIC_FILES[kernel])).read()
    recorded = [line.split(":", 1)[1].strip() for line in text.splitlines() if line.startswith("source_hash:")]
    assert len(recorded) == 1
    got = bench.load_traffic(kernel)
    if recorded[0] == bench.source_hash(kernel):
        assert got is not None and got > 0
    else:
        assert got is None


def test_stale_summary_is_ignored(tmp_path, monkeypatch):
    """A summary whose recorded hash differs from the sources' gives None."""
    (tmp_path / "x.md").write_text("source_hash: 0000000000000000\nbytes_per_launch: 123\n")
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    monkeypatch.setitem(bench.TRAFFIC_FILES, "k_exec_oplist", "x.md")
    assert bench.load_traffic("k_exec_oplist") is None


def test_more_than_one_gpu_is_refused():
    """bench.py measures one GPU: --gpus 2 exits with a message and status 2,
    before touching torch or the library."""
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert p.returncode == 2
    assert "one GPU" in json.loads(p.stdout.strip().splitlines()[-1])["error"]
