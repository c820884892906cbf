"""The workgroup tuner's host logic on the CPU: signatures, the cache file,
the choice among measured candidates, and the cache short-cut (no GPU: the
rounds and the clock are stand-ins)."""
from __future__ import annotations

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1905_00661_amd import autotune  # noqa: E402

W = {"program": "oplist", "n_words": 1 << 28, "granule": 16, "n_txns": 1 << 20, "p_hot": 0.5}


def test_signature_is_order_free_and_sensitive():
    a = autotune.signature(W, "gpu", "abc")
    assert autotune.signature(dict(reversed(list(W.items()))), "gpu", "abc") == a
    assert autotune.signature({**W, "granule": 64}, "gpu", "abc") != a
    assert autotune.signature({**W, "p_hot": 0.9}, "gpu", "abc") != a
    assert autotune.signature(W, "other gpu", "abc") != a
    assert autotune.signature(W, "gpu", "abd") != a


def test_library_hash_follows_the_sources():
    h = autotune.library_hash()
    assert len(h) == 16 and h == autotune.library_hash()


def test_cache_roundtrip_and_corrupt_file(tmp_path):
    p = tmp_path / "sub" / "t.json"
    c = autotune.TuneCache(str(p))
    assert c.get("x") is None
    c.put("x", {"exec_workgroups": 256})
    c.put("y", {"exec_workgroups": 128})
    assert c.get("x") == {"exec_workgroups": 256} and c.get("y")["exec_workgroups"] == 128
    assert not [f for f in os.listdir(p.parent) if f.endswith(".tmp")]
    p.write_text("{not json")
    assert c.get("x") is None
    c.put("z", {"exec_workgroups": 1})
    assert json.loads(p.read_text()) == {"z": {"exec_workgroups": 1}}


def test_pick_takes_the_lowest_median_then_the_smaller():
    times = {128: [3.0, 1.0, 3.0], 256: [2.0, 2.0, 9.0], 512: [2.0, 2.0, 2.0]}
    it = {k: iter(v) for k, v in times.items()}
    best, table = autotune.pick([128, 256, 512], lambda c: next(it[c]), repeats=3)
    assert best == 256                       # medians 3, 2, 2: the tie goes to the smaller width
    assert [r["median_s"] for r in table] == [3.0, 2.0, 2.0]
    assert table[0]["min_s"] == 1.0


def test_pick_keeps_the_default_within_the_margin():
    cost = {128: 1.00, 256: 1.015, 512: 1.2}
    assert autotune.pick(cost, cost.get, repeats=1, default=256, margin=0.02)[0] == 256
    assert autotune.pick(cost, cost.get, repeats=1, default=256, margin=0.01)[0] == 128
    assert autotune.pick(cost, cost.get, repeats=1, default=384, margin=0.5)[0] == 128   # not a candidate
    assert autotune.pick(cost, cost.get, repeats=1)[0] == 128


def test_candidates_around_one_per_cu():
    assert autotune.candidates_for(256) == [128, 192, 256, 384, 512]
    assert autotune.candidates_for(1, (0.1, 1.0)) == [1]


class FakeRounds:
    """Round time as a function of the width set, on a fake clock."""

    def __init__(self, cost):
        self.cost, self.wg, self.t, self.rounds, self.sets = cost, None, 0.0, 0, []

    def set_wg(self, wg):
        self.wg = wg
        self.sets.append(wg)

    def run(self):
        self.rounds += 1
        self.t += self.cost(self.wg)


def test_tune_measures_then_uses_the_cache(tmp_path):
    cache = autotune.TuneCache(str(tmp_path / "t.json"))
    f = FakeRounds(lambda wg: abs(wg - 180) + 1.0)
    r = autotune.tune_exec_workgroups(f.set_wg, f.run, 256, sig="s1", cache=cache, repeats=2, timer=lambda: f.t)
    assert r["cached"] is False and r["exec_workgroups"] == 192      # nearest candidate to 180, well ahead of 256
    assert f.sets[-1] == 192 and f.rounds == 5 * 2 * (2 + 8)       # five widths, two repeats, 2 warm + 8 timed
    assert [t["median_s"] for t in r["table"]] == [53.0, 13.0, 77.0, 205.0, 333.0]   # seconds per round
    assert cache.get("s1")["exec_workgroups"] == 192
    g = FakeRounds(lambda wg: 1.0)
    r2 = autotune.tune_exec_workgroups(g.set_wg, g.run, 256, sig="s1", cache=cache, timer=lambda: g.t)
    assert r2["cached"] is True and r2["exec_workgroups"] == 192
    assert g.rounds == 0 and g.sets == [192]                        # no round run, the width still set
    r3 = autotune.tune_exec_workgroups(g.set_wg, g.run, 256, sig="s2", cache=cache, repeats=1, timer=lambda: g.t)
    assert r3["cached"] is False and r3["exec_workgroups"] == 256   # all equal: one per CU stays
    h = FakeRounds(lambda wg: 1.0 if wg == 192 else 1.01)
    r4 = autotune.tune_exec_workgroups(h.set_wg, h.run, 256, sig="s3", repeats=1, timer=lambda: h.t)
    assert r4["exec_workgroups"] == 256                              # 1% faster is within the margin
    r5 = autotune.tune_exec_workgroups(h.set_wg, h.run, 256, sig="s4", repeats=1, timer=lambda: h.t, margin=0.005)
    assert r5["exec_workgroups"] == 192
