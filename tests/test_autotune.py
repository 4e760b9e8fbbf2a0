"""Autotuner logic on the CPU: a stand-in forest records the settings it is
given and reports a chosen cost per setting."""
from __future__ import annotations

import json

from paper_2607_20211_amd import autotune


class FakeForest:
    def __init__(self, cost):
        self.cost = cost
        self.setting = None
        self.restores = 0

    def set_tuning(self, r, l, m):
        self.setting = (r, l, m)

    def snapshot(self):
        return None

    def restore(self, snap):
        self.restores += 1


def test_tune_picks_fastest_and_caches(tmp_path, monkeypatch):
    monkeypatch.setenv("DRSF_TUNE_CACHE", str(tmp_path / "tune.json"))
    monkeypatch.setattr("paper_2607_20211_amd.drsf.drsf_snapshot_free", lambda s: None)
    clock = [0.0]
    monkeypatch.setattr(autotune.time, "perf_counter", lambda: clock[0])
    best = (3, 4, 1)
    f = FakeForest(lambda s: 1.0 if s == best else 2.0 + s[0] * 0.01)

    def sample(fr):
        clock[0] += fr.cost(fr.setting)

    r = autotune.tune(f, sample, "k1")
    assert (r["rounds_queued"], r["levels_queued"], r["sweep_mode"]) == best
    assert f.setting == best and not r["cached"] and r["tried"] == len(autotune.CANDIDATES)
    saved = json.load(open(tmp_path / "tune.json"))
    assert saved["k1"]["rounds_queued"] == 3
    # a second call takes the cached choice without measuring
    f2 = FakeForest(lambda s: 5.0)
    r2 = autotune.tune(f2, sample, "k1")
    assert r2["cached"] and f2.setting == best and f2.restores == 0
