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


class FakeMulti(FakeForest):
    def __init__(self, th, cost):
        super().__init__(cost)
        self.th = th
        self.small = (0, 0)
        self.closed = False

    def set_small_schedule(self, t, w):
        self.small = (t, w)

    def close(self):
        self.closed = True


def test_tune_batched_searches_threshold_schedule_and_rounds(monkeypatch):
    monkeypatch.setattr("paper_2607_20211_amd.drsf.drsf_snapshot_free", lambda s: None)
    clock = [0.0]
    monkeypatch.setattr(autotune.time, "perf_counter", lambda: clock[0])
    made = []

    def cost(f):
        c = {0: 5.0, 1024: 4.0, 2048: 3.0, 4096: 3.5, 8192: 6.0}[f.th]
        c -= 0.5 if f.small == (1024, 128) else 0.0
        c -= 0.25 if f.setting == (4, 2, 0) else 0.0
        return c

    def make(th):
        f = FakeMulti(th, None)
        made.append(f)
        return f

    def sample(fr):
        clock[0] += cost(fr)

    f, ch = autotune.tune_batched(make, sample, "b")
    assert f.th == 2048 and not f.closed
    assert all(m.closed for m in made if m is not f)
    assert (ch["small_threads"], ch["small_workgroups"]) == (1024, 128) and f.small == (1024, 128)
    assert (ch["rounds_queued"], ch["levels_queued"], ch["sweep_mode"]) == (4, 2, 0)
    assert ch["small_graph_vertices"] == 2048
