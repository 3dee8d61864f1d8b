"""Autotuner host logic (no GPU): sampling and the cache round trip."""
import os

import pytest


class _T:
    def __init__(self, n):
        self.nrows = n


def test_sample_is_stratified_and_bounded():
    pytest.importorskip("torch")
    from paper_2606_24647_amd import autotune
    frags = [(_T(n), [], 10) for n in range(1, 5001)]
    s = autotune.sample_fragments(frags, k=100)
    assert 90 <= len(s) <= 100
    rows = sorted(t.nrows for t, _, _ in s)
    assert rows[0] == 1 and rows[-1] == 5000          # both ends of the size range
    small = autotune.sample_fragments(frags[:50], k=100)
    assert len(small) == 50


def test_cache_round_trip(tmp_path, monkeypatch):
    from paper_2606_24647_amd import autotune
    monkeypatch.setenv("GQ_AUTOTUNE_CACHE", str(tmp_path / "c.json"))
    assert autotune._load() == {}
    autotune._save({"k": {"config": {"tile_rows": 8192}}})
    assert autotune._load()["k"]["config"]["tile_rows"] == 8192
    assert os.path.exists(tmp_path / "c.json")


def test_coordinate_descent_finds_separable_minimum(monkeypatch):
    # A synthetic cost, separable in the parameters, with its minimum away from
    # the starting point: the search must reach it, and the check on the whole
    # workload must keep it.
    pytest.importorskip("torch")
    from paper_2606_24647_amd import autotune
    target = {"radix_min_groups": 1024, "lds_max_groups": 64, "load_factor": 0.7, "tile_rows": 16384,
              "blocks_per_cu": 2}
    calls = []

    def cost(ctx, frags, keys, aggs, cfg, reps=3):
        calls.append((len(frags), dict(cfg)))
        return 1.0 + sum(abs(autotune.CANDIDATES[k].index(cfg[k]) - autotune.CANDIDATES[k].index(v))
                         for k, v in target.items())

    monkeypatch.setattr(autotune, "time_plan", cost)
    monkeypatch.setattr(autotune, "shape_key", lambda frags: "test")
    frags = [(_T(n), [], 10) for n in range(1, 2001)]
    best = autotune.best_batch_config(None, frags, [0], [], use_cache=False)
    assert best == target
    assert any(n == 2000 for n, _ in calls)            # verified on the whole workload


def test_full_workload_check_keeps_start_when_sample_misleads(monkeypatch):
    pytest.importorskip("torch")
    from paper_2606_24647_amd import autotune

    def cost(ctx, frags, keys, aggs, cfg, reps=3):
        better = cfg["tile_rows"] == 4096
        if len(frags) == 2000:                          # whole workload: the sample's pick is worse
            return 2.0 if better else 1.0
        return 1.0 if better else 2.0

    monkeypatch.setattr(autotune, "time_plan", cost)
    monkeypatch.setattr(autotune, "shape_key", lambda frags: "test")
    frags = [(_T(n), [], 10) for n in range(1, 2001)]
    best = autotune.best_batch_config(None, frags, [0], [], use_cache=False)
    assert best == autotune.START
