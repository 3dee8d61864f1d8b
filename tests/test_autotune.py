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
