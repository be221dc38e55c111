"""Host-side logic that needs no GPU: the tuner cache, the benchmark's
traffic lookup against the committed counter summary, and its argument
defaults."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2509_19267_amd import tune  # noqa: E402


def test_tuned_choices_are_complete():
    for form in ("fp64", "mixed_f32"):
        ch = tune.lookup("dense", 20000, 5000, form)
        assert ch is not None, form
        for key in ("k_col", "k_row", "inner_tol", "inner_max", "tile_rows"):
            assert key in ch, (form, key)
        assert 0 < ch["k_col"] <= 5000 and 0 < ch["k_row"] <= 5000


def test_counted_traffic_matches_the_tuned_tiles():
    # the committed counter summary is for the tuned row tiles: the
    # benchmark's roofline then carries measured traffic, not null
    for form, prec in (("fp64", "f64"), ("mixed_f32", "f32")):
        tr = tune.lookup("dense", 20000, 5000, form)["tile_rows"]
        t = bench.counted_traffic(prec, tr, 20000, 5000)
        assert isinstance(t, int), (form, tr)
        alg = 20000 * 5000 * (8 if prec == "f64" else 4)
        assert alg <= t <= 1.1 * alg
    assert bench.counted_traffic("f32", 12345, 20000, 5000) is None
    assert bench.counted_traffic("f32", 224, 1000, 500) is None


def test_tune_cache_roundtrip(tmp_path, monkeypatch):
    monkeypatch.setattr(tune, "CACHE", str(tmp_path / "t.json"))
    assert tune.lookup("dense", 3, 4, "fp64") is None
    tune.store("dense", 3, 4, "fp64", {"k_col": 2, "k_row": 3})
    tune.store("dense", 3, 4, "mixed_f32", {"k_col": 1, "k_row": 1})
    assert tune.lookup("dense", 3, 4, "fp64") == {"k_col": 2, "k_row": 3}
    data = json.load(open(tmp_path / "t.json"))
    assert set(data) == {"dense:3x4:fp64", "dense:3x4:mixed_f32"}


def test_bench_defaults(monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    a = bench.parse()
    assert a.gpus == 1 and a.steps >= 1 and a.warmup >= 0
    assert (a.m, a.n, a.tol) == (20000, 5000, 1e-8)
