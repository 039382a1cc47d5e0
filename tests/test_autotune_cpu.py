"""The autotuner's cache (host logic only): keys by architecture, precision
and log2 N; an untuned size takes the nearest tuned one; contexts of
several clusters take the ensemble entry of their size when there is one
and a single-system entry otherwise; the shipped cache parses and holds
valid tunings."""
import json
import os

import pytest

from paper_0909_0879_amd import autotune, binding


@pytest.fixture
def arch(monkeypatch):
    monkeypatch.setattr(autotune, "arch_name", lambda: "gfx950")


def test_keys(arch):
    assert autotune.cache_key(binding.MIXED, 1 << 20) == "gfx950/mixed/20"
    assert autotune.cache_key(binding.FP64, 979217) == "gfx950/fp64/20"      # log2 rounded
    assert autotune.cache_key(binding.MIXED, 979217, True) == "gfx950/mixed/20/ensemble"


def test_store_and_load_with_ensemble_fallback(arch, tmp_path):
    path = str(tmp_path / "cache.json")
    assert autotune.load(binding.MIXED, 4096, path) is None
    autotune.store(binding.MIXED, 4096, {"variant": 1}, path)
    assert autotune.load(binding.MIXED, 4096, path) == {"variant": 1}
    # several clusters, no ensemble entry yet: the single-system one
    assert autotune.load(binding.MIXED, 4096, path, n_clusters=8) == {"variant": 1}
    autotune.store(binding.MIXED, 4096, {"variant": 2}, path, ensemble=True)
    assert autotune.load(binding.MIXED, 4096, path, n_clusters=8) == {"variant": 2}
    assert autotune.load(binding.MIXED, 4096, path, n_clusters=1) == {"variant": 1}
    assert autotune.load(binding.FP64, 4096, path) is None
    with open(path) as f:
        assert set(json.load(f)) == {"gfx950/mixed/12", "gfx950/mixed/12/ensemble"}


def test_nearest_tuned_size(arch, tmp_path):
    path = str(tmp_path / "cache.json")
    for b in (12, 16, 20):
        autotune.store(binding.MIXED, 1 << b, {"variant": b}, path)
    autotune.store(binding.MIXED, 1 << 20, {"variant": 99}, path, ensemble=True)
    assert autotune.load(binding.MIXED, 1 << 16, path)["variant"] == 16   # exact
    assert autotune.load(binding.MIXED, 1 << 17, path)["variant"] == 16   # tie: smaller
    assert autotune.load(binding.MIXED, 1 << 19, path)["variant"] == 20
    assert autotune.load(binding.MIXED, 1 << 8, path)["variant"] == 12
    assert autotune.load(binding.MIXED, 1 << 24, path)["variant"] == 20
    # ensembles: the ensemble entry of exactly their size, else the nearest
    # single-system one
    assert autotune.load(binding.MIXED, 1 << 20, path, n_clusters=4)["variant"] == 99
    assert autotune.load(binding.MIXED, 1 << 17, path, n_clusters=4)["variant"] == 16
    assert autotune.load(binding.FP64, 1 << 17, path) is None


def test_shipped_cache_is_valid():
    with open(autotune.DEFAULT_CACHE) as f:
        cache = json.load(f)
    assert cache
    for key, t in cache.items():
        parts = key.split("/")
        assert parts[1] in autotune.PRECISION_NAMES.values() and parts[2].isdigit(), key
        assert t["variant"] in (1, 2, 3, 4)
        assert t.get("acc_variant", 0) in (0, 1, 2, 3, 4)
        assert len(t["i_slots"]) == binding.TUNE_BUCKETS
        assert len(t["target_items"]) == binding.TUNE_BUCKETS
        for p in t["i_slots"]:
            assert 1 <= p <= 256 and p & (p - 1) == 0, key
        for q in t["target_items"]:
            assert 1 <= q <= (1 << 20), key
        # the binding turns every entry into the ABI struct
        tt = binding.Tuning.from_dict(t)
        assert tt.variant == t["variant"]
