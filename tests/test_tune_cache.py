"""The autotuner's per-device cache (host logic only)."""
import json

from paper_2010_03090_amd import tune


def test_cache_roundtrip_and_key_match(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    key_a = {"device": "gpu-a", "arch": "gfx950", "cus": 256, "library": "abc"}
    key_b = dict(key_a, library="def")
    assert tune.read_cache(path) == []
    tune.store(key_a, {"unroll": 4, "waves_per_cu": 24}, {"single_ms": [1.0]}, path)
    tune.store(key_b, {"unroll": 2, "waves_per_cu": 16}, {}, path)
    entries = tune.read_cache(path)
    assert len(entries) == 2
    assert tune.lookup(key_a, entries) == {"unroll": 4, "waves_per_cu": 24}
    assert tune.lookup(key_b, entries) == {"unroll": 2, "waves_per_cu": 16}
    assert tune.lookup(dict(key_a, cus=128), entries) is None        # other device shape: not applied
    tune.store(key_a, {"unroll": 8, "waves_per_cu": 40}, {}, path)   # replaces, does not duplicate
    entries = tune.read_cache(path)
    assert len(entries) == 2 and tune.lookup(key_a, entries)["unroll"] == 8


def test_corrupt_cache_is_ignored(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    assert tune.read_cache(str(path)) == []
    path.write_text(json.dumps({"key": 1}))
    assert tune.read_cache(str(path)) == []
    path.write_text(json.dumps([{"key": {"x": 1}, "config": "bad"}]))
    assert tune.lookup({"x": 1}, tune.read_cache(str(path))) is None
