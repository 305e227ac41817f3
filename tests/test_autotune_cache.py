"""The autotuning cache (host logic only): keys, round trip through the
JSON file, and recovery from a missing or corrupt file."""
import json
import os

from paper_2310_14649_amd.autotune import TuneCache, default_path, make_key


def test_key_is_order_independent_and_distinguishes_shapes():
    a = make_key("sg_matvec", "gfx950", n=10, P=35, L=15)
    b = make_key("sg_matvec", "gfx950", L=15, P=35, n=10)
    assert a == b
    assert a != make_key("sg_matvec", "gfx950", n=11, P=35, L=15)
    assert a != make_key("sg_matvec", "gfx942", n=10, P=35, L=15)
    assert a != make_key("ras_apply", "gfx950", n=10, P=35, L=15)


def test_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    c = TuneCache(path)
    assert c.get("k") is None
    c.put("k", {"tiles": 2, "ms": [0.13, 0.11, 0.15]})
    c.put("r", {"path": "dense"})
    d = TuneCache(path)
    assert d.get("k") == {"tiles": 2, "ms": [0.13, 0.11, 0.15]}
    assert d.get("r") == {"path": "dense"}
    assert json.load(open(path))["version"] == 1
    assert [f for f in os.listdir(os.path.dirname(path)) if f.startswith(".autotune.")] == []


def test_corrupt_or_foreign_file_starts_empty(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    assert TuneCache(str(path)).entries == {}
    path.write_text(json.dumps([1, 2, 3]))
    c = TuneCache(str(path))
    assert c.entries == {}
    c.put("k", 1)
    assert TuneCache(str(path)).get("k") == 1


def test_default_path_follows_environment(monkeypatch, tmp_path):
    monkeypatch.setenv("SGSOLVE_TUNE_CACHE", str(tmp_path / "x.json"))
    assert default_path() == str(tmp_path / "x.json")
    monkeypatch.delenv("SGSOLVE_TUNE_CACHE")
    monkeypatch.setenv("XDG_CACHE_HOME", str(tmp_path))
    assert default_path() == os.path.join(str(tmp_path), "sgsolve", "autotune.json")
