"""Tuned-parameter cache on the CPU: keys, persistence across instances,
atomic rewrite, rejection of bad entries, and that a cache hit sets the
parameters without tuning (the tuner and setter are injected)."""
import json
import os
from types import SimpleNamespace

import pytest

from paper_1711_00231_amd import tuning

G = SimpleNamespace(n=4096, m=65536)


def _tuner(result):
    calls = []

    def tune(g, sources):
        calls.append((g.n, g.m, tuple(sources)))
        return dict(result)

    return tune, calls


def test_key_format_and_validation():
    assert tuning.cache_key("rmat", 10, 20, "gfx950") == "rmat|n=10|m=20|arch=gfx950"
    for bad in ("", "a|b"):
        with pytest.raises(ValueError):
            tuning.cache_key(bad, 1, 1, "gfx950")


def test_miss_tunes_then_hit_reuses(tmp_path):
    path = str(tmp_path / "sub" / "bins.json")
    applied = []
    tune, calls = _tuner({"mdt": 1024, "t_wave": 32, "t_block": 256})
    b, hit = tuning.tuned_bins(G, [1, 2], "rmat", tuning.BinsCache(path), "gfx950", tune,
                               lambda **k: applied.append(k))
    assert not hit and calls == [(4096, 65536, (1, 2))] and applied == [b]
    # a new cache object (another process) hits without tuning
    b2, hit2 = tuning.tuned_bins(G, [1, 2], "rmat", tuning.BinsCache(path), "gfx950", tune,
                                 lambda **k: applied.append(k))
    assert hit2 and b2 == b and len(calls) == 1 and applied == [b, b]
    # another architecture, class or size is another key
    for cls, arch, g in (("rmat", "gfx942", G), ("grid", "gfx950", G),
                         ("rmat", "gfx950", SimpleNamespace(n=4096, m=65537))):
        tuning.tuned_bins(g, [1], cls, tuning.BinsCache(path), arch, tune, lambda **k: None)
    assert len(calls) == 4
    data = json.load(open(path))
    assert data["version"] == tuning.VERSION and len(data["entries"]) == 4
    assert not [f for f in os.listdir(os.path.dirname(path)) if f.endswith(".tmp")]


def test_bad_entries_and_files_are_ignored(tmp_path):
    path = tmp_path / "bins.json"
    key = tuning.cache_key("uniform", G.n, G.m, "gfx950")
    good = tuning.cache_key("grid", 1, 2, "gfx950")
    path.write_text(json.dumps({"version": 1, "entries": {
        key: {"mdt": 10, "t_wave": 8, "t_block": 16},          # mdt below the minimum
        good: {"mdt": 0, "t_wave": 0, "t_block": 0}}}))
    c = tuning.BinsCache(str(path))
    assert c.get(key) is None and c.get(good) == {"mdt": 0, "t_wave": 0, "t_block": 0}
    tune, calls = _tuner({"mdt": 256, "t_wave": 16, "t_block": 1024})
    b, hit = tuning.tuned_bins(G, [0], "uniform", c, "gfx950", tune, lambda **k: None)
    assert not hit and calls and c.get(key) == b and c.get(good) is not None
    path.write_text("{not json")
    with pytest.warns(UserWarning):
        assert c.load() == {}
    path.write_text(json.dumps({"version": 99, "entries": {}}))
    with pytest.warns(UserWarning):
        assert c.load() == {}
    with pytest.raises(ValueError):
        c.put(key, {"mdt": 128, "t_wave": 64, "t_block": 32})


def test_default_path_follows_environment(monkeypatch, tmp_path):
    monkeypatch.setenv("LBG_TUNE_CACHE", str(tmp_path / "x.json"))
    assert tuning.BinsCache().path == str(tmp_path / "x.json")
    monkeypatch.delenv("LBG_TUNE_CACHE")
    assert tuning.default_path().endswith(os.path.join(".cache", "lbg", "bins.json"))
