"""Autotuner bookkeeping (no GPU): keys, cache round trip, choice."""
from paper_1212_2245_amd import autotune


def test_classes_and_key():
    assert autotune.radius_class(31, 31) == 16
    assert autotune.radius_class(1, 15) == 8
    assert autotune.radius_class(65, 1) == 32
    assert autotune.size_class(1024, 1024) == 1 << 20
    assert autotune.size_class(768, 768) == 1 << 20
    assert autotune.size_class(192, 192) == 1 << 16
    assert autotune.key("gfx950", "7.0", 512, 512, 31, 31) == "gfx950|7.0|px262144|r16"


def test_cache_round_trip_and_choice(tmp_path, monkeypatch):
    path = str(tmp_path / "sub" / "tiles.json")
    monkeypatch.setenv(autotune.CACHE_ENV, path)
    assert autotune.cache_path() == path
    assert autotune.load_cache() == {}
    autotune.save_cache({"k": {"tile": 3}})
    assert autotune.load_cache() == {"k": {"tile": 3}}
    assert autotune.choose({1: 5.0, 2: 3.0, 3: 3.0, 4: 9.0}) == 2
    (tmp_path / "bad.json").write_text("not json")
    assert autotune.load_cache(str(tmp_path / "bad.json")) == {}
