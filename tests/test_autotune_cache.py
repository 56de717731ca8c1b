"""Host logic of the tuning cache (no GPU)."""
from paper_2512_13267_amd import autotune


def test_histogram_and_key():
    assert autotune.size_histogram([1536, 2000, 4000, 4000, 12288]) == "2^10:2,2^11:2,2^13:1"
    assert autotune.size_histogram([4000] * 3) == "2^11:3"
    k1 = autotune.cache_key("gfx950", "fp32", [4000, 4001])
    k2 = autotune.cache_key("gfx950", "fp32", [4001, 4000])
    assert k1 == k2 and k1.startswith("gfx950|fp32|")
    assert autotune.cache_key("gfx950", "fp64", [4000]) != autotune.cache_key("gfx950", "fp32", [4000])
    # a different build of the library never reuses an entry
    assert autotune.cache_key("gfx950", "fp32", [4000], "aaaa") != autotune.cache_key("gfx950", "fp32", [4000], "bbbb")
    assert len(autotune.library_digest()) == 12


def test_store_and_load_roundtrip(tmp_path):
    path = str(tmp_path / "sub" / "cache.json")
    assert autotune.load_cache(path) == {}
    autotune.store("a", {"config": {"queue_depth": 4}}, path)
    autotune.store("b", {"config": {"queue_depth": 8}}, path)
    data = autotune.load_cache(path)
    assert data["a"]["config"]["queue_depth"] == 4 and data["b"]["config"]["queue_depth"] == 8
    (tmp_path / "bad.json").write_text("not json")
    assert autotune.load_cache(str(tmp_path / "bad.json")) == {}
