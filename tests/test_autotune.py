"""Host logic of the autotuner (no GPU)."""
from paper_2208_14639_amd import autotune


def test_bucket_keys():
    assert autotune.bucket_key(27000, 18, "bf16x3") == "gfx950:bf16x3:P4:N32768"
    assert autotune.bucket_key(120000, 60, "fp64") == "gfx950:fp64:P12:N122880"
    assert autotune.bucket_key(1, 1, "fp32") == "gfx950:fp32:P1:N8192"


def test_candidates_bounded_and_include_auto():
    c = autotune.candidates(9, 1, 20)
    assert 9 in c and min(c) >= 1 and max(c) <= 20 and c == sorted(set(c))
    assert autotune.candidates(1, 1, 1) == [1]


def test_cache_roundtrip(tmp_path):
    path = str(tmp_path / "t.json")
    assert autotune.load_cache(path) == {}
    cache = {autotune.bucket_key(27000, 18, "bf16x3"): {"jsplit": 7, "bgroups": 9}}
    autotune.save_cache(cache, path)
    back = autotune.load_cache(path)
    assert autotune.lookup(27000, 18, "bf16x3", back) == (7, 9)
    assert autotune.lookup(27000, 18, "fp64", back) is None
