"""Autotuner cache and selection logic (CPU, with a synthetic timer)."""
from paper_1903_10959_amd import autotune as AT


class _Ctx:
    p = 6


def test_candidates_cover_the_block():
    assert AT.candidates(568) == [64, 128, 192, 256, 384, 512, 568]
    assert AT.candidates(24) == [24]


def test_tuner_picks_fastest_and_caches(tmp_path):
    path = str(tmp_path / "cache.json")
    calls = []

    def timer(w):
        calls.append(w)
        return abs(w - 192) + 1.0      # fastest at 192

    assert AT.tune_block_width(_Ctx(), 568, None, "fp64", cache_path=path, timer=timer, arch="gfx950") == 192
    n = len(calls)
    # cached: no new timings
    assert AT.tune_block_width(_Ctx(), 568, None, "fp64", cache_path=path, timer=timer, arch="gfx950") == 192
    assert len(calls) == n
    # a different precision is a different key
    AT.tune_block_width(_Ctx(), 568, None, "fp32", cache_path=path, timer=timer, arch="gfx950")
    assert len(calls) > n
    c = AT.load_cache(path)
    assert set(c) == {"gfx950|p6|nb568|fp64", "gfx950|p6|nb568|fp32"}


def test_ties_prefer_the_smaller_width():
    assert AT.pick({128: 1.0, 256: 1.0, 64: 2.0}) == 128


def test_tile_variant_tuner_picks_fastest_and_caches(tmp_path):
    path = str(tmp_path / "cache.json")
    calls = []

    def timer(v):
        calls.append(v)
        return {0: 2.0, 1: 1.5}[v]

    assert AT.tune_tile_variant(_Ctx(), None, None, "fp32", cache_path=path, timer=timer, arch="gfx950") == 1
    assert calls == [0, 1]
    assert AT.tune_tile_variant(_Ctx(), None, None, "fp32", cache_path=path, timer=timer, arch="gfx950") == 1
    assert calls == [0, 1]                      # cached
    assert "tile|gfx950|p6|fp32" in AT.load_cache(path)


def test_tile_variant_ties_prefer_variant_zero():
    assert AT.pick({0: 1.0, 1: 1.0}) == 0


def test_cells_per_tile_tuner_picks_fastest_per_column_count(tmp_path):
    path = str(tmp_path / "cache.json")
    seen = []

    def timer(cpt):
        seen.append(cpt)
        return {1: 3.0, 2: 1.0, 4: 2.0}[cpt]

    assert AT.tune_cells_per_tile(_Ctx(), 24, None, "fp32", cache_path=path, timer=timer, arch="gfx950") == 2
    assert sorted(seen) == [1, 2, 4]
    n = len(seen)
    assert AT.tune_cells_per_tile(_Ctx(), 24, None, "fp32", cache_path=path, timer=timer, arch="gfx950") == 2
    assert len(seen) == n                      # cached
    AT.tune_cells_per_tile(_Ctx(), 40, None, "fp32", cache_path=path, timer=timer, arch="gfx950")
    assert len(seen) > n                       # another column count is another key


def test_cells_per_tile_tuner_keeps_one_cell_above_p6(tmp_path):
    class _P7:
        p = 7
    seen = []
    AT.tune_cells_per_tile(_P7(), 24, None, "fp32", cache_path=str(tmp_path / "c.json"),
                           timer=lambda c: seen.append(c) or 1.0, arch="gfx950")
    assert seen == [1]
