"""The schedule tuner's cache (host only): results round-trip through the
JSON file, keyed per GPU architecture, engine kind and size bucket."""
from paper_2309_00338_amd import tune


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "c" / "sched.json")
    assert tune.load_cache(path) == {}
    assert tune.schedule_for("gfx950/one/cells2^26/grids2^0", path) is None
    cache = {"gfx950/one/cells2^26/grids2^0": {"schedule": {"frac_near_per_cu": 5.5, "sweep_per_cu": 16},
                                                 "us_per_step": 437.0}}
    tune.save_cache(cache, path)
    assert tune.load_cache(path) == cache
    assert tune.schedule_for("gfx950/one/cells2^26/grids2^0", path)["sweep_per_cu"] == 16


def test_candidates_cover_the_schedule_fields():
    from paper_2309_00338_amd import ebit

    assert set(tune.CANDIDATES) == set(ebit.SCHEDULE_FIELDS)
    assert set(tune.ONE_GRID) <= set(tune.SEVERAL) <= set(tune.CANDIDATES)
