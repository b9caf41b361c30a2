"""Autotuner host logic (CPU): candidate space, cache keys and the JSON
cache round trip.  The timing itself runs on the GPU (test_gpu_parity)."""
import json

from paper_2402_06083_amd import tune


def test_candidate_space():
    fp64 = list(tune.candidates("fp64"))
    mixed = list(tune.candidates("mixed"))
    assert len(fp64) == 2 * 6 * 2
    assert len(mixed) == len(fp64) * len(tune.MIXED_SWITCHES)
    assert all(set(c) <= set(tune.TUNED_FIELDS) for c in mixed)
    assert len({json.dumps(c, sort_keys=True) for c in mixed}) == len(mixed)


def test_cache_key_and_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert tune.load_cache(path) == {}
    k1 = tune.cache_key("gfx950", [(0, 1), (0, 2)], "fp64")
    k2 = tune.cache_key("gfx950", [(0, 1), (0, 2)], "mixed")
    k3 = tune.cache_key("gfx950", [(0, 2), (0, 1)], "fp64")
    k4 = tune.cache_key("gfx950", [(0, 1), (0, 2)], "fp64", simple=True)
    assert len({k1, k2, k3, k4}) == 4
    tune.save_cache({k1: {"options": {"block_size": 128}, "ms": 1.0, "default_ms": 2.0}}, path)
    assert tune.lookup([(0, 1), (0, 2)], "fp64", path=path, arch="gfx950")["options"] == {"block_size": 128}
    assert tune.lookup([(0, 1), (0, 2)], "mixed", path=path, arch="gfx950") is None
    assert tune.lookup([(0, 1), (0, 2)], "fp64", path=path, arch="gfx950", simple=True) is None


def test_corrupt_cache_is_ignored(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    assert tune.load_cache(str(path)) == {}


def test_options_from_candidate():
    o = tune._options("mixed", True, {"block_size": 128, "seg_points": 64, "points_per_turn": 16,
                                      "fp32_switch": 2.0 ** -10})
    assert (o.block_size, o.seg_points, o.points_per_turn, o.fp32_switch) == (128, 64, 16, 2.0 ** -10)
    assert o.flags & 1 and o.precision == 1


def test_simple_flag_reaches_options():
    from paper_2402_06083_amd import msplit
    o = tune._options("fp64", True, {}, simple=True)
    assert o.flags & msplit.F_SIMPLE and o.flags & msplit.F_CERTIFY
    assert not tune._options("fp64", True, {}).flags & msplit.F_SIMPLE
