"""Autotuner host logic (no GPU): candidate sets, size buckets, JSON cache."""
import json

from paper_2106_08759_amd import autotune


def test_candidates_cover_the_knobs():
    c761 = autotune.candidates(761, 65536)
    assert {c["group_size"] for c in c761} == set(autotune.GROUP_SIZES)
    assert {c["lanes_per_key"] for c in c761} == {1, 2, 4, 8}
    assert {c["retry_passes"] for c in c761} == {1}
    c1277 = autotune.candidates(1277, 65536)
    assert {c["lanes_per_key"] for c in c1277} == {1, 2, 4, 8}
    assert {c["retry_passes"] for c in c1277} == {0, 1}
    assert {c["retry_lanes_per_key"] for c in c1277} == {4, 8}
    assert {c["retry_parallel_attempts"] for c in c1277} == {2, 4, 8}
    assert all(c["retry_lanes_per_key"] * c["retry_parallel_attempts"] <= 64 for c in c1277)
    assert all(c["group_size"] <= 16 for c in autotune.candidates(761, 10))
    assert {c["group_size"] for c in autotune.candidates(761, 10)} == {8, 16}
    assert {c["inverse_share"] for c in c761} == {1, 2, 4, 8}
    assert {c["inverse_share"] for c in c1277} == {1, 2, 4}          # LDS bound for p = 1277
    assert {(c["group_size"], c["inverse_share"]) for c in autotune.candidates(761, 10)} == {(8, 1), (8, 2), (16, 1)}


def test_bucket():
    assert [autotune.bucket(n) for n in (1, 2, 3, 1000, 1024, 1025, 65536)] == [1, 2, 4, 1024, 1024, 2048, 65536]


def test_cache_roundtrip(tmp_path):
    path = str(tmp_path / "tune.json")
    assert autotune.load_cache(path) == {}
    entry = {"config": {"group_size": 32, "lanes_per_key": 2, "retry_passes": 1, "retry_lanes_per_key": 8}, "ms": 5.6}
    data = {autotune._key("dev", 761, 60000): entry}
    autotune.save_cache(data, path)
    assert json.load(open(path)) == data
    assert autotune.lookup("dev", 761, 65536, path) == entry      # same bucket
    assert autotune.lookup("dev", 761, 70000, path) is None       # next bucket
    assert autotune.lookup("other", 761, 65536, path) is None
    assert autotune.lookup("dev", 761, 65536, path, mode="graph") is None   # per launch form


def test_phase1_times_group_knobs_with_each_lane_count():
    c = autotune.phase1_candidates(761, 65536)
    assert {x["lanes_per_key"] for x in c} == set(autotune.PHASE1_LANES)
    assert 1 in autotune.PHASE1_LANES   # one lane per key: the live-word divstep form
    # every (G, W) pair appears once per lane count
    pairs = [(x["group_size"], x["inverse_share"]) for x in c]
    assert len(pairs) == len(autotune.PHASE1_LANES) * len(autotune.group_candidates(761, 65536))
    assert (32, 8) in pairs and (64, 2) in pairs


def test_persistent_form_is_a_knob():
    assert "persistent" in autotune.KNOBS
    for g, w, l in autotune.PERSISTENT_CANDIDATES:
        assert l in (2, 4) and w in autotune.SHARES and g in autotune.GROUP_SIZES
