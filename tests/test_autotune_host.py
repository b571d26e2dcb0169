"""Host side of the launch-shape tuner: candidate sets the library accepts,
cache round trips, and lookups that need no timing."""
import json

import pytest

from paper_2110_07670_amd import _lib, autotune

GRIDS = [16, 24, 32, 40, 48, 64, 80, 96, 120, 128, 144, 160, 192]


@pytest.mark.parametrize("n", GRIDS)
@pytest.mark.parametrize("n_orb", [4, 9, 17, 128])
def test_every_candidate_is_a_valid_tiling(n, n_orb):
    plan = _lib.Plan(n, (10.0,) * 3, n_orb, "fp64", 0.25)
    for block, chunk in autotune.tile_candidates(n_orb):
        for c in [0] + autotune.pencil_candidates(n):
            plan.set_tiling(block, chunk, c)
            assert plan.tiling == (block, chunk, c)


def test_pencil_candidates_skip_the_default():
    assert autotune.pencil_candidates(96) == [8, 32]
    assert autotune.pencil_candidates(48) == [8]
    assert autotune.pencil_candidates(40) == []
    assert autotune.pencil_candidates(24) == []


def test_cache_round_trip_and_apply_without_tuning(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert autotune.load_cache(path) == {}
    k = autotune.key(48, "fp32", 20)
    autotune.save_cache({k: {"block": 8, "chunk": 32, "pencils": 8, "ms": 1.5, "tried": []}}, path)
    with open(path) as f:
        assert json.load(f)[k]["pencils"] == 8
    plan = _lib.Plan(48, (10.0,) * 3, 20, "fp32", 0.25)
    assert autotune.apply(plan, "fp32", cache_path=path, tune_missing=False) == (8, 32, 8)
    # a key that is not cached leaves the plan as it is when tuning is off
    other = _lib.Plan(64, (10.0,) * 3, 20, "fp32", 0.25)
    assert autotune.apply(other, "fp32", cache_path=path, tune_missing=False) == (16, 0, 0)


def test_tile_candidates_cover_blocks_and_splitting_chunks():
    c = autotune.tile_candidates(128)
    assert (16, 0) in c and (8, 0) in c
    # a chunk only where it splits a full tile's transforms (128 or 32)
    assert {ch for b, ch in c if b == 16} == {0, 16, 32, 64}
    assert {ch for b, ch in c if b == 8} == {0, 16}
    assert autotune.tile_candidates(8) == [(16, 0)]


def test_cached_four_pass_schedule_is_applied(tmp_path):
    path = str(tmp_path / "tune.json")
    k = autotune.key(64, "fp64", 12)
    autotune.save_cache({k: {"block": 8, "chunk": 0, "pencils": 16, "four_pass": True,
                             "ms": 1.0, "tried": []}}, path)
    plan = _lib.Plan(64, (10.0,) * 3, 12, "fp64", 0.25)
    assert autotune.apply(plan, "fp64", cache_path=path, tune_missing=False) == (8, 0, 16)
    assert plan.four_pass


def test_batch_cache_lookup_sets_every_instance(tmp_path):
    path = str(tmp_path / "tune.json")
    plans = [_lib.Plan(n, (10.0,) * 3, k, "fp32", 0.25) for n, k in [(48, 20), (96, 64)]]
    key = autotune.batch_key([(p.n, p.n_orb) for p in plans], "fp32")
    assert key == "batch/fp32/48x20,96x64"
    autotune.save_cache({key: {"shapes": [[8, 0, 0, False], [16, 32, 8, True]], "ms": 3.0,
                               "tried": []}}, path)
    e = autotune.tune_batch(plans, "fp32", cache_path=path)
    assert e["ms"] == 3.0 and e["lanes"]  # entries without the mode: the lanes
    assert plans[0].tiling == (8, 0, 0) and not plans[0].four_pass
    assert plans[1].tiling == (16, 32, 8) and plans[1].four_pass
