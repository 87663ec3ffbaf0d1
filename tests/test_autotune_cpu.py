"""Autotuner search logic (no GPU): coordinate search over a synthetic cost."""
from paper_1312_3691_amd import autotune as AT


def test_search_finds_separable_minimum():
    want = {"refill_lanes": 32, "tile_particles": 65536, "groups_per_cu": 4}

    def cost(t):
        return sum(abs(t[k] - want[k]) / want[k] for k in want)

    best, trials = AT.coordinate_search(cost)
    assert best == want
    keys = [tuple(sorted(t.tuning.items())) for t in trials]
    assert len(keys) == len(set(keys)), "a setting was measured twice"
    assert trials[0].tuning == AT.DEFAULT


def test_search_keeps_start_on_ties_and_flat_cost():
    best, trials = AT.coordinate_search(lambda t: 1.0)
    assert best == AT.DEFAULT
    # one pass over every axis value, nothing repeated
    assert len(trials) == 1 + sum(len(v) - 1 for _, v in AT.AXES)


def test_search_coupled_axes_second_round():
    # the best tile depends on refill: a second round follows the coupling
    def cost(t):
        good_tile = 4096 if t["refill_lanes"] == 24 else 16384
        return (0.0 if t["refill_lanes"] == 24 else 1.0) + (0.0 if t["tile_particles"] == good_tile else 0.5)

    best, _ = AT.coordinate_search(cost, rounds=2)
    assert best["refill_lanes"] == 24 and best["tile_particles"] == 4096


def test_sample_queries_scales_particles():
    qs = [{"n": 10_000_000}, {"n": 30_000_000}]
    s = AT.sample_queries(qs, 4_000_000)
    assert [q["n"] for q in s] == [1_000_000, 3_000_000]
    assert AT.sample_queries(qs, 10 ** 9) == qs
    assert AT.sample_queries([{"n": 100}, {"n": 10 ** 8}], 10 ** 6)[0]["n"] == 100
    tiny = AT.sample_queries([{"n": 10_000_000}, {"n": 5000}], 1_000_000)
    assert min(q["n"] for q in tiny) >= 4096


def test_held_settings_are_not_searched():
    axes = AT.free_axes({"tile_particles": 65536})
    assert [name for name, _ in axes] == ["refill_lanes", "groups_per_cu"]
    start = dict(AT.DEFAULT, tile_particles=65536)
    best, trials = AT.coordinate_search(lambda t: t["refill_lanes"] + t["groups_per_cu"], start=start, axes=axes)
    assert all(t.tuning["tile_particles"] == 65536 for t in trials)
    assert best == {"refill_lanes": 16, "tile_particles": 65536, "groups_per_cu": 4}
    assert AT.free_axes(None) == list(AT.AXES)
    try:
        AT.free_axes({"tiles": 1})
    except ValueError:
        pass
    else:
        raise AssertionError("an unknown field must be rejected")
