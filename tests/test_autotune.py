"""Host logic of the autotuner (no GPU): candidate choice, size buckets and
the JSON cache round trip."""
import json

from paper_2603_19764_amd import autotune


def test_choose_picks_fastest_and_keeps_first_on_ties():
    t = {4: 3.0, 8: 1.5, 16: 1.5}
    best, times = autotune.choose((4, 8, 16), t.__getitem__)
    assert best == 8 and times == t


def test_choose_keeps_earlier_candidate_within_margin():
    # 8 is 2% faster than 4: within the 5% margin, 4 stays; 16 is 7% faster
    t = {4: 1.00, 8: 0.98, 16: 1.01}
    assert autotune.choose((4, 8, 16), t.__getitem__)[0] == 4
    t = {4: 1.00, 8: 0.98, 16: 0.93}
    assert autotune.choose((4, 8, 16), t.__getitem__)[0] == 16
    assert autotune.choose((4, 8, 16), t.__getitem__, margin=0.0)[0] == 16
    t = {4: 1.00, 8: 0.98}
    assert autotune.choose((4, 8), t.__getitem__, margin=0.0)[0] == 8


def test_size_bucket_groups_powers_of_two():
    assert autotune.size_bucket(1) == 0
    assert autotune.size_bucket(226722) == autotune.size_bucket(200000) == 17
    assert autotune.size_bucket(7_158_540) == 22
    assert autotune.cache_key("gfx950", 1, 226722) == "gfx950|prec1|n2^17"


def test_cache_round_trip(tmp_path):
    p = tmp_path / "tune.json"
    c = autotune.TuneCache(str(p))
    assert c.get("k") is None
    c.put("k", {"lanes_step": 16, "cell_scale_permille": 1150})
    assert json.loads(p.read_text())["k"]["lanes_step"] == 16
    c2 = autotune.TuneCache(str(p))
    assert c2.get("k") == {"lanes_step": 16, "cell_scale_permille": 1150}


def test_knob_names_cover_plan():
    assert {autotune.KNOB_NAMES[k] for k, _, _ in autotune.PLAN} == set(autotune.KNOB_NAMES.values())


def test_per_precision_candidates_start_with_the_library_default():
    """Knobs with per-precision candidates list both precisions, with the
    same values in each and the library's default for that precision first
    (the choice keeps it unless another value is clearly faster)."""
    from paper_2603_19764_amd import sph
    defaults = {sph.SPH_FP64: 1, sph.SPH_FP32_CELLREL: 2}   # fused-sweep depth
    for knob, _, values in autotune.PLAN:
        if isinstance(values, dict):
            assert set(values) == {sph.SPH_FP64, sph.SPH_FP32_CELLREL}
            assert sorted(values[0]) == sorted(values[1])
            if knob == sph.SPH_TUNE_SWEEP_DEPTH:
                for prec, first in defaults.items():
                    assert values[prec][0] == first
