"""Launch-shape knobs: every setting the autotuner may pick gives the same
step (FP64, up to the order of the pair sums), and the tuner returns valid
settings."""
import numpy as np
import pytest

from paper_2603_19764_amd import inputs
from tests.gpu_harness import norm_err, say

pytestmark = pytest.mark.gpu

FIELDS = ("x", "vx", "u", "S", "a", "dudt", "dS", "rho", "G")


def _steps(w, prec, knobs, steps=2):
    import torch
    from paper_2603_19764_amd import sph
    n = int(w["x"].size)
    ctx = sph.Context(n, 128)
    for knob, v in knobs.items():
        sph.sph_set_tuning(ctx, knob, prec, v)
        assert sph.sph_get_tuning(ctx, knob, prec) == v
    st = sph.State(w)
    sph.sph_init(ctx, st, w["mats"], w["params"], prec)
    for _ in range(steps):
        sph.sph_step(ctx, st, w["mats"], w["params"], prec)
    torch.cuda.synchronize()
    ctx.check(sph.lib().sph_sync_status(ctx.h, None))
    out = st.to_host()
    ctx.close()
    return out


@pytest.mark.parametrize("prec", [0, 1])
def test_every_knob_setting_gives_the_same_step(prec):
    from paper_2603_19764_amd import sph
    w = inputs.c1_block(10, variant="s")
    ref = _steps(w, prec, {})
    # FP64: only the order of the pair sums changes.  FP32: the cell grid
    # also moves the cell-relative origins; each result is within the FP32
    # parity bounds of the FP64 oracle (largest 2e-5, du/dt), so two of them
    # are within twice that of each other.
    tol = 1e-12 if prec == 0 else 4e-5
    for knobs in ({sph.SPH_TUNE_LANES_STEP: 4, sph.SPH_TUNE_LANES_DENSITY: 16},
                  {sph.SPH_TUNE_LANES_STEP: 16, sph.SPH_TUNE_LANES_DENSITY: 4},
                  {sph.SPH_TUNE_CELL_SCALE: 1300},
                  {sph.SPH_TUNE_BUILD_RANGE: 32}, {sph.SPH_TUNE_BUILD_RANGE: 128},
                  {sph.SPH_TUNE_SWEEP_DEPTH: 1}, {sph.SPH_TUNE_SWEEP_DEPTH: 2},
                  {sph.SPH_TUNE_BUILD_TILE: 128}, {sph.SPH_TUNE_BUILD_TILE: 192},
                  {sph.SPH_TUNE_SWEEP_DEPTH: 1, sph.SPH_TUNE_LANES_STEP: 4}):
        got = _steps(w, prec, knobs)
        e = max(norm_err(got[k], ref[k]) for k in FIELDS)
        say(f"prec {prec} knobs {knobs}: max err {e:.1e}")
        assert e <= tol


def test_bad_knob_values_are_rejected():
    from paper_2603_19764_amd import sph
    ctx = sph.Context(16, 32)
    for knob, v in ((sph.SPH_TUNE_LANES_STEP, 3), (sph.SPH_TUNE_CELL_SCALE, 999),
                    (sph.SPH_TUNE_BUILD_RANGE, 48), (sph.SPH_TUNE_SWEEP_DEPTH, 3),
                    (sph.SPH_TUNE_BUILD_TILE, 100), (17, 8)):
        with pytest.raises(sph.SphError):
            sph.sph_set_tuning(ctx, knob, 0, v)
    ctx.close()


def test_tuner_returns_valid_settings(tmp_path):
    from paper_2603_19764_amd import autotune
    w = inputs.c1_block(12)
    cache = autotune.TuneCache(str(tmp_path / "tune.json"))
    r = autotune.tune(w, 1, steps=2, cache=cache)
    say("tuned", r["settings"])
    s = r["settings"]
    assert s["lanes_step"] in autotune.LANES and s["lanes_density"] in autotune.LANES
    assert s["cell_scale_permille"] in autotune.CELL_SCALES
    assert s["build_range"] in autotune.BUILD_RANGES
    assert s["sweep_depth"] in autotune.SWEEP_DEPTHS[1]
    assert s["build_tile"] in autotune.BUILD_TILES
    again = autotune.tune(w, 1, steps=2, cache=cache)
    assert again["cached"] and again["settings"] == s
