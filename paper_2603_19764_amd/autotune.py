"""Autotuner of the launch shapes of the step: lanes per particle of the
fused gradient + force sweep and of the density sweep, and the cell edge
(as a multiple of 2 h_max).

Each candidate is timed with the library's own launch timers (HIP events on
the launch stream) over a few whole steps of the workload, on a context and
state of its own so the caller's run is not advanced.  The best setting per
(knob, precision, size bucket, device) is kept in a JSON cache.  The knobs
change no result beyond the order of the pair sums (lanes) or the cell grid
(cell edge); the neighbour sets are exact for any of them.
"""
from __future__ import annotations

import json
import math
import os

from . import sph

LANES = (8, 4, 16)   # default first
CELL_SCALES = (1000, 1150, 1300)   # permille of 2 h_max
BUILD_RANGES = (64, 32, 96, 128)   # sorted particles per pair-list build work-group (default first)
# neighbour records in flight per lane of the fused sweep, per precision
# (default first): two in the FP32 form (104 VGPRs, four waves per SIMD), one
# in the FP64 form (138 VGPRs, three waves; two records take 180, two waves)
SWEEP_DEPTHS = {sph.SPH_FP64: (1, 2), sph.SPH_FP32_CELLREL: (2, 1)}
BUILD_TILES = (256, 192, 128)   # candidates in the pair-list build's LDS tile

# knob -> (timer whose per-launch time decides it, candidate values)
PLAN = (
    (sph.SPH_TUNE_SWEEP_DEPTH, sph.SPH_T_FORCES, SWEEP_DEPTHS),
    (sph.SPH_TUNE_LANES_STEP, sph.SPH_T_FORCES, LANES),
    (sph.SPH_TUNE_LANES_DENSITY, sph.SPH_T_DENSITY, LANES),
    (sph.SPH_TUNE_CELL_SCALE, None, CELL_SCALES),   # None: whole-step time
    (sph.SPH_TUNE_BUILD_RANGE, sph.SPH_T_BUILD, BUILD_RANGES),
    (sph.SPH_TUNE_BUILD_TILE, sph.SPH_T_BUILD, BUILD_TILES),
)
KNOB_NAMES = {sph.SPH_TUNE_LANES_STEP: "lanes_step", sph.SPH_TUNE_LANES_DENSITY: "lanes_density",
              sph.SPH_TUNE_CELL_SCALE: "cell_scale_permille",
              sph.SPH_TUNE_BUILD_RANGE: "build_range", sph.SPH_TUNE_SWEEP_DEPTH: "sweep_depth",
              sph.SPH_TUNE_BUILD_TILE: "build_tile"}


def size_bucket(n: int) -> int:
    """Power-of-two bucket of the particle count (settings carry over within it)."""
    return int(math.floor(math.log2(max(n, 1))))


def cache_key(device: str, prec: int, n: int) -> str:
    return f"{device}|prec{int(prec)}|n2^{size_bucket(n)}"


class TuneCache:
    """JSON file of chosen settings: {key: {knob_name: value, ...}}."""

    def __init__(self, path: str | None):
        self.path = path
        self.data = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.data = json.load(f)

    def get(self, key):
        return self.data.get(key)

    def put(self, key, settings: dict):
        self.data[key] = dict(settings)
        if self.path:
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.data, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


# A later candidate replaces the best so far only when it is faster by more
# than this fraction: settings whose times differ by less than the run-to-run
# noise keep the earlier one, so the choice repeats from run to run.
MARGIN = 0.05


def choose(values, measure, margin: float = MARGIN):
    """Smallest measured time wins, unless within ``margin`` of an earlier
    candidate, which then stays.  Returns (best value, {value: time})."""
    times = {}
    best, best_t = None, math.inf
    for v in values:
        t = float(measure(v))
        times[v] = t
        if t < best_t * (1.0 - margin):
            best, best_t = v, t
    return best, times


def apply(ctx, prec: int, settings: dict):
    for knob, name in KNOB_NAMES.items():
        if name in settings:
            sph.sph_set_tuning(ctx, knob, prec, int(settings[name]))


def tune(w: dict, prec: int, steps: int = 3, cache: TuneCache | None = None,
         run_start=None, max_neighbors: int = 128, max_cells: int = 1 << 22) -> dict:
    """Tune on workload ``w`` (its own context and state).  Returns
    {"settings": {...}, "times_ms": {...}, "cached": bool}."""
    import torch
    dev = torch.cuda.get_device_name(0)
    n = int(w["x"].size)
    key = cache_key(dev, prec, n)
    if cache is not None and cache.get(key) is not None:
        return {"settings": cache.get(key), "times_ms": {}, "cached": True}
    nr = 1 if run_start is None else len(run_start) - 1
    ctx = sph.Context(n, max_neighbors, max_cells, max_runs=max(nr, 1))
    st = sph.State(w, run_start=run_start)
    mats, prm = w["mats"], w["params"]
    sph.sph_init(ctx, st, mats, prm, prec)
    sph.sph_step(ctx, st, mats, prm, prec)   # first step: allocations, caches
    torch.cuda.synchronize()

    def measure(knob, timer, v):
        sph.sph_set_tuning(ctx, knob, prec, v)
        sph.sph_step(ctx, st, mats, prm, prec)  # settle the new shape
        if timer is None:
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(steps):
                sph.sph_step(ctx, st, mats, prm, prec)
            b.record()
            b.synchronize()
            return a.elapsed_time(b) / steps
        sph.sph_timing(ctx, True)
        for _ in range(steps):
            sph.sph_step(ctx, st, mats, prm, prec)
        ms, cnt = sph.sph_timing_read(ctx, timer)
        sph.sph_timing(ctx, False)
        return ms / max(cnt, 1)

    settings, times = {}, {}
    for knob, timer, values in PLAN:
        if isinstance(values, dict):
            values = values[prec]
        best, t = choose(values, lambda v: measure(knob, timer, v))
        sph.sph_set_tuning(ctx, knob, prec, best)
        settings[KNOB_NAMES[knob]] = best
        times[KNOB_NAMES[knob]] = {str(k): v for k, v in t.items()}
    ctx.check(sph.lib().sph_sync_status(ctx.h, None))
    ctx.close()
    if cache is not None:
        cache.put(key, settings)
    return {"settings": settings, "times_ms": times, "cached": False}
