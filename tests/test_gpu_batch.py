"""Batched runs and graph replay of the whole step.

Several independent runs share one set of buffers (run-keyed sort, per-run
cell grids, per-run CFL step): each run must evolve exactly as it does alone.
The runs overlap in space, so a pair that crossed runs would show at once.
A two-step hipGraph of sph_step must reproduce eager steps on every replay."""
import numpy as np
import pytest

from paper_2603_19764_amd import inputs
from tests.gpu_harness import norm_err, say

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1
FIELDS = ("x", "y", "z", "vx", "vy", "vz", "u", "S", "a", "dudt", "dS", "eps2", "rho", "G")


def _runs():
    r0 = inputs.c1_block(6, variant="s")
    r1 = inputs.c1_block(8, variant="y", seed_pos=7)
    r1["u"] = r1["u"] * 50.0            # hotter: another sound speed, another step
    r2 = inputs.c1_block(7, seed_pos=11, seed_vel=12)
    for k in ("vx", "vy", "vz"):
        r2[k] = r2[k] * 100.0           # faster shear: viscosity sets the step
    return [r0, r1, r2]


def _evolve(w, prec, steps, run_start=None):
    import torch
    from paper_2603_19764_amd import sph
    n = int(w["x"].size)
    nr = 1 if run_start is None else len(run_start) - 1
    ctx = sph.Context(n, 128, max_runs=max(nr, 1))
    st = sph.State(w, run_start=run_start)
    sph.sph_init(ctx, st, w["mats"], w["params"], prec)
    for _ in range(steps):
        sph.sph_step(ctx, st, w["mats"], w["params"], prec)
    torch.cuda.synchronize()
    ctx.check(sph.lib().sph_sync_status(ctx.h, None))
    out = st.to_host()
    out["time"] = st.time.cpu().numpy().copy()
    dt = st.dt.cpu().numpy().copy()
    ctx.close()
    return out, dt


def _slice(g, a, b):
    return {k: (v[..., a:b] if isinstance(v, np.ndarray) else v) for k, v in g.items()}


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_batched_runs_equal_single_runs(prec):
    runs = _runs()
    w = inputs.concat_runs(runs)
    rs = [int(v) for v in w["run_start"]]
    steps = 4
    gb, dtb = _evolve(w, prec, steps, rs)
    assert dtb.shape == (3,)
    worst = 0.0
    for r, run in enumerate(runs):
        gs, dts = _evolve(run, prec, steps)
        part = _slice(gb, rs[r], rs[r + 1])
        e = {k: norm_err(part[k], gs[k]) for k in FIELDS}
        e["dt"] = abs(dtb[r] - dts[0]) / dts[0]
        # each run's simulated time kept by the library: the sum of its steps
        e["time"] = abs(gb["time"][r] - gs["time"][0]) / gs["time"][0]
        say(f"run {r} prec {prec}", {k: f"{v:.1e}" for k, v in e.items()})
        worst = max(worst, max(e.values()))
    assert worst <= 1e-12
    # the runs really take different steps
    assert len(set(np.round(dtb / dtb.max(), 9))) == 3


def test_graph_replay_matches_eager():
    """Two steps captured once, replayed three times with eager work and
    synchronisation between replays; every replay equals the eager steps."""
    import torch
    from paper_2603_19764_amd import sph
    w = inputs.concat_runs(_runs())
    rs = [int(v) for v in w["run_start"]]
    n = int(w["x"].size)
    mats, prm = w["mats"], w["params"]

    ctx_e = sph.Context(n, 128, max_runs=3)
    st_e = sph.State(w, run_start=rs)
    sph.sph_init(ctx_e, st_e, mats, prm, FP64)
    snaps = []
    for _ in range(3):
        sph.sph_step(ctx_e, st_e, mats, prm, FP64)
        sph.sph_step(ctx_e, st_e, mats, prm, FP64)
        torch.cuda.synchronize()
        snaps.append((st_e.to_host(), st_e.dt.cpu().numpy().copy()))

    ctx = sph.Context(n, 128, max_runs=3)
    st = sph.State(w, run_start=rs)
    sph.sph_init(ctx, st, mats, prm, FP64)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    with torch.cuda.graph(g, stream=side):
        sph.sph_step(ctx, st, mats, prm, FP64)
        sph.sph_step(ctx, st, mats, prm, FP64)
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        got = st.to_host()
        dt = st.dt.cpu().numpy()
        ref, ref_dt = snaps[rep]
        e = max(norm_err(got[k], ref[k]) for k in FIELDS)
        say(f"replay {rep}: max field err {e:.1e}")
        assert e == 0.0
        assert np.array_equal(dt, ref_dt)
        # eager work between replays
        _ = torch.ones(1000, device="cuda").sum().item()
    ctx.check(sph.lib().sph_sync_status(ctx.h, None))
    del g
    ctx.close()
    ctx_e.close()
