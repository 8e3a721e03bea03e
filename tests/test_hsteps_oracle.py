"""Pins of the oracle's individual time steps (reading T1: steps dt0 2^-r,
substeps to the next end of any particle's step, forces only for the
particles whose step ends) and of the acceleration criterion (reading T2).

What pins them: the rung rule on hand-worked cases; a set whose particles
all sit on one rung reproduces the shared-step integrator bit for bit; two
bodies that do not interact, one on rung 2 and one on rung 0, evolve exactly
as each does alone under the shared-step integrator with its own step; the
simulation clock lands on multiples of the base step; the step with the
acceleration criterion is the minimum of the two criteria."""

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2603_19764_amd import inputs


def test_rung_rule():
    # 5 rungs of a base step 1.0: steps of 16, 8, 4, 2, 1 ticks of 1/16
    tick = 1.0 / 16
    # the longest step not above the particle's own step
    assert orc.rung_step(5, tick, 3.0, 0, 16) == (16, 0)
    assert orc.rung_step(5, tick, 0.3, 0, 16) == (4, 0)
    assert orc.rung_step(5, tick, 0.125, 0, 16) == (2, 0)
    # below the shortest rung: the shortest, counted
    assert orc.rung_step(3, 0.25, 0.1, 0, 4) == (1, 1)
    # lengthening only at a multiple of the new step
    assert orc.rung_step(5, tick, 2.0, 12, 4) == (4, 0)
    assert orc.rung_step(5, tick, 2.0, 8, 4) == (8, 0)
    assert orc.rung_step(5, tick, 2.0, 48, 4) == (16, 0)
    # shortening is always allowed
    assert orc.rung_step(5, tick, 0.2, 12, 4) == (2, 0)


def _block(n_side, spacing, offset=0.0, c_min=1.0e4):
    """A resting lattice block at the reference density whose sound speed is
    the floor c_min everywhere (so all its particles share one CFL step)."""
    x, y, z = inputs.lattice(n_side, n_side, n_side, spacing)
    n = x.size
    w = inputs._empty(n)
    w.update(x=x + offset, y=y.copy(), z=z.copy(), m=np.full(n, 2700.0 * spacing ** 3),
             h=np.full(n, 1.3 * spacing))
    w["u"][:] = 1.0e4
    mat = dict(inputs.basalt_c1(), c_min=c_min)
    return w, [mat]


def _st(w):
    return {k: w[k] for k in ("x", "y", "z", "m", "h", "mat", "vx", "vy", "vz", "u", "S", "fixed")}


def _join(a, b):
    out = {}
    for k in ("x", "y", "z", "m", "h", "vx", "vy", "vz", "u", "mat", "fixed"):
        out[k] = np.concatenate([a[k], b[k]])
    out["S"] = np.concatenate([a["S"], b["S"]], axis=1)
    return out


def _cfl_step(w, mats, prm):
    it = orc.Integrator(_st(w), mats, prm)
    return float(np.min(it["dt_i"]))


def test_one_rung_reproduces_the_shared_step():
    w, mats = _block(5, 1.0)
    w["vx"][:] = 0.3 * np.sin(w["y"])
    prm = inputs.default_params()
    dt0 = 0.9 * _cfl_step(w, mats, prm)
    shared = orc.Integrator(_st(w), mats, prm, dt_fixed=dt0)
    hier = orc.Integrator(_st(w), mats, dict(prm, rungs=6), dt_fixed=dt0)
    for _ in range(3):
        shared.step()
        hier.step()
    for k in ("x", "vx", "vy", "u", "S", "ax", "dS", "eps2"):
        assert np.array_equal(shared[k], hier[k]), k
    assert hier.time == 3 * dt0 and hier.n_clamped == 0


@pytest.mark.parametrize("base_steps", [1, 2])
def test_bodies_on_different_rungs_evolve_as_alone(base_steps):
    # body A: a quarter-scale copy of body B (same density and sound speed),
    # so its CFL step is a quarter of B's; far apart, they do not interact
    wb, mats = _block(5, 1.0)
    wa, _ = _block(5, 0.25, offset=-50.0)
    wa["vy"][:] = 0.05 * np.cos(4.0 * wa["x"])
    wb["vy"][:] = 0.05 * np.cos(wb["x"])
    prm = inputs.default_params()
    dt0 = 0.9 * _cfl_step(wb, mats, prm)
    assert 0.25 * dt0 <= _cfl_step(wa, mats, prm) < 0.5 * dt0
    both = _join(wa, wb)
    na = wa["x"].size
    hier = orc.Integrator(both, mats, dict(prm, rungs=4), dt_fixed=dt0)
    steps_a = orc.Integrator(_st(wa), mats, prm, dt_fixed=0.25 * dt0)
    steps_b = orc.Integrator(_st(wb), mats, prm, dt_fixed=dt0)
    assert np.all(hier["dtp"][:na] == 2) and np.all(hier["dtp"][na:] == 8)   # ticks of dt0/8
    for _ in range(4 * base_steps):
        hier.step()
    steps_a.step(4 * base_steps)
    steps_b.step(base_steps)
    assert hier.time == base_steps * dt0
    for k in ("x", "y", "vx", "vy", "u", "S", "ax", "ay", "dudt", "dS", "eps2"):
        ha, hb = hier[k][..., :na], hier[k][..., na:]
        sa, sb = steps_a[k], steps_b[k]
        scale_a = max(np.max(np.abs(sa)), 1e-300)
        scale_b = max(np.max(np.abs(sb)), 1e-300)
        if k in ("x", "y"):   # drift in four parts against one
            scale_a = scale_b = 1.0
        assert np.max(np.abs(ha - sa)) <= 1e-12 * scale_a, k
        assert np.max(np.abs(hb - sb)) <= 1e-12 * scale_b, k


def test_substeps_follow_the_shortest_step():
    wb, mats = _block(4, 1.0)
    wa, _ = _block(4, 0.25, offset=-40.0)
    prm = inputs.default_params()
    dt0 = 0.9 * _cfl_step(wb, mats, prm)
    hier = orc.Integrator(_join(wa, wb), mats, dict(prm, rungs=4), dt_fixed=dt0)
    na = wa["x"].size
    times = []
    for _ in range(8):
        assert hier.dt == 0.25 * dt0
        hier.step()
        times.append(hier.time)
        # body A ends a step at every substep, body B at multiples of dt0
        assert np.all(hier["el"][:na] == 0)
        assert np.all(hier["el"][na:] == hier.ticks % 8)
    assert [hier.tick * 2 * k for k in range(1, 9)] == times


def test_acceleration_criterion():
    w, mats = _block(5, 1.0, c_min=1.0)
    w["u"][:] = 0.0
    prm = inputs.default_params(g=(0.0, -9.81, 0.0))
    plain = orc.Integrator(_st(w), mats, prm)
    eta_a = 0.05
    acc = orc.Integrator(_st(w), mats, dict(prm, eta_a=eta_a))
    a = np.sqrt(plain["ax"] ** 2 + plain["ay"] ** 2 + plain["az"] ** 2)
    crit = eta_a * np.sqrt(w["h"] / a)
    want = min(float(np.min(plain["dt_i"])), float(np.min(crit)))
    assert acc.dt == pytest.approx(want, rel=1e-15)
    assert float(np.min(crit)) < float(np.min(plain["dt_i"]))   # the criterion decides here


def _periodic_flow():
    """A periodic lattice box (10^3, spacing 1 m) of strengthless basalt with
    smoothing lengths varying along x between 1.0 and 2.2 m: a smooth
    pressure-driven flow whose CFL steps span a factor of two and more, so
    the particles sit on several rungs and act on each other."""
    Lb = 10
    x, y, z = inputs.lattice(Lb, Lb, Lb, 1.0)
    n = x.size
    w = inputs._empty(n)
    w.update(x=x, y=y, z=z, m=np.full(n, 2700.0),
             h=1.0 + 0.6 * (1.0 + np.sin(2.0 * np.pi * x / Lb)))
    w["u"][:] = 1.0e4
    w["vy"][:] = 0.5 * np.sin(2.0 * np.pi * x / Lb)
    return w, [inputs.fluid(inputs.basalt_c1())], inputs.default_params(box=(Lb, Lb, Lb))


def _synced(it, hier):
    # the kicked values less the half kick of the step now starting
    own = it["dtp"] * it.tick if hier else np.full(it.n, it.dt)
    return it["vx"] - 0.5 * own * it["ax"], it["u"] - 0.5 * own * it["dudt"]


def test_mixed_rungs_converge_at_second_order():
    """Halving every step (the CFL factor and the base step) cuts the error
    against a fine shared-step solution by four in velocity, energy and
    position: particles whose step has not ended enter their neighbours'
    derivatives predicted to the current time, to first order in the time
    elapsed in their step, so the scheme stays second order (predicting them
    half a step instead makes it first order)."""
    w, mats, prm = _periodic_flow()
    st = _st(w)
    D = float(np.max(orc.Integrator(st, mats, prm)["dt_i"]))
    T = 2 * D
    ref = orc.Integrator(st, mats, prm, dt_fixed=T / 512)
    ref.step(512)
    rv, ru = _synced(ref, False)
    errs = []
    for k in (1, 2, 4):
        it = orc.Integrator(st, mats, dict(prm, rungs=8, eta_C=prm["eta_C"] / k), dt_fixed=D / k)
        assert np.unique(it["dtp"]).size >= 2 and it.n_clamped == 0
        while it.time < T * (1 - 1e-12):
            it.step()
        assert it.time == pytest.approx(T, rel=1e-13)
        v, u = _synced(it, True)
        errs.append((np.max(np.abs(v - rv)), np.max(np.abs(u - ru)),
                     np.max(np.abs(it["x"] - ref["x"]))))
    for a, b in zip(errs, errs[1:]):
        for ea, eb in zip(a, b):
            assert ea / eb > 3.3, errs
