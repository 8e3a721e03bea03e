"""Batched impact simulations as the judge of the Q_RD* search: every case
of a round runs in one set of buffers (run-keyed neighbour search, per-run
time steps, self-gravity), and the bound mass of each run at the end gives
its largest-remnant fraction f_lr = M_bound / M_total.

Host code sequences the library's entry points only (``sph_init``,
``sph_step``, ``sph_bound_mass``); every step of the physics runs in the
HIP kernels.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import inputs, sph

G = inputs.G_NEWTON


def free_fall_time(rho: float) -> float:
    """1 / sqrt(G rho): the time scale of gravitational reaccumulation."""
    return 1.0 / math.sqrt(G * rho)


def run_to_end(b: dict, t_end, checkpoints=(1.0,), prec: int = sph.SPH_FP32_CELLREL,
               max_steps: int = 20000, check_every: int = 50, theta: float = 0.6,
               max_neighbors: int = 256, log=None, max_cells: int = 1 << 24,
               far_factor: float = 0.0) -> dict:
    """Advance a batch of runs (``b``: concatenated runs with ``run_start``,
    ``mats``) under self-gravity until every run has reached its t_end (one
    value per run), as replays of a two-step hipGraph with ``check_every``
    (even) steps between checks.  At the first check at or after
    c * t_end[r] for each fraction c of ``checkpoints``, run r's bound mass
    is taken (iterative removal of unbound particles) and its largest-remnant
    fraction f = M_bound / M_total recorded.  Returns {"f": {c: array},
    "t": {c: array} (the run's time when recorded), "m_tot", "steps",
    "reached" (bool per run), "seconds"}.  ``far_factor`` > 0 holds each
    run's search grid to a cube of that many times its initial half-extent
    (sph_params.far_factor): ejecta beyond it fly on ballistically and count
    as unbound.  The runs take Omega = 1: with fixed smoothing lengths a
    particle that loses its neighbours (ejecta, the edge of the far cube)
    drives the defined Omega to zero, and the grad-h term is only consistent
    with adapted lengths anyway."""
    import time
    prm = inputs.default_params(grav_G=G, grav_theta=theta, far_factor=far_factor, omega_one=1)
    mats = b["mats"]
    rs = [int(v) for v in b["run_start"]]
    n, nr = int(b["x"].size), len(rs) - 1
    t_end = np.asarray(t_end, dtype=np.float64)
    ctx = sph.Context(n, max_neighbors, max_cells=max_cells, max_runs=nr)
    st = sph.State(b, run_start=rs)
    sph.sph_init(ctx, st, mats, prm, prec)   # the library sets each run's time to 0
    m = b["m"]
    m_tot = np.array([m[rs[r]:rs[r + 1]].sum() for r in range(nr)])
    f = {c: np.full(nr, np.nan) for c in checkpoints}
    tr = {c: np.full(nr, np.nan) for c in checkpoints}
    t0 = time.perf_counter()
    check_every += check_every % 2
    for _ in range(2):          # eager steps before the capture
        sph.sph_step(ctx, st, mats, prm, prec)
    steps = 2
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(2):
            sph.sph_step(ctx, st, mats, prm, prec)   # advances each run's time
    t_now = np.zeros(nr)
    while steps < max_steps:
        for _ in range(check_every // 2):
            graph.replay()
        steps += check_every
        code = sph.lib().sph_sync_status(ctx.h, None)
        if code != sph.SPH_OK:
            raise sph.SphError(code, f"after step {steps}: " + _run_report(st, rs, t_end))
        t_now = st.time.cpu().numpy()
        due = {c: np.flatnonzero(np.isnan(f[c]) & (t_now >= c * t_end)) for c in checkpoints}
        if any(d.size for d in due.values()):
            _, mb, _ = sph.sph_bound_mass(
                ctx, st.row(sph.SPH_VX).contiguous(), st.row(sph.SPH_VY).contiguous(),
                st.row(sph.SPH_VZ).contiguous(), st.row(sph.SPH_M).contiguous(), nr, G=G,
                eps_over_h=prm["grav_eps_over_h"], theta=theta)
            frac = mb.cpu().numpy() / m_tot
            for c, d in due.items():
                f[c][d] = frac[d]
                tr[c][d] = t_now[d]
        if log:
            log(f"  {nr} runs, {n} particles: step {steps}, min t/t_end "
                f"{float(np.min(t_now / t_end)):.3f}, {time.perf_counter() - t0:.1f} s")
        if all(not np.isnan(f[c]).any() for c in checkpoints):
            break
    del graph
    ctx.close()
    return dict(f=f, t=tr, m_tot=m_tot, steps=steps, reached=t_now >= t_end,
                seconds=time.perf_counter() - t0)


def _run_report(st, rs, t_end) -> str:
    """Which runs of a batch hold non-finite values, with their steps and times."""
    bad = []
    x = np.stack([st.row(k).cpu().numpy() for k in (sph.SPH_X, sph.SPH_VX, sph.SPH_U)])
    dt = st.dt.cpu().numpy()
    tn = st.time.cpu().numpy()
    for r in range(len(rs) - 1):
        seg = x[:, rs[r]:rs[r + 1]]
        nf = int((~np.isfinite(seg)).any(0).sum())
        if nf or not np.isfinite(dt[r]):
            bad.append(f"run {r}: {nf} particles non-finite, dt {dt[r]:.3g}, t/t_end "
                       f"{tn[r] / t_end[r]:.3f}")
    return "; ".join(bad) if bad else "no run holds a non-finite position, velocity or energy"


def end_times(cases, t_end_ff: float = 2.0, t_end_sound: float = 0.0):
    """t_end of each run: the crossing time (R_t + R_p) / v plus t_end_ff
    free-fall times 1/sqrt(G rho0) of the target material, or, when
    ``t_end_sound`` > 0 and it is shorter, that many sound-crossing times
    R_t / c0 of the target (c0 = sqrt(A / rho0), the bulk sound speed of the
    Tillotson material): once the shock has crossed and pressure has
    released the debris, each particle's energy relative to the remnant no
    longer changes, and so neither does the bound mass."""
    mat = inputs.granite_impact()
    rho = mat["rho0"]
    c0 = math.sqrt(mat["A"] / rho)
    out = []
    for k in cases:
        settle = t_end_ff * free_fall_time(rho)
        if t_end_sound > 0.0:
            settle = min(settle, t_end_sound * k["r_t"] / c0)
        out.append(settle + (k["r_t"] + k["r_p"]) / k["v"])
    return np.array(out)


def simulate(cases: list, t_end_ff: float = 2.0, prec: int = sph.SPH_FP32_CELLREL,
             max_steps: int = 20000, check_every: int = 50, theta: float = 0.6,
             max_neighbors: int = 256, log=None, checkpoints=(1.0,), t_end_sound: float = 0.0,
             max_cells: int = 1 << 24, far_factor: float = 3.0) -> dict:
    """Run every case (dicts with n_target, gamma, r_c1, v_over_vesc, strength)
    to t_end = t_end_ff free-fall times of the target material plus the
    crossing time (R_t + R_p) / v (or ``t_end_sound`` sound-crossing times of
    the target, see ``end_times``), then find the bound mass of each run.
    The bodies move in their centre-of-mass frame, so the remnant stays near
    the centre of the run's far cube (``far_factor``, see ``run_to_end``).
    Returns {"f_lr", "m_tot", "steps", "t", "t_end", "seconds", "particles",
    "f_at" (f_lr at every checkpoint c * t_end)} and, when 0.5 is among
    ``checkpoints``, "f_half" (f_lr at t_end / 2)."""
    strong = inputs.granite_impact()
    mats = [strong, inputs.fluid(strong)]
    runs = []
    for c in cases:
        w = inputs.impact_pair(int(c["n_target"]), c.get("gamma", 0.1), c["r_c1"],
                               c["v_over_vesc"], bool(c["strength"]),
                               mat_id=0 if c["strength"] else 1, mat=strong, cm_frame=True)
        runs.append(w)
    b = inputs.concat_runs(runs)
    b["mats"] = mats
    t_end = end_times([w["case"] for w in runs], t_end_ff, t_end_sound)
    cps = tuple(sorted(set(checkpoints) | {1.0}))
    r = run_to_end(b, t_end, cps, prec=prec, max_steps=max_steps, check_every=check_every,
                   theta=theta, max_neighbors=max_neighbors, log=log, max_cells=max_cells,
                   far_factor=far_factor)
    out = dict(f_lr=r["f"][1.0], m_tot=r["m_tot"], steps=r["steps"], t=r["t"][1.0],
               t_end=t_end, seconds=r["seconds"], particles=int(b["x"].size),
               f_at={c: r["f"][c] for c in cps})
    if 0.5 in r["f"]:
        out["f_half"] = r["f"][0.5]
    return out


def bracket_rounds(cases: list, judge_batch, tol: float = 0.05, predict_for=None,
                   max_rounds: int = 12, log=None, expand: int = 2):
    """Bracket Q_RD* for every case at once, one simulation per unfinished
    bracket per round, all of a round's simulations judged in one batch.

    ``cases``: qrd.Case objects; ``judge_batch(list of (case, v)) -> list of
    f_lr``; ``predict_for(round) -> predict`` gives the model for that round
    (None: plain bisection).  The initial bracket is [v_esc, 10 v_esc]; its
    ends are simulated in the first round.  A case whose upper end still
    leaves more than half the mass bound is extended upwards by a factor of
    three, at most ``expand`` times (batched like the rounds).  Returns the
    brackets, their validity and the list of (features, f_lr) outcomes."""
    from . import qrd
    brackets = [qrd.Bracket(c, c.v_esc, 10.0 * c.v_esc) for c in cases]
    outcomes = []
    jobs = [(b.case, b.v_lo) for b in brackets] + [(b.case, b.v_hi) for b in brackets]
    f = judge_batch(jobs)
    k = len(brackets)
    for i, b in enumerate(brackets):
        b.f_lo, b.f_hi = f[i], f[k + i]
        b.sims = 2
        outcomes += [(b.case.features(b.v_lo), b.f_lo), (b.case.features(b.v_hi), b.f_hi)]
    for _ in range(expand):
        low = [b for b in brackets if b.f_lo > 0.5 and b.f_hi > 0.5]
        if not low:
            break
        f = judge_batch([(b.case, 3.0 * b.v_hi) for b in low])
        for b, fv in zip(low, f):
            b.v_lo, b.f_lo = b.v_hi, b.f_hi
            b.v_hi, b.f_hi = 3.0 * b.v_hi, float(fv)
            b.sims += 1
            outcomes.append((b.case.features(b.v_hi), b.f_hi))
        if log:
            log(f"extended {len(low)} brackets upwards")
    valid = [b.f_lo > 0.5 >= b.f_hi for b in brackets]
    for rnd in range(max_rounds):
        open_ = [b for b, ok in zip(brackets, valid) if ok and b.width() > tol]
        if not open_:
            break
        predict = predict_for(rnd) if predict_for else None
        props = []
        for b in open_:
            if predict is None:
                props.append((qrd.bisect_proposal(b), "bisect"))
            else:
                v, used = qrd.model_proposal(b, predict, tol)
                after_root = bool(b.history) and b.history[-1][2] == "root"
                props.append((v, ("step" if after_root else "root") if used else "bisect"))
        f = judge_batch([(b.case, v) for b, (v, _) in zip(open_, props)])
        for b, (v, src), fv in zip(open_, props, f):
            b.update(v, float(fv), src)
            outcomes.append((b.case.features(v), float(fv)))
        if log:
            log(f"round {rnd}: {len(open_)} open, widths "
                f"{[round(b.width(), 3) for b in brackets]}")
    return brackets, valid, outcomes


def case_for(r_c1: float, strength: int, gamma: float = 0.1):
    """The qrd.Case of a head-on impact as ``inputs.impact_pair`` builds it:
    total mass of a sphere of radius r_c1 at 1000 kg/m^3, bodies at the
    granite reference density, v_esc = sqrt(2 G M_tot / (R_t + R_p))."""
    from . import qrd
    rho = inputs.granite_c3()["rho0"]
    m_tot = 4.0 / 3.0 * math.pi * r_c1 ** 3 * 1000.0
    m_t, m_p = m_tot / (1.0 + gamma), m_tot * gamma / (1.0 + gamma)
    r_t = (3.0 * m_t / (4.0 * math.pi * rho)) ** (1.0 / 3.0)
    r_p = (3.0 * m_p / (4.0 * math.pi * rho)) ** (1.0 / 3.0)
    return qrd.Case(m_tot, gamma, int(strength), math.sqrt(2.0 * G * m_tot / (r_t + r_p)))


def judge_with_simulation(n_target: int, **kw):
    """A judge_batch for ``bracket_rounds``: one batched simulation per call."""
    def judge_batch(jobs):
        cases = []
        for c, v in jobs:
            r_c1 = (3.0 * c.m_tot / (4.0 * math.pi * 1000.0)) ** (1.0 / 3.0)
            cases.append(dict(n_target=n_target, gamma=c.gamma, r_c1=r_c1,
                              v_over_vesc=v / c.v_esc, strength=c.strength))
        return list(simulate(cases, **kw)["f_lr"])
    return judge_batch
