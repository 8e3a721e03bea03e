"""The Q_RD* campaign at production size: rounds of batched impact
simulations judge the impact speeds that the learned proposal picks, and
plain log-v bisection runs beside it on held-out cases.

Cases are (total mass, strength) pairs of head-on impacts with mass ratio
gamma = 0.1 (sec. 3, Appendix A: the threshold Q_RD* at which the largest
remnant keeps half the total mass, bracketed in log v at fixed gamma and
interpolated in Q_R).  Every case has its own target particle count, drawn
log-uniform, and both methods simulate a case at the same resolution.

Two searches exist per case:

- ``bisect``: simulate v_esc and 10 v_esc, extend the upper end by 3x at
  most twice while it still leaves more than half the mass bound, then halve
  the bracket in log v until its relative Q_R width is at most ``tol``;
- ``net``: simulate the speed where the trained network's f_lr crosses 1/2
  on [v_esc, 10 v_esc]; step away from it by a window w in log v (doubling w
  after each step that does not cross the threshold) until the outcomes
  bracket it, then halve the bracket in log v.  w is the network's typical
  error in log v, measured on the training cases' own brackets.  When the
  network has no crossing on the interval the search starts as bisection.

Training rounds run the network search on training cases (the first round
at random speeds, since no network exists yet) and retrain the network from
scratch on every outcome after each round; the held-out rounds use the
network trained on the training outcomes only.  All simulations of a round
run in one batch (``scan.simulate``).  The state is a JSON-serialisable dict
so a campaign can run over several processes.

Host code only: the simulations and the network's training and inference
run in the library's kernels.
"""
from __future__ import annotations

import json
import math
import time

import numpy as np

from . import qrd, scan


# ------------------------------------------------------------------ cases
def draw_cases(n: int, seed: int, n_min: float = 3.0e4, n_max: float = 5.0e5,
               r_lo: float = 4.64e5, r_hi: float = 4.64e6, gamma: float = 0.1) -> list:
    """``n`` cases: target particle count and R_C1 log-uniform, strength on
    for every other case (half of the cases each way)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(n):
        nt = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        rc1 = math.exp(rng.uniform(math.log(r_lo), math.log(r_hi)))
        out.append(dict(n_target=nt, r_c1=rc1, strength=k % 2, gamma=gamma))
    return out


def case_of(spec: dict) -> qrd.Case:
    return scan.case_for(spec["r_c1"], spec["strength"], spec["gamma"])


def v_at_q(case: qrd.Case, q: float) -> float:
    """Impact speed of specific energy q (inverse of the Q_R equation)."""
    return math.sqrt(q / case.q(1.0))


# --------------------------------------------------------------- searches
def new_search(spec: dict, method: str) -> dict:
    return dict(spec=spec, method=method, pts=[], status="open", start=None)


def _sides(s: dict):
    """(v_lo, f_lo, v_hi, f_hi): the smallest simulated speed with f <= 1/2
    and the largest below it with f > 1/2, so that f crosses 1/2 between them
    (None where a side is unknown)."""
    below = [(v, f) for v, f, _ in s["pts"] if f <= 0.5]
    hi = min(below) if below else (None, None)
    above = [(v, f) for v, f, _ in s["pts"] if f > 0.5 and (hi[0] is None or v < hi[0])]
    lo = max(above) if above else (None, None)
    return lo[0], lo[1], hi[0], hi[1]


def width(s: dict) -> float:
    """Relative Q_R width of the bracket (inf while it is open on a side)."""
    v_lo, _, v_hi, _ = _sides(s)
    if v_lo is None or v_hi is None or v_hi <= v_lo:
        return math.inf
    c = case_of(s["spec"])
    return (c.q(v_hi) - c.q(v_lo)) / c.q(v_lo)


def q_rd(s: dict) -> float:
    """Threshold by linear interpolation in Q_R between the bracket ends."""
    v_lo, f_lo, v_hi, f_hi = _sides(s)
    c = case_of(s["spec"])
    b = qrd.Bracket(c, v_lo, v_hi, f_lo, f_hi)
    return b.q_rd()


def _bisect_next(s: dict, tol: float, max_extend: int = 2) -> list:
    c = case_of(s["spec"])
    if not s["pts"]:
        return [(c.v_esc, "end"), (10.0 * c.v_esc, "end")]
    v_lo, _, v_hi, _ = _sides(s)
    if v_hi is None:                    # even the upper end leaves > half bound
        ext = sum(1 for p in s["pts"] if p[2] == "extend")
        if ext >= max_extend:
            s["status"] = "invalid"
            return []
        return [(3.0 * max(p[0] for p in s["pts"]), "extend")]
    if v_lo is None:                    # disrupted at the escape speed
        s["status"] = "invalid"
        return []
    if width(s) <= tol:
        s["status"] = "done"
        return []
    return [(math.sqrt(v_lo * v_hi), "bisect")]


def model_threshold(case: qrd.Case, predict, v_lo: float, v_hi: float, n_grid: int = 129):
    """Speed where the model's f_lr first falls to 1/2 on [v_lo, v_hi] (log
    grid, linear interpolation between grid points), or None."""
    lv = np.linspace(math.log(v_lo), math.log(v_hi), n_grid)
    X = np.stack([case.features(v) for v in np.exp(lv)])
    f = np.asarray(predict(X), dtype=np.float64)
    if not (f[0] > 0.5 >= f[-1]):
        return None
    k = int(np.argmax(f <= 0.5))
    t = (f[k - 1] - 0.5) / (f[k - 1] - f[k])
    return math.exp(lv[k - 1] + t * (lv[k] - lv[k - 1]))


def _net_next(s: dict, predict, w: float, tol: float, v_max_factor: float = 30.0) -> list:
    c = case_of(s["spec"])
    if s["start"] == "bisect":
        return _bisect_next(s, tol)
    if not s["pts"]:
        v0 = None if predict is None else model_threshold(c, predict, c.v_esc, 10.0 * c.v_esc)
        if v0 is None:          # no crossing: start as bisection
            s["start"] = "bisect"
            return _bisect_next(s, tol)
        s["start"] = "net"
        return [(v0, "root")]
    v_lo, _, v_hi, _ = _sides(s)
    if (v_lo is None or v_hi is None) and predict is not None and not any(
            p[2] == "root" for p in s["pts"]):
        # started elsewhere (a random speed before any network existed): try
        # the network's threshold once, if it lies on the open side
        v0 = model_threshold(c, predict, c.v_esc, 10.0 * c.v_esc)
        if v0 is not None and ((v_hi is None and v0 > v_lo * (1.0 + 1e-9)) or
                               (v_lo is None and v0 < v_hi * (1.0 - 1e-9))):
            return [(v0, "root")]
    steps = sum(1 for p in s["pts"] if p[2] == "window")
    if v_hi is None:            # every outcome above 1/2: step up
        v = max(p[0] for p in s["pts"]) * math.exp(w * 2.0 ** steps)
        if v > v_max_factor * c.v_esc:
            s["status"] = "invalid"
            return []
        return [(v, "window")]
    if v_lo is None:            # every outcome at or below 1/2: step down
        vmin = min(p[0] for p in s["pts"])
        if vmin <= c.v_esc * (1.0 + 1e-12):
            s["status"] = "invalid"
            return []
        return [(max(vmin * math.exp(-w * 2.0 ** steps), c.v_esc), "window")]
    if width(s) <= tol:
        s["status"] = "done"
        return []
    return [(math.sqrt(v_lo * v_hi), "bisect")]


def next_speeds(s: dict, predict=None, w: float = 0.2, tol: float = 0.05,
                rng: np.random.Generator | None = None) -> list:
    """The impact speeds this search simulates next (empty when it is done
    or invalid).  A network search with no network yet starts at a random
    speed in [v_esc, 10 v_esc] (log-uniform) and continues by windows."""
    if s["status"] != "open":
        return []
    if s["method"] == "bisect":
        return _bisect_next(s, tol)
    if predict is None and not s["pts"] and rng is not None:
        c = case_of(s["spec"])
        s["start"] = "net"
        return [(c.v_esc * 10.0 ** rng.uniform(0.0, 1.0), "random")]
    return _net_next(s, predict, w, tol)


def sims(s: dict) -> int:
    return len(s["pts"])


# ----------------------------------------------------------- the network
def outcomes(searches: list) -> tuple:
    X, Y = [], []
    for s in searches:
        c = case_of(s["spec"])
        for v, f, _ in s["pts"]:
            X.append(c.features(v))
            Y.append(f)
    return np.array(X), np.array(Y)


def train(searches: list, seed: int = 1, epochs: int = 4000, lr: float = 3e-3):
    """A network trained from scratch on every outcome of ``searches``."""
    from .proposal import MlpProposer
    X, Y = outcomes(searches)
    net = MlpProposer(seed=seed, lr=lr)
    loss = net.fit(X, Y, epochs=epochs)
    return net, loss, int(Y.size)


def window(net, searches: list, tol: float, w_min: float = 0.03, w_max: float = 0.5,
           w_default: float = 0.2) -> tuple:
    """Window in log v: 1.5x the root-mean-square log-v distance between the
    network's threshold and the bracketed thresholds of the closed training
    searches (``w_default`` before any is closed)."""
    errs = []
    for s in searches:
        if s["status"] != "done":
            continue
        c = case_of(s["spec"])
        v_star = v_at_q(c, q_rd(s))
        v_net = model_threshold(c, net.predict, c.v_esc, 10.0 * c.v_esc)
        if v_net is not None:
            errs.append(math.log(v_net / v_star))
    if not errs:
        return w_default, None
    rms = float(np.sqrt(np.mean(np.square(errs))))
    return float(min(max(1.5 * rms, w_min), w_max)), rms


# --------------------------------------------------------------- the judge
def judge(jobs: list, log=None, **kw) -> tuple:
    """Simulate every (spec, v) of ``jobs`` in one batch: returns the
    largest-remnant fractions at t_end and at t_end / 2, and the run's record
    (steps, seconds, particles)."""
    cases = []
    for spec, v in jobs:
        c = case_of(spec)
        cases.append(dict(n_target=spec["n_target"], gamma=spec["gamma"], r_c1=spec["r_c1"],
                          v_over_vesc=v / c.v_esc, strength=spec["strength"]))
    r = scan.simulate(cases, checkpoints=(0.5, 1.0), log=log, **kw)
    return r["f_lr"], r["f_half"], dict(steps=r["steps"], seconds=r["seconds"],
                                         particles=r["particles"], runs=len(jobs))


# ------------------------------------------------------------- campaign
def new_campaign(n_train: int = 32, n_held: int = 16, seed: int = 6, tol: float = 0.05,
                 **draw) -> dict:
    train_specs = draw_cases(n_train, seed, **draw)
    held_specs = draw_cases(n_held, seed + 1000, **draw)
    return dict(tol=tol, seed=seed, draw=draw,
                train=[new_search(sp, "net") for sp in train_specs],
                held=[new_search(sp, m) for sp in held_specs for m in ("bisect", "net")],
                rounds=[], phase="train", w=None, w_rms=None)


def _round(state: dict, searches: list, predict, w: float, rng, log, judge_fn,
           judge_kw) -> bool:
    """Propose, simulate and record one round; False when nothing is open."""
    tol = state["tol"]
    props = []
    for k, s in enumerate(searches):
        for v, src in next_speeds(s, predict, w, tol, rng):
            props.append((k, v, src))
    if not props:
        return False
    # one simulation per distinct (case, speed)
    keyed = {}
    for k, v, src in props:
        key = (json.dumps(searches[k]["spec"], sort_keys=True), float(v))
        keyed.setdefault(key, []).append((k, src))
    jobs = [(searches[lst[0][0]]["spec"], key[1]) for key, lst in keyed.items()]
    f, fh, rec = judge_fn(jobs, log=log, **judge_kw)
    for (key, lst), fv, fhv in zip(keyed.items(), f, fh):
        for k, src in lst:
            searches[k]["pts"].append([key[1], float(fv), src])
    dfl = np.abs(np.asarray(f) - np.asarray(fh))
    rec.update(phase=state["phase"], w=w, f_change=float(np.nanmax(dfl)),
               f_change_median=float(np.nanmedian(dfl)),
               f_change_p90=float(np.nanpercentile(dfl, 90)))
    state["rounds"].append(rec)
    if log:
        log(f"round {len(state['rounds'])} ({state['phase']}): {rec}")
    return True


def run(state: dict, max_rounds: int = 100, budget_s: float = 1e30, log=None,
        train_rounds: int = 8, judge_fn=judge, trainer=train, save=None, **judge_kw) -> dict:
    """Advance the campaign by at most ``max_rounds`` rounds or until
    ``budget_s`` seconds have passed (checked between rounds); ``save(state)``
    is called after every round.  ``judge_fn`` and ``trainer`` default to the
    batched simulation and the network trained by the library's kernels."""
    t0 = time.perf_counter()
    rng = np.random.Generator(np.random.PCG64(state["seed"] + 7 + len(state["rounds"])))
    done_rounds = 0
    while done_rounds < max_rounds and time.perf_counter() - t0 < budget_s:
        if state["phase"] == "train":
            n_tr = sum(1 for r in state["rounds"] if r["phase"] == "train")
            predict, w = None, 0.2
            if any(s["pts"] for s in state["train"]):
                net, _, _ = trainer(state["train"])
                predict = net.predict
                w, _ = window(net, state["train"], state["tol"])
            if n_tr >= train_rounds or not _round(state, state["train"], predict, w, rng, log,
                                                  judge_fn, judge_kw):
                state["phase"] = "held"
                net, loss, m = trainer(state["train"])
                state["w"], state["w_rms"] = window(net, state["train"], state["tol"])
                state["train_loss"], state["train_outcomes"] = loss, m
                continue
        elif state["phase"] == "held":
            net, _, _ = trainer(state["train"])
            if not _round(state, state["held"], net.predict, state["w"], rng, log, judge_fn,
                          judge_kw):
                state["phase"] = "done"
                break
        else:
            break
        done_rounds += 1
        if save:
            save(state)
    if save:
        save(state)
    return state


def summary(state: dict) -> dict:
    """Simulations per held-out case for each method, their thresholds, and
    the campaign's record."""
    by = {}
    for s in state["held"]:
        key = json.dumps(s["spec"], sort_keys=True)
        by.setdefault(key, {})[s["method"]] = s
    rows = []
    for key, d in by.items():
        b, n = d["bisect"], d["net"]
        c = case_of(b["spec"])
        row = dict(m_tot=c.m_tot, strength=b["spec"]["strength"],
                   n_target=b["spec"]["n_target"], sims_bisect=sims(b), sims_net=sims(n),
                   status_bisect=b["status"], status_net=n["status"], net_start=n["start"])
        for name, s in (("bisect", b), ("net", n)):
            row[f"q_rd_{name}"] = q_rd(s) if s["status"] == "done" else None
        rows.append(row)
    ok = [r for r in rows if r["status_bisect"] == "done" and r["status_net"] == "done"]
    tr = [s for s in state["train"]]
    return dict(cases=rows, compared=len(ok),
                sims_bisect=sum(r["sims_bisect"] for r in ok),
                sims_net=sum(r["sims_net"] for r in ok),
                train_cases=len(tr), train_done=sum(1 for s in tr if s["status"] == "done"),
                train_sims=sum(sims(s) for s in tr), window=state.get("w"),
                window_rms=state.get("w_rms"), rounds=len(state["rounds"]),
                simulations=sum(r["runs"] for r in state["rounds"]),
                gpu_seconds=sum(r["seconds"] for r in state["rounds"]),
                max_f_change=max((r["f_change"] for r in state["rounds"]), default=None))


def settling(state: dict, factors=(0.5, 1.0, 2.0, 4.0), simulate=None, log=None,
             max_cases: int | None = None, **sim_kw) -> dict:
    """Run the ends of every closed held-out bisection bracket on, past t_end:
    f_lr at ``factors`` x t_end for the lower end (f > 1/2 at t_end) and the
    upper end (f <= 1/2), all in one batch.  Reports per case whether the
    ends still straddle 1/2 at each time and the threshold interpolated
    between them (None once they do not), so that the drift of the bound
    mass after t_end and its effect on Q_RD* are measured, not assumed.
    ``max_cases`` limits the check to the first that many closed brackets."""
    simulate = simulate or scan.simulate
    specs, jobs = [], []
    for s in state["held"]:
        if s["method"] != "bisect" or s["status"] != "done":
            continue
        if max_cases is not None and len(specs) >= max_cases:
            break
        v_lo, _, v_hi, _ = _sides(s)
        specs.append((s["spec"], v_lo, v_hi))
        for v in (v_lo, v_hi):
            c = case_of(s["spec"])
            jobs.append(dict(n_target=s["spec"]["n_target"], gamma=s["spec"]["gamma"],
                             r_c1=s["spec"]["r_c1"], v_over_vesc=v / c.v_esc,
                             strength=s["spec"]["strength"]))
    if not jobs:
        return dict(factors=list(factors), cases=[])
    r = simulate(jobs, checkpoints=tuple(factors), log=log, **sim_kw)
    rows = []
    for k, (spec, v_lo, v_hi) in enumerate(specs):
        c = case_of(spec)
        row = dict(m_tot=c.m_tot, strength=spec["strength"], n_target=spec["n_target"],
                   q_lo=c.q(v_lo), q_hi=c.q(v_hi), f_lo=[], f_hi=[], straddles=[], q_rd=[])
        for fac in factors:
            f_lo = float(r["f_at"][fac][2 * k])
            f_hi = float(r["f_at"][fac][2 * k + 1])
            ok = f_lo > 0.5 >= f_hi
            row["f_lo"].append(f_lo)
            row["f_hi"].append(f_hi)
            row["straddles"].append(bool(ok))
            row["q_rd"].append(qrd.Bracket(c, v_lo, v_hi, f_lo, f_hi).q_rd() if ok else None)
        rows.append(row)
    return dict(factors=list(factors), cases=rows, steps=r["steps"], seconds=r["seconds"],
                particles=r["particles"])


def main(argv=None):
    """Run or resume a campaign whose state lives in a JSON file."""
    import argparse
    import os
    import sys
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--state", required=True, help="JSON state file (created if missing)")
    ap.add_argument("--out", help="write the state here instead of --state")
    ap.add_argument("--rounds", type=int, default=100)
    ap.add_argument("--budget", type=float, default=1e30, help="seconds (checked between rounds)")
    ap.add_argument("--n-train", type=int, default=32)
    ap.add_argument("--n-held", type=int, default=16)
    ap.add_argument("--n-min", type=float, default=3.0e4)
    ap.add_argument("--n-max", type=float, default=1.0e5)
    ap.add_argument("--train-rounds", type=int, default=8)
    ap.add_argument("--t-end-ff", type=float, default=2.0)
    ap.add_argument("--t-end-sound", type=float, default=6.0,
                    help="end each run this many target sound-crossing times after contact "
                         "(0: use --t-end-ff free-fall times)")
    ap.add_argument("--max-cells", type=int, default=1 << 26)
    ap.add_argument("--far-factor", type=float, default=3.0)
    ap.add_argument("--check-every", type=int, default=10)
    ap.add_argument("--settling", metavar="OUT",
                    help="instead of advancing the campaign, run the ends of the closed "
                         "held-out bisection brackets to 4 t_end and write the result here")
    ap.add_argument("--settling-cases", type=int, default=None,
                    help="settling check on the first this many closed brackets only")
    ap.add_argument("--settling-factors", default="0.5,1,2,4",
                    help="multiples of t_end at which the settling check takes f_lr")
    a = ap.parse_args(argv)

    def log(*x):
        print(*x, file=sys.stderr, flush=True)

    if os.path.exists(a.state):
        with open(a.state) as f:
            state = json.load(f)
    else:
        state = new_campaign(a.n_train, a.n_held, n_min=a.n_min, n_max=a.n_max)
    out = a.out or a.state

    def save(st):
        tmp = out + ".tmp"
        with open(tmp, "w") as f:
            json.dump(st, f)
        os.replace(tmp, out)

    import torch
    torch.cuda.set_device(0)
    if a.settling:
        res = settling(state, log=log, max_cases=a.settling_cases,
                       factors=tuple(float(x) for x in a.settling_factors.split(",")),
                       t_end_ff=a.t_end_ff, t_end_sound=a.t_end_sound,
                       check_every=a.check_every, max_cells=a.max_cells,
                       far_factor=a.far_factor)
        with open(a.settling, "w") as f:
            json.dump(res, f)
        print(json.dumps(res), flush=True)
        return
    run(state, a.rounds, a.budget, log=log, train_rounds=a.train_rounds, save=save,
        t_end_ff=a.t_end_ff, t_end_sound=a.t_end_sound, check_every=a.check_every,
        max_cells=a.max_cells, far_factor=a.far_factor)
    print(json.dumps(summary(state)), flush=True)


if __name__ == "__main__":
    main()
