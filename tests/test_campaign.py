"""Host logic of the Q_RD* campaign (searches, windows, rounds) with a
synthetic judge: f_lr = 1 / (1 + (Q_R / Q*)^4) with a known threshold Q*
per case, so every bracket can be checked against the truth."""
import math

import numpy as np

from paper_2603_19764_amd import campaign


def q_star(spec):
    """Synthetic threshold: a power law in the total mass, higher with strength."""
    c = campaign.case_of(spec)
    return 1.5e5 * (c.m_tot / 1e22) ** 0.6 * (1.5 if spec["strength"] else 1.0)


def f_true(spec, v):
    c = campaign.case_of(spec)
    return 1.0 / (1.0 + (c.q(v) / q_star(spec)) ** 4)


def mock_judge(jobs, log=None, **kw):
    f = np.array([f_true(spec, v) for spec, v in jobs])
    return f, f, dict(steps=0, seconds=0.0, particles=0, runs=len(jobs))


class Exact:
    """A 'network' that knows the synthetic law, with its thresholds off by
    a factor ``bias`` in speed."""

    def __init__(self, specs, bias=1.0):
        self.specs = [(math.log10(campaign.case_of(s).m_tot), s) for s in specs]
        self.bias = bias

    def predict(self, X):
        out = []
        for lm, vv, _, st in X:
            spec = next(s for k, s in self.specs
                        if abs(k - lm) < 1e-6 and s["strength"] == int(st))
            c = campaign.case_of(spec)
            out.append(f_true(spec, vv * c.v_esc / self.bias))
        return np.array(out)


def _spec(r_c1, strength):
    return dict(n_target=1000, r_c1=r_c1, strength=strength, gamma=0.1)


def _run_search(s, predict=None, w=0.2, tol=0.05, rng=None):
    for _ in range(60):
        vs = campaign.next_speeds(s, predict, w, tol, rng)
        if not vs:
            break
        for v, src in vs:
            s["pts"].append([v, f_true(s["spec"], v), src])
    return s


def _threshold_in_range(spec):
    c = campaign.case_of(spec)
    v = campaign.v_at_q(c, q_star(spec))
    return 1.0 < v / c.v_esc < 10.0


def test_bisection_needs_nine_simulations_from_one_to_ten_vesc():
    spec = _spec(1.5e6, 1)
    assert _threshold_in_range(spec)
    s = _run_search(campaign.new_search(spec, "bisect"))
    assert s["status"] == "done"
    # two ends, then halvings of ln 10 until the Q_R width is <= 5% (2.47% in v)
    halvings = math.ceil(math.log2(math.log(10.0) / math.log(math.sqrt(1.05))))
    assert campaign.sims(s) == 2 + halvings == 9
    assert campaign.width(s) <= 0.05
    assert abs(campaign.q_rd(s) / q_star(spec) - 1.0) < 0.05


def test_exact_network_closes_in_three():
    specs = [_spec(r, st) for r in (6e5, 1.5e6, 3e6) for st in (0, 1)]
    net = Exact(specs)
    for spec in specs:
        if not _threshold_in_range(spec):
            continue
        s = _run_search(campaign.new_search(spec, "net"), net.predict, w=0.03)
        assert s["status"] == "done" and s["start"] == "net"
        assert campaign.sims(s) <= 3
        assert abs(campaign.q_rd(s) / q_star(spec) - 1.0) < 0.05


def test_biased_network_still_brackets_the_true_threshold():
    """A network whose thresholds are off by 30% in v still brackets the true
    one.  With the window matched to its error it needs fewer simulations
    than bisection; with a window six times too small, at most two more."""
    specs = [_spec(r, st) for r in (6e5, 1.5e6, 3e6) for st in (0, 1)]
    for bias in (0.7, 1.3):
        net = Exact(specs, bias=bias)
        for spec in specs:
            if not _threshold_in_range(spec):
                continue
            b = _run_search(campaign.new_search(spec, "bisect"))
            v_star = campaign.v_at_q(campaign.case_of(spec), q_star(spec))
            for w, extra in ((min(1.5 * abs(math.log(bias)), 0.5), -1), (0.05, 2)):
                s = _run_search(campaign.new_search(spec, "net"), net.predict, w=w)
                assert s["status"] == "done"
                v_lo, f_lo, v_hi, f_hi = campaign._sides(s)
                assert f_lo > 0.5 >= f_hi
                assert v_lo <= v_star <= v_hi
                assert campaign.sims(s) <= campaign.sims(b) + extra, (bias, w)


def test_no_crossing_starts_as_bisection_and_out_of_range_is_invalid():
    spec = _spec(1.5e6, 0)
    s = _run_search(campaign.new_search(spec, "net"), lambda X: np.ones(len(X)), w=0.1)
    assert s["start"] == "bisect" and s["status"] == "done"
    # a threshold far above 30 v_esc: both searches end invalid
    far = dict(spec, r_c1=4.64e5, strength=1)
    c = campaign.case_of(far)

    def f_far(v):
        return 1.0 if v < 100.0 * c.v_esc else 0.0

    for method in ("bisect", "net"):
        s = campaign.new_search(far, method)
        for _ in range(30):
            vs = campaign.next_speeds(s, lambda X: np.ones(len(X)), 0.2, 0.05)
            if not vs:
                break
            for v, src in vs:
                s["pts"].append([v, f_far(v), src])
        assert s["status"] == "invalid"


def test_sides_tolerate_non_monotone_outcomes():
    s = campaign.new_search(_spec(1.5e6, 0), "bisect")
    s["pts"] = [[1.0, 0.9, "end"], [2.0, 0.45, "bisect"], [3.0, 0.55, "bisect"],
                [10.0, 0.1, "end"]]
    v_lo, f_lo, v_hi, f_hi = campaign._sides(s)
    assert (v_lo, v_hi) == (1.0, 2.0) and f_lo > 0.5 >= f_hi


def test_campaign_rounds_with_synthetic_judge():
    state = campaign.new_campaign(n_train=8, n_held=6, seed=3, n_min=1000, n_max=2000)

    def trainer(searches):
        return Exact([s["spec"] for s in state["train"] + state["held"]], bias=1.05), 0.0, 0

    state = campaign.run(state, judge_fn=mock_judge, trainer=trainer)
    assert state["phase"] == "done"
    out = campaign.summary(state)
    assert out["compared"] >= 3
    assert out["sims_net"] < out["sims_bisect"]
    for r in out["cases"]:
        if r["status_bisect"] == "done" and r["status_net"] == "done":
            assert abs(r["q_rd_net"] / r["q_rd_bisect"] - 1.0) < 0.1
    # the window comes from the training searches' errors (5% bias in v)
    assert 0.03 <= state["w"] <= 0.5
    # rounds batch every open search: no more rounds than the slowest search
    assert out["rounds"] <= 8 + 12


def test_settling_runs_the_bracket_ends_past_t_end():
    """The settling check simulates both ends of every closed held-out
    bisection bracket at several multiples of t_end; with a synthetic
    outcome whose threshold drifts down by 3% per doubling of the time it
    must report the truth at each time, and at t_end the campaign's own
    thresholds."""
    state = campaign.new_campaign(n_train=4, n_held=5, seed=8, n_min=1000, n_max=2000)

    def trainer(searches):
        return Exact([s["spec"] for s in state["train"] + state["held"]]), 0.0, 0

    state = campaign.run(state, judge_fn=mock_judge, trainer=trainer)
    drift = 0.97

    def f_at(spec, v, fac):
        c = campaign.case_of(spec)
        return 1.0 / (1.0 + (c.q(v) / (q_star(spec) * drift ** math.log2(fac))) ** 4)

    calls = []

    def simulate(jobs, checkpoints, log=None, **kw):
        calls.append((len(jobs), tuple(checkpoints)))
        specs = [dict(n_target=j["n_target"], r_c1=j["r_c1"], strength=j["strength"],
                      gamma=j["gamma"]) for j in jobs]
        vs = [j["v_over_vesc"] * campaign.case_of(sp).v_esc for sp, j in zip(specs, jobs)]
        f = {c: np.array([f_at(sp, v, c) for sp, v in zip(specs, vs)]) for c in checkpoints}
        return dict(f_at=f, steps=0, seconds=0.0, particles=0)

    res = campaign.settling(state, simulate=simulate)
    closed = [s for s in state["held"] if s["method"] == "bisect" and s["status"] == "done"]
    assert len(res["cases"]) == len(closed) >= 3
    assert calls == [(2 * len(closed), (0.5, 1.0, 2.0, 4.0))]
    k1 = res["factors"].index(1.0)
    for row, s in zip(res["cases"], closed):
        v_lo, _, v_hi, _ = campaign._sides(s)
        assert row["straddles"][k1]
        assert abs(row["q_rd"][k1] / campaign.q_rd(s) - 1.0) < 1e-12
        for k, fac in enumerate(res["factors"]):
            want = f_at(s["spec"], v_lo, fac) > 0.5 >= f_at(s["spec"], v_hi, fac)
            assert row["straddles"][k] == want
            assert (row["q_rd"][k] is None) == (not want)
