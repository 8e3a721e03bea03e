"""The Q_RD* search with the simulation as judge: head-on impacts (self-
gravity, strength on or off) run in batches, one simulation per open
bracket per round; the bound-mass fraction of each run decides.  The
network is trained on the outcomes of training cases and then guides the
search on held-out cases next to plain bisection."""
import time

import numpy as np
import pytest

from tests.gpu_harness import say

pytestmark = pytest.mark.gpu


def test_qrd_scan_with_simulation_judge():
    from paper_2603_19764_amd import scan
    from paper_2603_19764_amd.proposal import MlpProposer
    t0 = time.perf_counter()
    judge = scan.judge_with_simulation(n_target=2000, t_end_ff=1.5, check_every=100, log=say)
    train = [scan.case_for(r, s) for r in (5e5, 9e5, 1.6e6, 2.8e6) for s in (0, 1)]
    held = [scan.case_for(r, s) for r in (1.2e6, 2.1e6) for s in (0, 1)]
    br_t, ok_t, outs = scan.bracket_rounds(train, judge, log=say)
    say(f"training brackets valid {ok_t}, sims {[b.sims for b in br_t]}, "
        f"{time.perf_counter() - t0:.0f} s")
    assert sum(ok_t) >= 6
    X = np.array([o[0] for o in outs])
    Y = np.array([o[1] for o in outs])
    net = MlpProposer(seed=1, lr=3e-3)
    loss = net.fit(X, Y, epochs=3000)
    say(f"network trained on {len(Y)} outcomes, mse {loss:.3e}")
    br_b, ok_b, _ = scan.bracket_rounds(held, judge, log=say)
    br_n, ok_n, _ = scan.bracket_rounds(held, judge, predict_for=lambda r: net.predict, log=say)
    sims_b = [b.sims for b, ok in zip(br_b, ok_b) if ok]
    sims_n = [b.sims for b, ok in zip(br_n, ok_n) if ok]
    q_b = [b.q_rd() for b, ok in zip(br_b, ok_b) if ok]
    q_n = [b.q_rd() for b, ok in zip(br_n, ok_n) if ok]
    say(f"held-out: bisection sims {sims_b} (Q_RD* {np.round(q_b, 0)}), "
        f"network sims {sims_n} (Q_RD* {np.round(q_n, 0)}), {time.perf_counter() - t0:.0f} s")
    assert ok_b == ok_n and sum(ok_b) >= 1
    for b, ok in zip(br_b + br_n, ok_b + ok_n):
        if ok:
            assert b.width() <= 0.05
    # the simulations each method needed to reach the same 5% brackets are
    # reported (and recorded in the design notes); at this resolution the
    # network's proposals do not reliably beat bisection, so no gain is
    # asserted here (the mock-judge test asserts the mechanism's gain)
    say(f"simulations: network {sum(sims_n)}, bisection {sum(sims_b)}")
    # both methods bracket the same thresholds
    for qb, qn in zip(q_b, q_n):
        assert abs(qn - qb) <= 0.05 * qb
