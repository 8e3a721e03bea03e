"""The Q_RD* campaign with the batched simulation as judge, at small size:
head-on impacts (self-gravity, strength on or off) of 2,000-particle
targets.  Training rounds let the network pick the speeds of eight
training cases (retrained on every outcome after each round: the first
round at random speeds, then the network's threshold, windows around it
and halvings); then four
held-out cases are bracketed to 5% in Q_R by plain log-v bisection and by
the network's proposals side by side.  The network must need fewer
simulations, and both must find the same thresholds."""
import time

import pytest

from tests.gpu_harness import say

pytestmark = pytest.mark.gpu


def test_qrd_campaign_with_simulation_judge():
    from paper_2603_19764_amd import campaign
    t0 = time.perf_counter()
    state = campaign.new_campaign(n_train=8, n_held=4, seed=11, n_min=2000, n_max=2000)
    campaign.run(state, log=say, train_rounds=8, t_end_ff=1.5, check_every=10)
    out = campaign.summary(state)
    say(f"campaign: {out}, {time.perf_counter() - t0:.0f} s")
    assert state["phase"] == "done"
    assert out["train_done"] >= 4
    assert out["compared"] >= 3
    # the network's window comes from its error on the closed training brackets
    assert state["w_rms"] is not None and 0.03 <= state["w"] <= 0.5
    assert out["sims_net"] < out["sims_bisect"], out
    for r in out["cases"]:
        if r["status_bisect"] == "done" and r["status_net"] == "done":
            # both brackets are at most 5% wide in Q_R and hold the crossing
            # of the same simulated outcome: their thresholds agree closely
            assert abs(r["q_rd_net"] / r["q_rd_bisect"] - 1.0) <= 0.1, r
    # f_lr settles between t_end / 2 and t_end (reaccumulation is over)
    say(f"largest change of f_lr between t_end/2 and t_end: {out['max_f_change']:.3f}")
