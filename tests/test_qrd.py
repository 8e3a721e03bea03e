"""Host logic of Q_RD* bracketing (no GPU): the Q_R definition, bisection
termination, threshold interpolation, and the model-proposal rules with an
exact, a biased and a non-monotone predictor."""
import math

import numpy as np

from paper_2603_19764_amd import qrd


def _case():
    return qrd.Case(m_tot=1e21, gamma=0.1, strength=1, v_esc=300.0)


def _judge(q_star):
    return lambda case, v: 1.0 / (1.0 + (case.q(v) / q_star) ** 2.5)


def _fresh(case, judge):
    b = qrd.Bracket(case, case.v_esc, 40 * case.v_esc)
    b.f_lo, b.f_hi = judge(case, b.v_lo), judge(case, b.v_hi)
    return b


def _exact_predictor(case, q_star):
    def predict(X):
        v = np.asarray(X)[:, 1] * case.v_esc
        return 1.0 / (1.0 + (np.array([case.q(vi) for vi in v]) / q_star) ** 2.5)
    return predict


def test_q_r_definition():
    # equal masses: Q_R = v^2 / 8
    assert math.isclose(qrd.q_r(1.0, 1.0, 4.0), 2.0)
    # projectile negligible: Q_R -> 1/2 (M_p/M_t) v^2
    assert math.isclose(qrd.q_r(1.0, 1e-9, 10.0), 0.5e-9 * 100, rel_tol=1e-8)


def test_bisection_terminates_and_brackets_threshold():
    c = _case()
    q_star = c.q(4.1 * c.v_esc)
    judge = _judge(q_star)
    b = qrd.bracket_to(_fresh(c, judge), judge, 0.05)
    assert b.width() <= 0.05
    assert c.q(b.v_lo) <= q_star <= c.q(b.v_hi)
    # each bisection halves log v: ceil(log2(ln 40 / ln(1.05^(1/2)))) steps at most
    assert b.sims <= math.ceil(math.log2(math.log(40) / (0.5 * math.log(1.05)))) + 1
    assert abs(b.q_rd() / q_star - 1) < 0.05


def test_exact_model_closes_in_two_simulations():
    c = _case()
    for vs in (2.3, 7.7, 15.0):
        q_star = c.q(vs * c.v_esc)
        judge = _judge(q_star)
        b = qrd.bracket_to(_fresh(c, judge), judge, 0.05, predict=_exact_predictor(c, q_star))
        assert b.width() <= 0.05 and b.sims == 2
        assert c.q(b.v_lo) <= q_star <= c.q(b.v_hi)


def test_biased_model_still_converges():
    c = _case()
    q_star = c.q(6.0 * c.v_esc)
    judge = _judge(q_star)
    wrong = _exact_predictor(c, 1.7 * q_star)
    b = qrd.bracket_to(_fresh(c, judge), judge, 0.05, predict=wrong)
    assert b.width() <= 0.05
    assert c.q(b.v_lo) <= q_star <= c.q(b.v_hi)
    assert b.sims < 30


def test_non_monotone_model_falls_back_to_bisection():
    c = _case()
    q_star = c.q(6.0 * c.v_esc)
    judge = _judge(q_star)
    wavy = lambda X: 0.5 + 0.4 * np.sin(np.asarray(X)[:, 1])
    b1 = qrd.bracket_to(_fresh(c, judge), judge, 0.05)
    b2 = qrd.bracket_to(_fresh(c, judge), judge, 0.05, predict=wavy)
    assert b2.sims == b1.sims
    assert all(src == "bisect" for _, _, src in b2.history)


def test_batched_rounds_extend_a_bracket_that_does_not_disrupt():
    # the batched driver with a mock judge: one case's threshold lies above
    # the initial upper end (10 v_esc), the other's inside; both close
    from paper_2603_19764_amd import scan
    c_in = qrd.Case(m_tot=1e21, gamma=0.1, strength=0, v_esc=300.0)
    c_out = qrd.Case(m_tot=2e21, gamma=0.1, strength=1, v_esc=350.0)
    q_star = {id(c_in): c_in.q(4.0 * c_in.v_esc), id(c_out): c_out.q(17.0 * c_out.v_esc)}
    calls = []

    def judge_batch(jobs):
        calls.append(len(jobs))
        return [1.0 / (1.0 + (c.q(v) / q_star[id(c)]) ** 2.5) for c, v in jobs]

    brackets, valid, outcomes = scan.bracket_rounds([c_in, c_out], judge_batch)
    assert valid == [True, True]
    assert brackets[1].v_hi > 10.0 * c_out.v_esc and brackets[1].v_lo >= 10.0 * c_out.v_esc
    for b, c in zip(brackets, (c_in, c_out)):
        assert b.width() <= 0.05
        assert abs(b.q_rd() / q_star[id(c)] - 1.0) < 0.05
    assert calls[0] == 4 and calls[1] == 1      # both ends of both, then one extension
    assert len(outcomes) == sum(b.sims for b in brackets)
