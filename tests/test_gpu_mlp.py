"""GPU network kernels against the FP64 oracle, and what the trained network
gains over plain bisection when bracketing Q_RD* to 5 %.

The judge here is synthetic (a smooth family of thresholds Q*(M, strength)
with a logistic fraction f_lr(Q_R)); the full impact simulation is the judge
of record in the batched scan."""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as mo
from tests.gpu_harness import norm_err, say

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda").contiguous()


def test_forward_backward_adam_match_oracle():
    import torch
    from paper_2603_19764_amd import sph
    rng = np.random.default_rng(2)
    p = mo.init_params(5) + rng.normal(0, 0.05, mo.N_PARAMS)
    X = rng.normal(0, 1, (300, 4))
    Y = rng.uniform(0, 1, 300)
    P, Xd, Yd = _dev(p), _dev(X), _dev(Y)
    B = 300
    out = torch.empty(B, device="cuda")
    h1 = torch.empty((B, 64), device="cuda")
    h2 = torch.empty((B, 64), device="cuda")
    work = torch.empty(B * 129, device="cuda")
    G = torch.empty(mo.N_PARAMS, device="cuda")
    sph.sph_mlp_forward(Xd, P, out, h1, h2)
    sph.sph_mlp_backward(Xd, Yd, P, out, h1, h2, work, G)
    torch.cuda.synchronize()
    ro, rh1, rh2 = mo.forward(p, X)
    e_out = norm_err(out.cpu().numpy(), ro)
    e_h1 = norm_err(h1.cpu().numpy().T, rh1.T)
    rg = mo.backward(p, X, Y)
    e_g = norm_err(G.cpu().numpy(), rg)
    # Adam step
    m = rng.normal(0, 1e-3, mo.N_PARAMS)
    v = rng.uniform(0, 1e-5, mo.N_PARAMS)
    Md, Vd = _dev(m), _dev(v)
    g = G.cpu().numpy().astype(np.float64)
    sph.sph_mlp_adam(P, G, Md, Vd, 7, lr=1e-3)
    torch.cuda.synchronize()
    rp, rm, rv = mo.adam_step(p, g, m, v, 7, lr=1e-3)
    e_p = norm_err(P.cpu().numpy() - p, rp - p)
    say("mlp", dict(out=f"{e_out:.1e}", h1=f"{e_h1:.1e}", grad=f"{e_g:.1e}", adam=f"{e_p:.1e}"))
    assert e_out < 1e-5 and e_h1 < 1e-5
    # the loss kernel: mean squared error of the forward outputs
    loss = torch.empty(1, device="cuda")
    sph.sph_mlp_loss(out, Yd, loss)
    o64 = out.cpu().numpy().astype(np.float64)
    assert abs(float(loss.item()) - np.mean((o64 - Y) ** 2)) <= 1e-6 * np.mean((o64 - Y) ** 2)
    assert e_g < 1e-4
    assert e_p < 1e-4


def _judge_family():
    """Synthetic threshold Q*(M, strength) [J/kg] and f_lr(Q) = 1/(1+(Q/Q*)^2.5)."""
    def qstar(m_tot, strength):
        lm = math.log10(m_tot) - 20.0
        q = 3e4 * 10 ** (0.55 * lm)
        if strength:
            q *= 1.0 + 4.0 * 10 ** (-0.45 * (lm + 1.0))
        return q

    def judge(case, v):
        q = case.q(v)
        return 1.0 / (1.0 + (q / qstar(case.m_tot, case.strength)) ** 2.5)
    return judge


def _case(rng):
    from paper_2603_19764_amd.qrd import Case
    lm = rng.uniform(18.5, 22.5)
    m = 10 ** lm
    rho, gamma = 2700.0, 0.1
    r = (3 * m / (4 * math.pi * rho)) ** (1 / 3)
    G = 6.674e-11
    v_esc = math.sqrt(2 * G * m / (r * (1 + gamma ** (1 / 3))))
    return Case(m, gamma, int(rng.integers(0, 2)), v_esc)


def test_trained_network_needs_fewer_simulations_than_bisection():
    from paper_2603_19764_amd import qrd
    from paper_2603_19764_amd.proposal import MlpProposer
    judge = _judge_family()
    rng = np.random.default_rng(9)

    def fresh(case):
        return qrd.Bracket(case, case.v_esc * 1.0, case.v_esc * 40.0)

    # rounds of bisection on training cases give the network its data
    X, Y = [], []
    for _ in range(40):
        c = _case(rng)
        b = fresh(c)
        b.f_lo, b.f_hi = judge(c, b.v_lo), judge(c, b.v_hi)
        if not (b.f_lo > 0.5 >= b.f_hi):
            continue
        qrd.bracket_to(b, judge, 0.05)
        for v, f, _ in b.history + [(b.v_lo, b.f_lo, ""), (b.v_hi, b.f_hi, "")]:
            X.append(c.features(v))
            Y.append(f)
    net = MlpProposer(seed=1, lr=3e-3)
    loss = net.fit(np.array(X), np.array(Y), epochs=2500)
    say(f"trained on {len(Y)} outcomes, mse {loss:.2e}")
    assert loss < 2e-3
    n_bis, n_net = [], []
    for _ in range(12):
        c = _case(rng)
        b1, b2 = fresh(c), fresh(c)
        for b in (b1, b2):
            b.f_lo, b.f_hi = judge(c, b.v_lo), judge(c, b.v_hi)
        if not (b1.f_lo > 0.5 >= b1.f_hi):
            continue
        qrd.bracket_to(b1, judge, 0.05)
        qrd.bracket_to(b2, judge, 0.05, predict=net.predict)
        assert b1.width() <= 0.05 and b2.width() <= 0.05
        n_bis.append(b1.sims)
        n_net.append(b2.sims)
    say(f"held-out cases: bisection {np.mean(n_bis):.2f} sims, network {np.mean(n_net):.2f} sims")
    assert len(n_net) >= 6
    assert np.mean(n_net) < 0.6 * np.mean(n_bis)
