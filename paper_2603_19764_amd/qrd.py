"""Bracketing the catastrophic disruption threshold Q_RD* (impact energy at
which the largest remnant keeps half the total mass), with plain bisection
or with proposals from the small network trained on the GPU.

The specific impact energy follows the paper's Q_R equation,
Q_R = 1/2 M_t M_p v^2 / (M_t + M_p)^2 (sec. 3, catastrophic disruption), and
the bisection runs in log v at fixed mass ratio with linear interpolation in
Q_R for the threshold (Appendix A).  A "judge" is any callable that returns
the largest-remnant fraction f_lr of an impact; the full simulation is the
judge of record, a synthetic one serves the tests.  This is host-side
control logic: the network's forward, backward and Adam steps run in the
library's kernels (``sph_mlp_*``).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def q_r(m_target: float, m_proj: float, v: float) -> float:
    """Specific impact energy 1/2 M_t M_p v^2 / (M_t + M_p)^2."""
    mt = m_target + m_proj
    return 0.5 * m_target * m_proj * v * v / (mt * mt)


@dataclass
class Case:
    """One (total mass, strength) case: target/projectile masses, escape speed."""
    m_tot: float
    gamma: float          # M_p / M_t
    strength: int
    v_esc: float

    @property
    def m_t(self):
        return self.m_tot / (1.0 + self.gamma)

    @property
    def m_p(self):
        return self.m_tot * self.gamma / (1.0 + self.gamma)

    def q(self, v):
        return q_r(self.m_t, self.m_p, v)

    def features(self, v):
        return np.array([math.log10(self.m_tot), v / self.v_esc, self.gamma,
                         float(self.strength)], dtype=np.float64)


@dataclass
class Bracket:
    case: Case
    v_lo: float            # f_lr(v_lo) > 1/2 (disruption below threshold)
    v_hi: float            # f_lr(v_hi) <= 1/2
    f_lo: float = 1.0
    f_hi: float = 0.0
    sims: int = 0
    last_ratio: float = 0.0
    history: list = field(default_factory=list)

    def width(self) -> float:
        """Relative width of the bracket in Q_R."""
        q_lo, q_hi = self.case.q(self.v_lo), self.case.q(self.v_hi)
        return (q_hi - q_lo) / q_lo

    def q_rd(self) -> float:
        """Threshold by linear interpolation in Q_R between the bracket ends."""
        q_lo, q_hi = self.case.q(self.v_lo), self.case.q(self.v_hi)
        if self.f_lo == self.f_hi:
            return 0.5 * (q_lo + q_hi)
        return q_lo + (self.f_lo - 0.5) * (q_hi - q_lo) / (self.f_lo - self.f_hi)

    def update(self, v, f, source: str = "bisect"):
        old = math.log(self.v_hi / self.v_lo)
        self.sims += 1
        self.history.append((v, f, source))
        if f > 0.5:
            self.v_lo, self.f_lo = v, f
        else:
            self.v_hi, self.f_hi = v, f
        self.last_ratio = old / max(math.log(self.v_hi / self.v_lo), 1e-300)


def bisect_proposal(b: Bracket) -> float:
    """Midpoint of the bracket in log v."""
    return math.sqrt(b.v_lo * b.v_hi)


def model_root(b: Bracket, predict, n_grid: int = 65):
    """Impact speed where the model's f_lr crosses 1/2 inside the bracket, or
    None when the prediction is not monotone decreasing there or does not
    cross."""
    lv = np.linspace(math.log(b.v_lo), math.log(b.v_hi), n_grid)
    X = np.stack([b.case.features(vi) for vi in np.exp(lv)])
    f = np.asarray(predict(X), dtype=np.float64)
    if np.any(np.diff(f) > 1e-6) or not (f[0] > 0.5 > f[-1]):
        return None
    k = int(np.argmax(f <= 0.5))
    t = (f[k - 1] - 0.5) / (f[k - 1] - f[k])
    return math.exp(lv[k - 1] + t * (lv[k] - lv[k - 1]))


def model_proposal(b: Bracket, predict, tol: float = 0.05) -> tuple[float, bool]:
    """Next impact speed from the model (returns used_model).

    - Right after a simulation at a model root, step across it by a factor
      (1 + 0.4 tol) in v (about 0.8 tol in Q_R, since Q_R grows as v^2), on
      the side the outcome says the threshold lies: if the model was right
      this closes the bracket to within tol.
    - A step that did not close the bracket means the model is off here:
      the next proposal is the log-v midpoint.
    - Otherwise propose the model root, kept a little inside the bracket.
    - Fall back to the log-v midpoint when the model is not monotone or does
      not cross 1/2 on the bracket."""
    step = 1.0 + 0.4 * tol
    last = b.history[-1][2] if b.history else None
    if last == "root":
        v_last, f_last, _ = b.history[-1]
        v = v_last * step if f_last > 0.5 else v_last / step
        if b.v_lo < v < b.v_hi:
            return v, True
    if last == "step":
        return bisect_proposal(b), False
    root = model_root(b, predict)
    if root is None:
        return bisect_proposal(b), False
    lo, hi = b.v_lo * (1.0 + 0.1 * tol), b.v_hi / (1.0 + 0.1 * tol)
    return min(max(root, lo), hi), True


def bracket_to(b: Bracket, judge, tol: float = 0.05, predict=None, max_sims: int = 60) -> Bracket:
    """Refine a bracket until its relative Q_R width is <= tol: plain
    bisection in log v, or model proposals when ``predict`` (inputs -> f_lr)
    is given."""
    while b.width() > tol and b.sims < max_sims:
        if predict is None:
            b.update(bisect_proposal(b), float(judge(b.case, bisect_proposal(b))), "bisect")
            continue
        v, used = model_proposal(b, predict, tol)
        after_root = bool(b.history) and b.history[-1][2] == "root"
        source = ("step" if after_root else "root") if used else "bisect"
        b.update(v, float(judge(b.case, v)), source)
    return b
