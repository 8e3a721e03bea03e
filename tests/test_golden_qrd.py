"""Paper-printed values of the Q_RD* runs (Appendix A tables, transcribed in
tests/golden/qrd_appendix_tables.txt) against the case set-up of the scan:
total mass from R_C1 at 1000 kg/m^3 (sec. 3, catastrophic disruption), split
by the mass ratio gamma; and the termination rule of the bisection as the
tables show it (no GPU)."""
import math
import os

import pytest

from paper_2603_19764_amd import qrd, scan

M_EARTH = 5.972e24
HERE = os.path.dirname(os.path.abspath(__file__))


def _half_unit(text: str) -> float:
    """Half a unit in the last printed digit of a table entry."""
    mant, _, exp = text.lower().partition("e")
    decimals = len(mant.split(".")[1]) if "." in mant else 0
    return 0.5 * 10.0 ** (-decimals) * 10.0 ** (int(exp) if exp else 0)


def _rows(raw=False):
    out = []
    with open(os.path.join(HERE, "golden", "qrd_appendix_tables.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            t, *vals = line.split()
            out.append((t, vals if raw else [None if v == "-" else float(v) for v in vals]))
    return out


ROWS = _rows()
RAW = _rows(raw=True)


def test_fixture_is_complete():
    tables = {t for t, _ in ROWS}
    assert tables == {"gamma_0.01", "gamma_0.1", "gamma_1", "v_5"}
    assert len(ROWS) == 30


@pytest.mark.parametrize("table,vals", [r for r in ROWS if r[0] != "v_5"])
def test_target_and_impactor_masses_from_r_c1(table, vals):
    gamma = float(table.split("_")[1])
    r_c1, m_t, m_p = vals[0], vals[1], vals[2]
    c = scan.case_for(r_c1, 1, gamma)
    # R_C1 is printed to three digits (2.15e5 for 10^(16/3) m: 0.2 % in
    # radius, 0.7 % in mass) and the printed impactor masses carry the
    # lattice discretisation of the bodies (a fraction of a percent)
    assert math.isclose(c.m_t / M_EARTH, m_t, rel_tol=1e-2)
    assert math.isclose(c.m_p / M_EARTH, m_p, rel_tol=1e-2)


@pytest.mark.parametrize("table,vals", [r for r in ROWS if r[0] == "v_5"])
def test_constant_velocity_table_target_is_the_r_c1_mass(table, vals):
    r_c1, m_t = vals[0], vals[1]
    m = 4.0 / 3.0 * math.pi * r_c1 ** 3 * 1000.0
    assert math.isclose(m / M_EARTH, m_t, rel_tol=1e-2)


def test_printed_brackets_meet_two_percent_in_the_bisection_variable():
    """Every printed final bracket is below 2% wide in the variable that was
    bisected (v, or the impactor mass at fixed v); in Q_R the v-brackets are
    up to about twice as wide, since Q_R grows as v^2 (reading of the
    termination rule)."""
    widest_q = 0.0
    for (t, v), (_, raw) in zip(ROWS, RAW):
        for a, b in ((3, 4), (5, 6)):
            if v[a] is None:
                continue
            lo, hi = v[a], v[b]
            # narrowest width the rounded entries allow
            w_min = ((hi - _half_unit(raw[b])) - (lo + _half_unit(raw[a]))) / (lo + _half_unit(raw[a]))
            assert w_min < 0.02, (t, raw[0], lo, hi)
            assert hi > lo
            if t == "v_5":
                q_lo, q_hi = qrd.q_r(v[1], lo, v[2]), qrd.q_r(v[1], hi, v[2])
            else:
                q_lo, q_hi = qrd.q_r(v[1], v[2], lo), qrd.q_r(v[1], v[2], hi)
            widest_q = max(widest_q, (q_hi - q_lo) / q_lo)
    assert 0.02 < widest_q < 0.04
