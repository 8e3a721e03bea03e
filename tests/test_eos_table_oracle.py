"""Pins of the oracle's tabulated EOS (sec. 2.3 takes P, c and T from
tables; the interpolation between nodes is the bilinear reading K7b).

Each pin checks the oracle against something other than itself: node values
given by the table, closed-form bilinear functions (which bilinear
interpolation reproduces exactly), the second-order error of bilinear
interpolation on a smooth function, clamping at the grid edges, and the
state routine's use of the table."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2603_19764_amd import inputs


def _grid(n_rho=7, n_u=11, seed=0):
    rng = np.random.default_rng(seed)
    rho = np.sort(2000.0 + 3000.0 * rng.random(n_rho))
    u = np.concatenate([[0.0], np.sort(1.0e7 * rng.random(n_u - 1))])
    return rho, u


def _mat(table, c_min=1.0):
    return dict(inputs.basalt_c1(), c_min=c_min, eos_table=table)


def _bilinear_table(rho, u):
    # three different bilinear functions of (rho, u), none symmetric in the axes
    R, U = np.meshgrid(rho, u, indexing="ij")
    P = 3.0e9 + 2.0e6 * R - 7.0e2 * U + 0.4 * R * U
    c = 3000.0 + 0.2 * R + 1.0e-4 * U + 2.0e-8 * R * U
    T = 300.0 + 1.0e-3 * R + 1.25e-3 * U - 1.0e-8 * R * U
    return dict(rho=rho, u=u, P=P, c=c, T=T)


def test_node_values():
    rho, u = _grid()
    tab = _bilinear_table(rho, u)
    R, U = np.meshgrid(rho, u, indexing="ij")
    P, c, T = orc.eos(_mat(tab), R, U)
    for got, want in ((P, tab["P"]), (c, tab["c"]), (T, tab["T"])):
        assert np.max(np.abs(got - want) / np.abs(want)) <= 2.3e-16


def test_bilinear_functions_reproduced():
    rho, u = _grid(n_rho=9, n_u=5, seed=1)
    tab = _bilinear_table(rho, u)
    rng = np.random.default_rng(2)
    r = rho[0] + (rho[-1] - rho[0]) * rng.random(4000)
    e = u[0] + (u[-1] - u[0]) * rng.random(4000)
    P, c, T = orc.eos(_mat(tab), r, e)
    want = (3.0e9 + 2.0e6 * r - 7.0e2 * e + 0.4 * r * e,
            3000.0 + 0.2 * r + 1.0e-4 * e + 2.0e-8 * r * e,
            300.0 + 1.0e-3 * r + 1.25e-3 * e - 1.0e-8 * r * e)
    for got, w in zip((P, c, T), want):
        assert np.max(np.abs(got - w) / np.abs(w)) < 1e-13


def test_outside_points_take_the_edge_values():
    rho, u = _grid(seed=3)
    tab = _bilinear_table(rho, u)
    mat = _mat(tab)
    r = np.array([rho[0] * 0.5, rho[-1] * 2.0, rho[0] * 0.9, 0.5 * (rho[2] + rho[3]), rho[-1] * 1.5])
    e = np.array([-1.0e6, u[-1] * 3.0, 0.5 * (u[4] + u[5]), -5.0, 0.5 * (u[1] + u[2])])
    rc, ec = np.clip(r, rho[0], rho[-1]), np.clip(e, u[0], u[-1])
    got = orc.eos(mat, r, e)
    want = (3.0e9 + 2.0e6 * rc - 7.0e2 * ec + 0.4 * rc * ec,
            3000.0 + 0.2 * rc + 1.0e-4 * ec + 2.0e-8 * rc * ec,
            300.0 + 1.0e-3 * rc + 1.25e-3 * ec - 1.0e-8 * rc * ec)
    for g, w in zip(got, want):
        assert np.max(np.abs(g - w) / np.abs(w)) < 1e-13


def test_second_order_convergence():
    # smooth, non-bilinear function on uniform grids: the maximum error of
    # bilinear interpolation falls by 4 when the spacing halves
    def f(R, U):
        return np.exp(R / 3000.0) * np.cos(U / 4.0e6) + (R / 3000.0) ** 3

    rng = np.random.default_rng(4)
    r = 2000.0 + 3000.0 * rng.random(20000)
    e = 1.0e7 * rng.random(20000)
    errs = []
    for n in (17, 33, 65):
        rho, u = np.linspace(2000.0, 5000.0, n), np.linspace(0.0, 1.0e7, n)
        R, U = np.meshgrid(rho, u, indexing="ij")
        v = f(R, U)
        tab = dict(rho=rho, u=u, P=v, c=v, T=v)
        P, _, _ = orc.eos(_mat(tab, c_min=0.0), r, e)
        errs.append(np.max(np.abs(P - f(r, e))))
    for a, b in zip(errs, errs[1:]):
        assert 3.3 < a / b < 4.7, errs


def test_sound_speed_floor():
    rho, u = _grid(seed=5)
    tab = _bilinear_table(rho, u)
    tab = dict(tab, c=np.full_like(tab["c"], 10.0))
    _, c, _ = orc.eos(_mat(tab, c_min=250.0), np.array([2500.0, 4000.0]), np.array([1e5, 5e6]))
    assert np.all(c == 250.0)


def test_state_uses_the_table():
    # P, c, T from the table; yield and the Poisson-route modulus from them
    tab = inputs.eos_table_stiffened(rho0=2700.0, c0=3000.0, gamma0=1.2, n_rho=12, n_u=10)
    mat = dict(inputs.granite_c3(), eos_table=tab)      # Poisson route, thermal softening
    rng = np.random.default_rng(6)
    rho = 2700.0 * (0.8 + 0.5 * rng.random(300))
    u = 2.0e6 * rng.random(300)
    P, c, T, Y, Gam = orc.state(rho, u, np.zeros(300, np.int32), [mat])
    Pe, ce, Te = orc.eos(mat, rho, u)
    assert np.array_equal(P, Pe) and np.array_equal(c, ce) and np.array_equal(T, Te)
    assert np.array_equal(Y, orc.yield_strength(mat, P, T, rho))
    nu = mat["nu"]
    np.testing.assert_allclose(Gam, 3 * (1 - 2 * nu) / (2 * (1 + nu)) * rho * c * c, rtol=1e-14)
    # the table is not Tillotson: the same material without it differs
    Pt, _, _, _ = orc.tillotson(mat, rho, u)
    assert np.max(np.abs(Pt - P)) > 1e6


def test_stiffened_table_is_exact_for_pressure():
    # P of the stiffened-gas law is bilinear in (rho, u), so the table gives
    # it exactly between nodes; T is linear in u
    tab = inputs.eos_table_stiffened(rho0=2700.0, c0=3000.0, gamma0=1.2, n_rho=20, n_u=16)
    rng = np.random.default_rng(7)
    rho = 2700.0 * (0.3 + 3.0 * rng.random(2000))
    u = 5.0e7 * rng.random(2000)
    P, c, T = orc.eos(dict(inputs.basalt_c1(), eos_table=tab), rho, u)
    Pw = 3000.0 ** 2 * (rho - 2700.0) + 1.2 * rho * u
    assert np.max(np.abs(P - Pw)) <= 1e-12 * np.max(np.abs(Pw))
    np.testing.assert_allclose(T, 300.0 + u / 800.0, rtol=1e-13)


@pytest.mark.parametrize("rho_over_rho0", [0.95, 1.0, 1.1, 1.4])
def test_fine_table_of_tillotson_converges(rho_over_rho0):
    # a fine table filled with the oracle's Tillotson reproduces it to the
    # interpolation error (cold compressed branch, u below E_iv)
    mat = inputs.basalt_c1()
    rho = np.linspace(2000.0, 4500.0, 401)
    u = np.linspace(0.0, 4.0e6, 201)
    R, U = np.meshgrid(rho, u, indexing="ij")
    P, c, _, _ = orc.tillotson(mat, R.ravel(), U.ravel())
    tab = dict(rho=rho, u=u, P=P.reshape(R.shape), c=c.reshape(R.shape),
               T=mat["T_ref"] + U / mat["cv"])
    r = np.full(50, 2700.0 * rho_over_rho0)
    e = np.linspace(1.0e4, 3.9e6, 50)
    Pt, ct, _ = orc.eos(dict(mat, eos_table=tab), r, e)
    Pw, cw, _, _ = orc.tillotson(mat, r, e)
    scale = mat["A"] * 0.05
    assert np.max(np.abs(Pt - Pw)) < 1e-4 * scale + 1e-5 * np.max(np.abs(Pw))
    np.testing.assert_allclose(ct, cw, rtol=2e-4)


def test_tillotson_tension_cut():
    """Reading K7c: with rho_limit the cold formula gives no pressure below
    rho_limit rho0; above it, and in the hot branch, nothing changes; in the
    blend the cold part vanishes, so P runs from 0 at E_iv to the hot value at
    E_cv."""
    base = inputs.granite_c3()
    cut = dict(base, rho_limit=0.9)
    r0, eiv, ecv = base["rho0"], base["Eiv"], base["Ecv"]
    rho = np.array([0.5, 0.85, 0.899]) * r0
    u = np.full(3, 1.0e3)                          # cold: the thermal term is small
    P, c, _, _ = orc.tillotson(cut, rho, u)
    assert np.all(P == 0.0) and np.all(c == base["c_min"])
    P0, _, _, _ = orc.tillotson(base, rho, u)
    assert np.all(P0 < -1e8)                       # the formula's tension that is cut
    rho = np.array([0.9, 0.95, 1.0, 1.3]) * r0
    u = np.array([0.0, 0.5 * eiv, 2.0 * ecv, 0.9 * eiv])
    for a, b in zip(orc.tillotson(cut, rho, u), orc.tillotson(base, rho, u)):
        assert np.array_equal(a, b)
    hot_rho = np.array([0.3, 0.6, 0.85]) * r0
    for a, b in zip(orc.tillotson(cut, hot_rho, np.full(3, 1.5 * ecv)),
                    orc.tillotson(base, hot_rho, np.full(3, 1.5 * ecv))):
        assert np.array_equal(a, b)
    # blend: zero at E_iv, the uncut hot value at E_cv
    Pl, _, _, _ = orc.tillotson(cut, hot_rho, np.full(3, eiv * (1 + 1e-12)))
    assert np.all(np.abs(Pl) < 1e-6 * base["A"])
    Ph, _, _, _ = orc.tillotson(cut, hot_rho, np.full(3, ecv * (1 - 1e-12)))
    Pb, _, _, _ = orc.tillotson(base, hot_rho, np.full(3, ecv))
    np.testing.assert_allclose(Ph, Pb, rtol=1e-9, atol=1e-3)
