"""Pins of the oracle's artificial viscosity and of the Tillotson EOS away
from the reference state.

The artificial viscosity (sec. 2.1: the Monaghan viscosity term of the
momentum equation, the mean-kernel-gradient form, and the AV_heating eq.)
is checked against what it exists to do, not against a retyped formula:
it must repel approaching pairs and heat them, leave receding pairs alone
exactly, grow linearly with the approach speed when that is small against
the sound speed and quadratically when it is large, stay finite when two
particles coincide (the role of the epsilon h_bar^2 term), and give a
planar shock whose jumps meet the Rankine-Hugoniot conditions, which follow
from conservation alone.

The Tillotson EOS (reading R9/K7: the published form, Tillotson 1962 as
restated by Melosh 1989) is checked in its limits: the hot expanded branch
becomes the ideal gas P = a rho u once the non-ideal part, damped as a
Gaussian in z = rho0/rho - 1, has died out; the Grueneisen parameter
(1/rho) dP/du of the compressed branch runs from a + b at low energy to a at
high energy; at zero energy the compressed branch is the polynomial cold
curve A mu + B mu^2.
"""
import math

import numpy as np
import pytest

from paper_2603_19764_amd import inputs


# ------------------------------------------------------ artificial viscosity
def _pair_forces(orc, v, r=1.0, h=1.0, c=1000.0, rho=2700.0, approach=True, prm=None):
    """Two equal particles on the x axis at +r/2 (i) and -r/2 (j), moving
    towards each other (approach) or apart at relative speed v, with zero
    pressure and stress so that only the viscosity acts."""
    s = -1.0 if approach else 1.0
    x = np.array([0.5 * r, -0.5 * r])
    zero = np.zeros(2)
    vx = np.array([0.5 * s * v, -0.5 * s * v])
    m = np.full(2, 1000.0)
    hh = np.full(2, h)
    rr = np.full(2, rho)
    prm = prm or inputs.default_params()
    a, du, _ = orc.forces(x, zero, zero, vx, zero, zero, m, hh, rr, np.ones(2), zero,
                          np.full(2, c), np.zeros((5, 2)), prm)
    return a, du, vx, m


@pytest.mark.parametrize("v", [1e-3, 1.0, 3.0e3, 1.0e6])
def test_av_repels_and_heats_approaching_pairs(orc, v):
    """An approaching pair is pushed apart (a_i along +x for the particle at
    +x) and both particles heat up; the heating equals the kinetic energy
    the viscosity removes, and is positive."""
    a, du, vx, m = _pair_forces(orc, v)
    assert a[0, 0] > 0.0 and a[0, 1] < 0.0
    assert a[1, 0] == 0.0 and a[2, 0] == 0.0
    assert du[0] > 0.0 and du[1] > 0.0
    work = np.sum(m * vx * a[0])
    heat = np.sum(m * du)
    assert work < 0.0
    assert heat == pytest.approx(-work, rel=1e-12)


@pytest.mark.parametrize("v", [1e-3, 1.0, 3.0e3, 1.0e6])
def test_av_ignores_receding_and_sliding_pairs(orc, v):
    """A receding pair, and a pair sliding past each other (v_ij
    perpendicular to x_ij), feel no viscosity at all: with zero pressure and
    stress every derivative is exactly zero."""
    a, du, _, _ = _pair_forces(orc, v, approach=False)
    assert np.all(a == 0.0) and np.all(du == 0.0)
    x = np.array([0.5, -0.5])
    zero = np.zeros(2)
    vy = np.array([0.5 * v, -0.5 * v])
    a, du, _ = orc.forces(x, zero, zero, zero, vy, zero, np.full(2, 1e3), np.ones(2),
                          np.full(2, 2700.0), np.ones(2), zero, np.full(2, 1e3),
                          np.zeros((5, 2)), inputs.default_params())
    assert np.all(a == 0.0) and np.all(du == 0.0)


def test_av_linear_then_quadratic_in_approach_speed(orc):
    """Monaghan's viscosity is a bulk (alpha, linear in the approach speed)
    plus a von Neumann-Richtmyer (beta, quadratic) term: doubling a small
    approach speed doubles the repulsion, doubling a large one quadruples
    it.  With alpha = 0 it is quadratic at every speed, with beta = 0
    linear."""
    def ratio(v, **kw):
        prm = inputs.default_params(**kw)
        return _pair_forces(orc, 2 * v, prm=prm)[0][0, 0] / _pair_forces(orc, v, prm=prm)[0][0, 0]
    assert ratio(1e-3) == pytest.approx(2.0, rel=1e-5)
    assert ratio(1e7) == pytest.approx(4.0, rel=1e-3)
    assert ratio(1.0, av_alpha=0.0) == pytest.approx(4.0, rel=1e-12)
    assert ratio(1e6, av_beta=0.0) == pytest.approx(2.0, rel=1e-12)


def test_av_stays_finite_when_particles_coincide(orc):
    """The epsilon h_bar^2 term keeps the viscosity finite as two approaching
    particles close in: at fixed approach speed the repulsion vanishes like
    r^2 (halving r quarters it) instead of growing like 1/r."""
    v = 1.0
    a1 = _pair_forces(orc, v, r=1e-4)[0][0, 0]
    a2 = _pair_forces(orc, v, r=2e-4)[0][0, 0]
    assert a1 > 0.0
    assert a2 / a1 == pytest.approx(4.0, rel=1e-2)
    a0 = _pair_forces(orc, v, r=1e-7)[0][0, 0]
    assert a0 < 1e-5 * a1


def _layers(nx, ny, nz):
    k = np.arange(nx * ny * nz) % nx
    return k


def test_planar_shock_meets_rankine_hugoniot(orc):
    """Two half-spaces of basalt (fluid, Tillotson, u = 0, at rho0) collide
    head on at +-v = 1 km/s in a column periodic across the flow.  Two
    shocks run outwards and leave the material between them at rest.
    Conservation across a shock moving at D (lab frame) into material
    arriving at v fixes the jumps whatever the dissipation that forms it:
        mass      rho1 D = rho0 (D + v)
        momentum  P1 = rho0 (D + v) v
        energy    u1 = v^2 / 2
    Checked on the layers between the two fronts, away from the contact
    (where SPH shows the known excess heating) and from the fronts."""
    nx, ny, nz = 100, 6, 6
    x, y, z = inputs.lattice(nx, ny, nz, 1.0)
    N = x.size
    layer = _layers(nx, ny, nz)
    mat = inputs.fluid(inputs.basalt_c1())
    prm = inputs.default_params(box=(0.0, ny, nz))
    rho0 = mat["rho0"]
    m = np.full(N, rho0)
    rho, _ = orc.density(x, y, z, m, np.full(N, 1.3), prm)
    interior = (layer >= 5) & (layer < nx - 5)
    m = m * rho0 / rho[interior].mean()        # interior lattice at rho0, P = 0
    v = 1.0e3
    vx = np.where(layer < nx // 2, v, -v)
    st = dict(x=x, y=y, z=z, m=m, h=np.full(N, 1.3), mat=np.zeros(N, np.int32), vx=vx,
              vy=np.zeros(N), vz=np.zeros(N), u=np.zeros(N), S=np.zeros((5, N)),
              fixed=np.zeros(N, np.uint8))
    it = orc.Integrator(st, [mat], prm)
    xc = 0.5 * nx
    e0 = np.sum(m * (0.5 * vx * vx))

    def profile():
        lx = np.bincount(layer, it["x"], nx) / (ny * nz)
        lr = np.bincount(layer, it["rho"], nx) / (ny * nz)
        return lx, lr

    def fronts(lx, lr, rho1):
        mid = 0.5 * (rho0 + rho1)
        out = []
        for ks in (range(nx // 2, nx - 1), range(nx // 2 - 1, 0, -1)):
            for k in ks:
                k2 = k + 1 if ks.step == 1 else k - 1
                if lr[k] >= mid > lr[k2]:
                    f = (lr[k] - mid) / (lr[k] - lr[k2])
                    out.append(abs(lx[k] + f * (lx[k2] - lx[k]) - xc))
                    break
        assert len(out) == 2
        return 0.5 * (out[0] + out[1])

    t = 0.0
    while t < 2.0e-3:
        t += it.dt
        it.step()
    lx1, lr1 = profile()
    t1 = t
    while t < 4.0e-3:
        t += it.dt
        it.step()
    lx2, lr2 = profile()
    t2 = t
    # shocked layers: 5..12 m from the contact on either side at t2
    d = np.abs(lx2 - xc)
    band = (d > 5.0) & (d < 12.0)
    sel = band[layer]
    rho1 = float(it["rho"][sel].mean())
    u1 = float(it["u"][sel].mean())
    P1 = float(it["P"][sel].mean())
    assert abs(float(it["vx"][sel].mean())) < 1e-3 * v
    D = (fronts(lx2, lr2, rho1) - fronts(lx1, lr1, rho1)) / (t2 - t1)
    assert rho1 > 1.1 * rho0
    assert u1 == pytest.approx(0.5 * v * v, rel=0.05)
    assert rho1 * D == pytest.approx(rho0 * (D + v), rel=0.05)
    assert P1 == pytest.approx(rho0 * (D + v) * v, rel=0.05)
    # the whole column keeps its energy (kinetic + internal) through the
    # shock heating, to the accuracy of the time integration
    e1 = np.sum(m * (0.5 * it["vx"] ** 2 + it["u"]))
    assert e1 == pytest.approx(e0, rel=0.02)


# ------------------------------------------------------------------ Tillotson
def _granite():
    return inputs.granite_c3()


@pytest.mark.parametrize("eta", [0.25, 0.1])
def test_tillotson_hot_expanded_limit_is_ideal_gas(orc, eta):
    """Hot (u >= E_cv) and expanded: the non-ideal part is damped by
    exp(-alpha z^2), z = rho0/rho - 1, so by z = 3 (exp(-45)) the pressure is
    the ideal gas P = a rho u to double precision, at any energy above
    E_cv."""
    for mat in (_granite(), inputs.basalt_c1()):
        rho = eta * mat["rho0"]
        for u in (mat["Ecv"], 2.0 * mat["Ecv"], 1.0e9):
            P = orc.tillotson(mat, np.array([rho]), np.array([u]))[0][0]
            assert P / (rho * u) == pytest.approx(mat["a"], rel=1e-12)


def test_tillotson_hot_expanded_near_reference_density(orc):
    """Hot and barely expanded: as rho -> rho0 from below the damping factors
    go to 1 and the hot branch meets the compressed branch (both are
    a rho u + b rho u / (u/E0 + 1) at rho0)."""
    mat = _granite()
    u = 2.0 * mat["Ecv"]
    rho0 = mat["rho0"]
    below = orc.tillotson(mat, np.array([rho0 * (1 - 1e-10)]), np.array([u]))[0][0]
    above = orc.tillotson(mat, np.array([rho0]), np.array([u]))[0][0]
    at = (mat["a"] + mat["b"] / (u / mat["E0"] + 1.0)) * rho0 * u
    assert above == pytest.approx(at, rel=1e-14)
    assert below == pytest.approx(at, rel=1e-8)


@pytest.mark.parametrize("eta", [1.0, 1.2, 1.6])
def test_tillotson_grueneisen_limits_when_compressed(orc, eta):
    """Compressed branch: the Grueneisen parameter (1/rho) (dP/du)_rho is
    a + b at low energy and falls to a at high energy (finite differences
    of P, independent of the oracle's analytic derivative)."""
    for mat in (_granite(), inputs.basalt_c1()):
        rho = eta * mat["rho0"]

        def gamma(u, du):
            P = orc.tillotson(mat, np.array([rho, rho]), np.array([u + du, u - du]))[0]
            return (P[0] - P[1]) / (2 * du) / rho

        assert gamma(1e-5 * mat["E0"], 1e-7 * mat["E0"]) == pytest.approx(
            mat["a"] + mat["b"], rel=1e-4)
        assert gamma(1e6 * mat["E0"], 1e3 * mat["E0"]) == pytest.approx(mat["a"], rel=1e-5)


def test_tillotson_cold_compression_curve(orc):
    """At zero internal energy the compressed branch is the polynomial cold
    curve P = A mu + B mu^2, mu = rho/rho0 - 1: its bulk modulus at rho0 is A
    and it stiffens with compression through B (second difference 2B)."""
    for mat in (_granite(), inputs.basalt_c1()):
        rho0 = mat["rho0"]
        mu = np.array([0.05, 0.2, 0.5, 1.0])
        P = orc.tillotson(mat, rho0 * (1 + mu), np.zeros(mu.size))[0]
        np.testing.assert_allclose(P, mat["A"] * mu + mat["B"] * mu * mu, rtol=1e-13)
        d = 0.1
        Pm, P0, Pp = orc.tillotson(mat, rho0 * np.array([1.3 - d, 1.3, 1.3 + d]), np.zeros(3))[0]
        assert (Pp - 2 * P0 + Pm) / (d * d) == pytest.approx(2 * mat["B"], rel=1e-9)
