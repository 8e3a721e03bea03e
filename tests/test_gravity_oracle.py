"""Pins of the FP64 direct-sum gravity and bound-mass oracle against closed
forms and invariants (no GPU)."""
import math

import numpy as np
import pytest

from oracle import oracle
from paper_2603_19764_amd import inputs

G = 6.674e-11


def test_two_bodies_closed_form():
    x = np.array([0.0, 3.0]); y = np.array([0.0, 4.0]); z = np.zeros(2)
    m = np.array([2.0e10, 5.0e10])
    eps = 0.5
    ax, ay, az, phi = oracle.gravity(x, y, z, m, G, eps)
    q = 25.0 + eps * eps
    assert math.isclose(ax[0], G * 5.0e10 * 3.0 / q ** 1.5, rel_tol=1e-14)
    assert math.isclose(ay[0], G * 5.0e10 * 4.0 / q ** 1.5, rel_tol=1e-14)
    assert math.isclose(ax[1], -G * 2.0e10 * 3.0 / q ** 1.5, rel_tol=1e-14)
    assert az[0] == 0.0
    assert math.isclose(phi[0], -G * 5.0e10 / math.sqrt(q), rel_tol=1e-14)
    assert math.isclose(phi[1], -G * 2.0e10 / math.sqrt(q), rel_tol=1e-14)


def test_momentum_conservation_and_inactive_sources():
    rng = np.random.default_rng(3)
    n = 300
    x, y, z = rng.normal(0, 1e3, (3, n))
    m = rng.uniform(1e9, 3e9, n)
    ax, ay, az, phi = oracle.gravity(x, y, z, m, G, 10.0)
    for a in (ax, ay, az):
        assert abs(np.sum(m * a)) <= 1e-12 * np.sum(m * np.abs(a))
    # inactive particles exert nothing but still feel the others
    act = (rng.uniform(size=n) < 0.5).astype(np.int32)
    bx, _, _, bphi = oracle.gravity(x, y, z, m, G, 10.0, active=act)
    keep = act.astype(bool)
    cx, _, _, cphi = oracle.gravity(x[keep], y[keep], z[keep], m[keep], G, 10.0)
    np.testing.assert_allclose(bx[keep], cx, rtol=1e-12, atol=1e-30)
    np.testing.assert_allclose(bphi[keep], cphi, rtol=1e-12)


def test_uniform_ball_potential_energy_and_interior_field():
    """A BCC ball of uniform density: W = 1/2 sum m phi -> -3 G M^2 / (5 R)
    and a(r) -> -G M r / R^3 inside, up to lattice discreteness."""
    P, sp = inputs.bcc_ball(20000, 1000.0)
    n = P.shape[0]
    R = 1000.0
    M = 1.0e15
    m = np.full(n, M / n)
    ax, ay, az, phi = oracle.gravity(P[:, 0], P[:, 1], P[:, 2], m, G, 0.05 * sp)
    W = 0.5 * np.sum(m * phi)
    assert abs(W / (-0.6 * G * M * M / R) - 1.0) < 0.01
    r = np.sqrt(np.sum(P * P, axis=1))
    inner = (r > 0.2 * R) & (r < 0.7 * R)
    ar = (ax * P[:, 0] + ay * P[:, 1] + az * P[:, 2])[inner] / r[inner]
    np.testing.assert_allclose(ar, -G * M * r[inner] / R ** 3, rtol=0.03)


def test_far_field_is_point_mass():
    rng = np.random.default_rng(4)
    n = 200
    x, y, z = rng.uniform(-1.0, 1.0, (3, n))
    m = rng.uniform(1.0, 2.0, n) * 1e9
    D = 1000.0
    x = np.append(x, D); y = np.append(y, 0.0); z = np.append(z, 0.0); m = np.append(m, 1.0)
    ax, _, _, _ = oracle.gravity(x, y, z, m, G, 0.0)
    xc = np.sum(m[:-1] * x[:-1]) / np.sum(m[:-1])
    assert abs(ax[-1] / (-G * np.sum(m[:-1]) / (D - xc) ** 2) - 1.0) < 1e-5


def test_runs_do_not_interact():
    rng = np.random.default_rng(5)
    a = rng.normal(0, 10, (3, 50)); b = rng.normal(0, 10, (3, 70))
    ma, mb = rng.uniform(1, 2, 50) * 1e9, rng.uniform(1, 2, 70) * 1e9
    X = np.concatenate([a, b], axis=1); Mm = np.concatenate([ma, mb])
    ax, _, _, phi = oracle.gravity(*X, Mm, G, 1.0, run_start=[0, 50, 120])
    ax_a, _, _, phi_a = oracle.gravity(*a, ma, G, 1.0)
    ax_b, _, _, phi_b = oracle.gravity(*b, mb, G, 1.0)
    np.testing.assert_array_equal(ax, np.concatenate([ax_a, ax_b]))
    np.testing.assert_array_equal(phi, np.concatenate([phi_a, phi_b]))


def test_bound_mass_cluster_with_escapers():
    """A cold cluster keeps every particle; particles launched well above
    escape speed leave, and only they."""
    P, sp = inputs.bcc_ball(2000, 100.0)
    n = P.shape[0]
    M = 1.0e14
    m = np.full(n, M / n)
    v = np.zeros((3, n))
    v_esc = math.sqrt(2 * G * M / 100.0)
    out = np.arange(0, n, 97)
    v[0, out] = 5.0 * v_esc
    bound, mb = oracle.bound_mass(P[:, 0], P[:, 1], P[:, 2], *v, m, G, 0.1 * sp)
    assert set(np.flatnonzero(bound == 0)) == set(out)
    assert math.isclose(mb[0], M * (n - out.size) / n, rel_tol=1e-12)


def test_bound_mass_two_receding_clusters_per_run():
    """Two clusters receding at many times their mutual escape speed: in one
    run nothing stays bound to the common centre of mass; a cluster alone in
    its own run at rest is entirely bound."""
    P, sp = inputs.bcc_ball(500, 10.0)
    n = P.shape[0]
    m = np.full(n, 1e12 / n)
    X = np.concatenate([P - [1000.0, 0, 0], P + [1000.0, 0, 0]])
    V = np.zeros((2 * n, 3)); V[:n, 0] = -50.0; V[n:, 0] = 50.0
    mm = np.concatenate([m, m])
    _, mb = oracle.bound_mass(*X.T, *V.T, mm, G, 0.1 * sp)
    assert mb[0] == 0.0
    _, mb2 = oracle.bound_mass(*np.concatenate([P, P]).T, *np.zeros((3, 2 * n)),
                               mm, G, 0.1 * sp, run_start=[0, n, 2 * n])
    np.testing.assert_allclose(mb2, [m.sum(), m.sum()], rtol=1e-12)
