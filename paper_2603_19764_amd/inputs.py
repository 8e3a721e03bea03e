"""Seeded synthetic inputs for the strength-SPH hot path.

This module only lays out particles, draws random numbers and fills input
tables; it holds none of the method's arithmetic (no kernel, Tillotson, yield
or force formula, no table interpolation).  Both the GPU path and the CPU
oracle take their inputs from here.  The one closed form evaluated here is the
stiffened-gas law that fills the synthetic EOS table (``eos_table_stiffened``),
a stand-in for an M-ANEOS table, which is data for the method.

A workload is a dict of numpy arrays in SI units:
  x, y, z, vx, vy, vz, m, h, u   float64 (n,)
  S                              float64 (5, n)   components xx, yy, xy, xz, yz
  mat                            int32 (n,)       index into ``mats``
  fixed                          uint8 (n,)       1 = boundary particle, never integrated
plus ``mats`` (list of material dicts), ``params`` (dict) and ``name``.

Material parameters are inputs of a workload.  Tillotson constants are the
published basalt and granite sets; the strength constants follow the
workload descriptions (pressure-dependent Collins yield, Drucker-Prager
friction for the granular column).
"""
from __future__ import annotations

import math

import numpy as np

# Tillotson basalt (Benz & Asphaug 1999) and granite (Melosh 1989) constants.
_BASALT_EOS = dict(rho0=2700.0, A=26.7e9, B=26.7e9, E0=487.0e6, Eiv=4.72e6, Ecv=18.2e6,
                   a=0.5, b=1.5, alpha=5.0, beta=5.0)
_GRANITE_EOS = dict(rho0=2680.0, A=18.0e9, B=18.0e9, E0=16.0e6, Eiv=3.5e6, Ecv=18.0e6,
                    a=0.5, b=1.3, alpha=5.0, beta=5.0)


def _cmin(eos):
    # sound-speed floor: one tenth of the linear bulk sound speed sqrt(A/rho0)
    return 0.1 * math.sqrt(eos["A"] / eos["rho0"])


def basalt_c1() -> dict:
    """Basalt with constant shear modulus 22.7 GPa, Collins yield Y0 = 10 MPa,
    Ym = 3.5 GPa, mu_i = 1.5, mu_d = 0.8, thermal softening xi = 1.2,
    T_melt = 1373 K."""
    e = dict(_BASALT_EOS)
    return dict(e, cv=800.0, T_ref=300.0, c_min=_cmin(e), shear_modulus=22.7e9, nu=0.25,
                Y0=10.0e6, Ym=3.5e9, mu_i=1.5, mu_d=0.8, xi=1.2, T_melt=1373.0,
                strength_on=1, thermal_softening_on=1)


def granular_c2() -> dict:
    """Granular basalt (rho0 = 2600): zero cohesion, friction tan(30 deg), shear
    modulus from the bulk modulus with nu = 0.25, no thermal softening."""
    e = dict(_BASALT_EOS, rho0=2600.0)
    return dict(e, cv=800.0, T_ref=300.0, c_min=_cmin(e), shear_modulus=0.0, nu=0.25,
                Y0=0.0, Ym=3.5e9, mu_i=2.0, mu_d=math.tan(math.radians(30.0)), xi=1.2,
                T_melt=1373.0, strength_on=1, thermal_softening_on=0)


def granite_c3() -> dict:
    """Granite with Collins yield (Y0 = 0, Ym = 3.5 GPa, mu_i = 2.0, mu_d = 0.8),
    thermal softening xi = 1.2, T_melt = 1373 K, Poisson-route shear modulus."""
    e = dict(_GRANITE_EOS)
    return dict(e, cv=800.0, T_ref=300.0, c_min=_cmin(e), shear_modulus=0.0, nu=0.25,
                Y0=0.0, Ym=3.5e9, mu_i=2.0, mu_d=0.8, xi=1.2, T_melt=1373.0,
                strength_on=1, thermal_softening_on=1)


def granite_impact() -> dict:
    """The granite of the two-sphere impact with cold expanded states cut to
    zero pressure below 0.9 rho0 (``rho_limit``): the material of the
    batched impact scans, whose bodies run for thousands of steps with free
    surfaces."""
    return dict(granite_c3(), rho_limit=0.9)


def fluid(mat: dict) -> dict:
    """The same material with strength switched off."""
    return dict(mat, strength_on=0)


def eos_table_stiffened(rho0: float, c0: float, gamma0: float, cv: float = 800.0,
                        T_ref: float = 300.0, rho_range=(0.25, 4.0), u_max: float = 1.0e8,
                        n_rho: int = 96, n_u: int = 96, u_first: float = 1.0e3) -> dict:
    """Synthetic tabulated EOS standing in for an M-ANEOS table.

    Node values follow the stiffened-gas (linear Mie-Grueneisen) law
        P = c0^2 (rho - rho0) + gamma0 rho u,
        c^2 = c0^2 + gamma0 u + gamma0 P / rho   (clipped at 0),
        T = T_ref + u / cv,
    on density nodes geometric over rho_range * rho0 and energy nodes 0 plus
    a geometric series from u_first to u_max.  Returns the dict that
    materials take as ``eos_table``: rho (n_rho), u (n_u), P, c, T
    (n_rho x n_u)."""
    rho = rho0 * np.geomspace(rho_range[0], rho_range[1], n_rho)
    u = np.concatenate([[0.0], np.geomspace(u_first, u_max, n_u - 1)])
    R, U = np.meshgrid(rho, u, indexing="ij")
    P = c0 * c0 * (R - rho0) + gamma0 * R * U
    c2 = c0 * c0 + gamma0 * U + gamma0 * P / R
    return dict(rho=rho, u=u, P=P, c=np.sqrt(np.maximum(c2, 0.0)), T=T_ref + U / cv)


def tabulated(mat: dict, table: dict) -> dict:
    """The same material with its EOS taken from ``table``."""
    return dict(mat, eos_table=table)


def default_params(**kw) -> dict:
    """Monaghan artificial viscosity alpha = 1, beta = 2, epsilon = 0.01;
    Courant factor 0.3; objective Jaumann rotation sign; correction tensor on;
    self-gravity off (grav_G = 0; softening 0.5 h_max and opening angle 0.6
    when switched on)."""
    p = dict(av_alpha=1.0, av_beta=2.0, av_eps=0.01, eta_C=0.3, rot_sign=1.0,
             g=(0.0, 0.0, 0.0), box=(0.0, 0.0, 0.0), use_correction=1, omega_one=0,
             grav_G=0.0, grav_eps_over_h=0.5, grav_theta=0.6, adapt_ngb=0.0, adapt_skin=1.25,
             eta_a=0.0, rungs=0, far_factor=0.0)
    p.update(kw)
    return p


def _empty(n):
    return dict(vx=np.zeros(n), vy=np.zeros(n), vz=np.zeros(n), u=np.zeros(n),
                S=np.zeros((5, n)), mat=np.zeros(n, dtype=np.int32),
                fixed=np.zeros(n, dtype=np.uint8))


def lattice(nx, ny, nz, spacing, origin=(0.0, 0.0, 0.0)):
    """Cubic lattice of cell centres, x fastest."""
    i = np.arange(nx, dtype=np.float64)
    j = np.arange(ny, dtype=np.float64)
    k = np.arange(nz, dtype=np.float64)
    Z, Y, X = np.meshgrid(k, j, i, indexing="ij")
    return (origin[0] + (X.ravel() + 0.5) * spacing,
            origin[1] + (Y.ravel() + 0.5) * spacing,
            origin[2] + (Z.ravel() + 0.5) * spacing)


def c1_block(n_side: int = 16, variant: str = "", seed_pos: int = 1, seed_vel: int = 2,
             seed_S: int = 3) -> dict:
    """Single strength step workload: n_side^3 particles on a cubic lattice of
    spacing 1 m, positions jittered uniformly by +/-0.05 m, m = 2700 kg,
    h = 1.3 m, u = 1e4 J/kg, v = (1e-2 y, 0, 0) + N(0, (1e-3 m/s)^2) per
    component, S = 0.  Variants: "s" draws S ~ N(0, (10 MPa)^2) per component,
    "y" draws S ~ N(0, (200 MPa)^2) so that the plastic rescaling is active."""
    sp = 1.0
    x, y, z = lattice(n_side, n_side, n_side, sp)
    n = x.size
    rng = np.random.Generator(np.random.PCG64(seed_pos))
    jit = rng.uniform(-0.05 * sp, 0.05 * sp, size=(3, n))
    x, y, z = x + jit[0], y + jit[1], z + jit[2]
    w = _empty(n)
    rv = np.random.Generator(np.random.PCG64(seed_vel))
    noise = rv.normal(0.0, 1e-3, size=(3, n))
    w.update(x=x, y=y, z=z, m=np.full(n, 2700.0 * sp ** 3), h=np.full(n, 1.3 * sp),
             u=np.full(n, 1.0e4))
    w["vx"] = 1e-2 * y + noise[0]
    w["vy"] = noise[1]
    w["vz"] = noise[2]
    if variant:
        sig = {"s": 10.0e6, "y": 200.0e6}[variant]
        rs = np.random.Generator(np.random.PCG64(seed_S))
        w["S"] = rs.normal(0.0, sig, size=(5, n))
    w.update(mats=[basalt_c1()], params=default_params(),
             name=f"c1_{n_side}^3{('_' + variant) if variant else ''}")
    return w


def c2_column(scale: float = 1.0) -> dict:
    """Granular column: a 0.2 x 0.1 x 0.05 m block (x length, y height, z
    width) on a cubic lattice of spacing 1.70998 mm (117 x 58 x 29 =
    196,794 mobile particles, no jitter), rho0 = 2600 kg/m^3, u = 0, v = 0,
    S = 0, on a floor of 4 layers of fixed particles below y = 0 spanning
    x in [-0.02, 0.42] m and the block's width; g = (0, -9.81, 0).

    ``scale`` < 1 shrinks every extent (same spacing) for small test copies."""
    sp = 1.70998e-3
    nx = int(round(0.2 * scale / sp))
    ny = int(round(0.1 * scale / sp))
    nz = int(round(0.05 * scale / sp))
    bx, by, bz = lattice(nx, ny, nz, sp)
    i0 = int(math.floor(-0.02 * scale / sp))
    i1 = int(math.ceil(0.42 * scale / sp))
    fx, fy, fz = lattice(i1 - i0, 4, nz, sp, origin=(i0 * sp, -4 * sp, 0.0))
    x = np.concatenate([bx, fx])
    y = np.concatenate([by, fy])
    z = np.concatenate([bz, fz])
    n = x.size
    w = _empty(n)
    w["fixed"][bx.size:] = 1
    w.update(x=x, y=y, z=z, m=np.full(n, 2600.0 * sp ** 3), h=np.full(n, 1.3 * sp))
    w.update(mats=[granular_c2()], params=default_params(g=(0.0, -9.81, 0.0)),
             name=f"c2_column_{bx.size}+{fx.size}fixed", n_mobile=int(bx.size))
    return w


def _cache_path(tag: str) -> str:
    """File under the temporary directory for a generated input, keyed by the
    text of this module (a changed generator never reads an old file)."""
    import hashlib
    import os
    import tempfile
    with open(__file__, "rb") as f:
        key = hashlib.sha256(f.read() + tag.encode()).hexdigest()[:24]
    d = os.path.join(tempfile.gettempdir(), "sph_inputs_cache")
    os.makedirs(d, exist_ok=True)
    return os.path.join(d, f"{key}.npy")


GLASS_PASSES = 16
GLASS_STEP = 0.25


def stratified_ball(n_target: int, radius: float, seed: int, passes: int = GLASS_PASSES):
    """Glass-like points in a ball (a seeded, relaxed random packing): one
    uniform random point per cubic cell of a lattice whose spacing sp gives
    ~n_target points inside the ball, then `passes` relaxation passes in
    which every pair closer than sp pushes its two points apart by
    GLASS_STEP sp (1 - r/sp)^2 along their separation (a damped soft
    repulsion), points leaving the ball being put back on its surface.
    Sixteen passes take the nearest-neighbour distance from >= 0.36 sp
    (median 0.70) to >= 0.71 sp (median 0.87) for a million points.  The
    result is cached on disk (keyed by this module's text and the
    arguments), since the passes take ~20 s for a million points."""
    sp = radius * (4.0 / 3.0 * math.pi / n_target) ** (1.0 / 3.0)
    path = _cache_path(f"ball|{n_target}|{radius!r}|{seed}|{passes}")
    try:
        return np.load(path), sp
    except (OSError, ValueError):
        pass
    nside = int(math.ceil(2 * radius / sp)) + 2
    rng = np.random.Generator(np.random.PCG64(seed))
    c = (np.arange(nside) - nside / 2.0) * sp
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    P = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    P = P + rng.uniform(0.0, sp, size=P.shape)
    P = P[np.einsum("ij,ij->i", P, P) < radius * radius]
    n = P.shape[0]
    from scipy.spatial import cKDTree
    for _ in range(passes):
        pr = cKDTree(P).query_pairs(sp, output_type="ndarray")
        if pr.size == 0:
            break
        d = P[pr[:, 0]] - P[pr[:, 1]]
        r = np.sqrt(np.einsum("ij,ij->i", d, d)) + 1e-12 * sp
        wgt = GLASS_STEP * sp * (1.0 - r / sp) ** 2 / r
        for a in range(3):
            f = wgt * d[:, a]
            P[:, a] += np.bincount(pr[:, 0], f, n) - np.bincount(pr[:, 1], f, n)
        rr = np.sqrt(np.einsum("ij,ij->i", P, P))
        out = rr > radius
        P[out] *= (radius / rr[out])[:, None]
    try:
        tmp = path + ".tmp.npy"
        np.save(tmp, P)
        import os
        os.replace(tmp, path)
    except OSError:
        pass
    return P, sp


def c3_impact(n_target: int = 1_000_000, n_proj: int = 100_000, seed: int = 4) -> dict:
    """Two-sphere impact: granite target of radius 50 km with ~n_target
    particles and a projectile of equal particle mass with ~n_proj particles,
    glass-like arrangement, h = 1.3 spacing; projectile centre at
    (R_t + R_p)(-cos 45, sin 45, 0) from the target centre moving at
    (3000, 0, 0) m/s; u = 0, S = 0, gravity off."""
    Rt = 50.0e3
    mat = granite_c3()
    Pt, sp = stratified_ball(n_target, Rt, seed)
    Rp = Rt * (n_proj / n_target) ** (1.0 / 3.0)
    Pp, _ = stratified_ball(n_proj, Rp, seed + 1000)
    d = (Rt + Rp + 0.5 * sp)
    off = np.array([-d * math.cos(math.radians(45)), d * math.sin(math.radians(45)), 0.0])
    Pp = Pp + off
    P = np.concatenate([Pt, Pp])
    n = P.shape[0]
    w = _empty(n)
    mass = mat["rho0"] * sp ** 3
    w.update(x=P[:, 0].copy(), y=P[:, 1].copy(), z=P[:, 2].copy(), m=np.full(n, mass),
             h=np.full(n, 1.3 * sp))
    w["vx"][Pt.shape[0]:] = 3000.0
    w.update(mats=[mat], params=default_params(), name=f"c3_impact_{Pt.shape[0]}+{Pp.shape[0]}",
             n_target=int(Pt.shape[0]))
    return w


def random_cloud(n: int, seed: int, h_spread: float = 0.0, box: float = 6.0) -> dict:
    """Small random set for parity edge cases: n uniform points in a cube of
    side ``box`` m (mean spacing ~1 m for box^3 ~ n), h = 1.3 m times a factor
    drawn from U(1 - h_spread, 1 + h_spread), random velocity, energy and
    stress of C1 magnitudes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    P = rng.uniform(0.0, box, size=(3, n))
    w = _empty(n)
    hs = 1.3 * (1.0 + h_spread * rng.uniform(-1.0, 1.0, size=n))
    w.update(x=P[0].copy(), y=P[1].copy(), z=P[2].copy(), m=np.full(n, 2700.0), h=hs,
             u=rng.uniform(5e3, 2e4, size=n))
    w["vx"], w["vy"], w["vz"] = rng.normal(0.0, 0.05, size=(3, n))
    w["S"] = rng.normal(0.0, 20.0e6, size=(5, n))
    w.update(mats=[basalt_c1()], params=default_params(), name=f"cloud_{n}_{seed}")
    return w


_PER_PARTICLE = ("x", "y", "z", "vx", "vy", "vz", "u", "m", "h", "mat", "fixed")


def concat_runs(runs: list) -> dict:
    """Several independent workloads in one set of buffers (a batched scan):
    per-particle arrays concatenated run after run, ``run_start`` the n_runs + 1
    offsets.  The runs share the material table and parameters of the first."""
    w = {k: np.concatenate([r[k] for r in runs]) for k in _PER_PARTICLE}
    w["S"] = np.concatenate([r["S"] for r in runs], axis=1)
    w["run_start"] = np.concatenate([[0], np.cumsum([r["x"].size for r in runs])]).astype(np.int64)
    w.update(mats=runs[0]["mats"], params=runs[0]["params"],
             name="+".join(r.get("name", "run") for r in runs))
    return w


G_NEWTON = 6.674e-11


def bcc_ball(n_target: int, radius: float):
    """Body-centred cubic lattice clipped to a ball, spacing chosen so that
    about n_target points fall inside (two points per cubic cell of edge a).
    Returns the points and the mean interparticle spacing (1/n)^(1/3)."""
    a = (2.0 * (4.0 / 3.0) * math.pi * radius ** 3 / n_target) ** (1.0 / 3.0)
    k = int(math.ceil(radius / a)) + 1
    c = np.arange(-k, k + 1) * a
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    corner = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    P = np.concatenate([corner, corner + 0.5 * a])
    P = P[np.einsum("ij,ij->i", P, P) < radius * radius]
    return P, a / 2.0 ** (1.0 / 3.0)


def impact_pair(n_target: int, gamma: float = 0.1, r_c1: float = 1.0e6, v_over_vesc: float = 2.0,
                strength: bool = True, mat_id: int = 0, mat: dict | None = None,
                cm_frame: bool = False) -> dict:
    """Head-on collision of two BCC spheres of one material with equal
    particle masses: target of ~n_target particles and projectile of mass
    ratio gamma = M_p / M_t.  The total mass is that of a sphere of radius
    r_c1 at 1000 kg/m^3; each body's radius is that of its nominal mass at
    the material's reference density.  The target holds exactly M_t; the
    projectile is the BCC lattice clipped to R_p with about gamma times the
    target's count (within a few percent), so its mass and density are
    gamma M_t and rho0 to within as much (the case records the nominal
    masses, which Q_R uses).  The
    projectile starts one spacing from contact on the -x side and moves at
    v = v_over_vesc * v_esc along +x, with v_esc = sqrt(2 G M_tot / (R_t + R_p));
    the target is at rest (with ``cm_frame``, both move so that the total
    momentum is zero).  u = 0, S = 0.  ``strength`` only labels the run (the
    material row at ``mat_id`` decides what the step computes)."""
    mat = mat or granite_c3()
    rho = mat["rho0"]
    m_tot = 4.0 / 3.0 * math.pi * r_c1 ** 3 * 1000.0
    m_t, m_p = m_tot / (1.0 + gamma), m_tot * gamma / (1.0 + gamma)
    r_t = (3.0 * m_t / (4.0 * math.pi * rho)) ** (1.0 / 3.0)
    r_p = (3.0 * m_p / (4.0 * math.pi * rho)) ** (1.0 / 3.0)
    Pt, sp = bcc_ball(n_target, r_t)
    mpart = m_t / Pt.shape[0]
    Pp, _ = bcc_ball(max(int(round(Pt.shape[0] * gamma)), 1), r_p)
    v_esc = math.sqrt(2.0 * G_NEWTON * m_tot / (r_t + r_p))
    Pp = Pp + np.array([-(r_t + r_p + sp), 0.0, 0.0])
    P = np.concatenate([Pt, Pp])
    n = P.shape[0]
    w = _empty(n)
    w.update(x=P[:, 0].copy(), y=P[:, 1].copy(), z=P[:, 2].copy(), m=np.full(n, mpart),
             h=np.full(n, 1.3 * sp))
    w["vx"][Pt.shape[0]:] = v_over_vesc * v_esc
    if cm_frame:
        w["vx"] -= w["vx"].sum() / n
    w["mat"][:] = mat_id
    w.update(mats=[mat], params=default_params(), n_target=int(Pt.shape[0]),
             name=f"impact_{Pt.shape[0]}+{Pp.shape[0]}",
             case=dict(m_tot=m_tot, gamma=gamma, strength=int(strength), v_esc=v_esc,
                       v=v_over_vesc * v_esc, r_t=r_t, r_p=r_p))
    return w


def scan_batch(n_runs: int = 64, seed: int = 5, n_min: int = 20_000, n_max: int = 300_000,
               gamma: float = 0.1, scale: float = 1.0, cm_frame: bool = False) -> dict:
    """A batched Q_RD* scan: n_runs head-on impacts with target particle counts
    log-uniform in [n_min, n_max] (times ``scale`` for small copies), mass
    ratio gamma, R_C1 log-uniform in [4.64e5, 4.64e6] m, v/v_esc log-uniform
    in [1, 10] and strength on or off with probability 1/2.  Material 0 is
    granite with strength, material 1 the same without; runs are concatenated
    (``run_start``) and ``cases`` lists each run's parameters; ``cm_frame``
    puts each run in its centre-of-mass frame."""
    rng = np.random.Generator(np.random.PCG64(seed))
    strong = granite_impact()
    mats = [strong, fluid(strong)]
    runs, cases = [], []
    for _ in range(n_runs):
        nt = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max))) * scale))
        rc1 = math.exp(rng.uniform(math.log(4.64e5), math.log(4.64e6)))
        vv = math.exp(rng.uniform(0.0, math.log(10.0)))
        st = bool(rng.integers(0, 2))
        w = impact_pair(max(nt, 8), gamma, rc1, vv, st, mat_id=0 if st else 1, mat=strong,
                        cm_frame=cm_frame)
        runs.append(w)
        cases.append(w["case"])
    b = concat_runs(runs)
    b["mats"] = mats
    b["cases"] = cases
    b["name"] = f"scan_{n_runs}runs_{b['x'].size}"
    return b
