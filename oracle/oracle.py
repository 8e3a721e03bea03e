"""ctypes wrapper of the FP64 CPU oracle (``oracle/sph_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, by the smoke check and
by the CPU-baseline leg of the benchmark; never by the GPU library or its
Python binding.  It shares no code with them.

Arrays are numpy float64 (int32 material ids, uint8 fixed flags); stress is
component-major ``(5, n)`` with components (xx, yy, xy, xz, yz); tensors are
``(9, n)`` with component index 3a+b.

Each function below forwards to one C routine of the oracle, which states the
passage of the paper it follows.  ``derivs`` chains them in the order the
paper evaluates a step (sec. 2.1 density, sec. 2.3 yield and rescaling,
sec. 2.2 gradients and stress rate, sec. 2.1/2.2 forces) for any subset of
target particles, computing the density only where the targets need it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sph_oracle.c")
_SRC_GRAV = os.path.join(_HERE, "gravity_oracle.c")
# SPH_ORACLE_LIB names another build of the same source to load instead (a
# build with a planted mistake, to check that the pins catch it)
_LIB = os.environ.get("SPH_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FP contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, _SRC_GRAV, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Material(C.Structure):
    _fields_ = [(k, C.c_double) for k in (
        "rho0", "A", "B", "E0", "Eiv", "Ecv", "a", "b", "alpha", "beta",
        "cv", "T_ref", "c_min", "shear_modulus", "nu",
        "Y0", "Ym", "mu_i", "mu_d", "xi", "T_melt")] + [
        ("strength_on", C.c_int32), ("thermal_softening_on", C.c_int32),
        ("tmelt_n", C.c_int32), ("tmelt_pad", C.c_int32),
        ("tmelt_rho", C.c_double * 8), ("tmelt_T", C.c_double * 8),
        ("eos_nrho", C.c_int32), ("eos_nu", C.c_int32)] + [
        (k, C.POINTER(C.c_double)) for k in ("eos_rho", "eos_u", "eos_P", "eos_c", "eos_T")] + [
        ("rho_limit", C.c_double)]


class Params(C.Structure):
    _fields_ = [("av_alpha", C.c_double), ("av_beta", C.c_double), ("av_eps", C.c_double),
                ("eta_C", C.c_double), ("rot_sign", C.c_double),
                ("g", C.c_double * 3), ("box", C.c_double * 3),
                ("use_correction", C.c_int32), ("omega_one", C.c_int32),
                ("adapt_ngb", C.c_double), ("adapt_skin", C.c_double),
                ("eta_a", C.c_double), ("rungs", C.c_int32), ("rungs_pad", C.c_int32)]


class _State(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(k, C.POINTER(C.c_double)) for k in (
        "x", "y", "z", "vx", "vy", "vz", "u", "S", "ax", "ay", "az", "dudt", "dS",
        "eps2", "m", "h")] + [
        ("mat", C.POINTER(C.c_int32)), ("fixed", C.POINTER(C.c_uint8))] + [
        (k, C.POINTER(C.c_double)) for k in (
            "rho", "omega", "P", "cs", "T", "Y", "Gam", "G", "dt_i")] + [
        ("dt", C.c_double), ("n_singular", C.c_int64), ("pairs", C.c_int64),
        ("dtp", C.POINTER(C.c_int64)), ("el", C.POINTER(C.c_int64)),
        ("ticks", C.c_int64), ("tick", C.c_double), ("n_clamped", C.c_int64),
        ("time", C.c_double)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build(force=False)
            _lib = C.CDLL(_LIB)
            _declare(_lib)
    return _lib


_D = C.POINTER(C.c_double)
_I64 = C.POINTER(C.c_int64)
_I32 = C.POINTER(C.c_int32)
_U8 = C.POINTER(C.c_uint8)


def _declare(L):
    L.or_W.restype = C.c_double
    L.or_K.restype = C.c_double
    L.or_dWdh.restype = C.c_double
    for f in (L.or_W, L.or_K, L.or_dWdh):
        f.argtypes = [C.c_double, C.c_double]
    L.or_J2.restype = C.c_double
    L.or_J2.argtypes = [_D]
    L.or_yield.restype = C.c_double
    L.or_yield.argtypes = [C.POINTER(Material), C.c_double, C.c_double, C.c_double]
    L.or_rung_step.restype = C.c_int64
    L.or_rung_step.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_int64, C.c_int64,
                               C.POINTER(C.c_int64)]
    L.or_shear_modulus.restype = C.c_double
    L.or_shear_modulus.argtypes = [C.POINTER(Material), C.c_double, C.c_double]


def _p(a, t=_D):
    return a.ctypes.data_as(t) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- structures
def _eos_arrays(tab):
    """Contiguous float64 copies of a tabulated EOS: dict with node vectors
    ``rho`` (n_rho), ``u`` (n_u) and value grids ``P``, ``c``, ``T``
    (n_rho x n_u)."""
    r, u = _f64(tab["rho"]).ravel(), _f64(tab["u"]).ravel()
    vals = [_f64(tab[k]).reshape(r.size, u.size) for k in ("P", "c", "T")]
    return [r, u] + vals


def material(d: dict) -> Material:
    """Material block.  With an ``eos_table`` entry (a dict, treated as
    immutable) the block points into float64 copies of the table that this
    module keeps for the life of the process."""
    m = Material()
    for k, _ in Material._fields_:
        if k.startswith("tmelt_") or k.startswith("eos_") or k == "rho_limit":
            continue
        setattr(m, k, d[k])
    m.rho_limit = float(d.get("rho_limit", 0.0))
    tab = d.get("eos_table")
    if tab is not None:
        hit = _EOS_KEEP.get(id(tab))
        if hit is None or hit[0] is not tab:
            hit = (tab, _eos_arrays(tab))
            _EOS_KEEP[id(tab)] = hit
        arrs = hit[1]
        m.eos_nrho, m.eos_nu = arrs[0].size, arrs[1].size
        for k, a in zip(("eos_rho", "eos_u", "eos_P", "eos_c", "eos_T"), arrs):
            setattr(m, k, _p(a))
    tab_r, tab_t = d.get("tmelt_rho"), d.get("tmelt_T")
    if tab_r is not None:
        assert len(tab_r) == len(tab_t) <= 8
        m.tmelt_n = len(tab_r)
        for k, (r, t) in enumerate(zip(tab_r, tab_t)):
            m.tmelt_rho[k], m.tmelt_T[k] = r, t
    return m


# tables referenced by Material blocks (keyed by the table dict; small)
_EOS_KEEP = {}


def materials(lst) -> C.Array:
    arr = (Material * len(lst))()
    for i, d in enumerate(lst):
        arr[i] = material(d)
    return arr


def params(d: dict) -> Params:
    p = Params()
    p.av_alpha, p.av_beta, p.av_eps = d["av_alpha"], d["av_beta"], d["av_eps"]
    p.eta_C, p.rot_sign = d["eta_C"], d["rot_sign"]
    for k in range(3):
        p.g[k] = d["g"][k]
        p.box[k] = d.get("box", (0.0, 0.0, 0.0))[k]
    p.use_correction = int(d["use_correction"])
    p.omega_one = int(d.get("omega_one", 0))
    p.adapt_ngb = float(d.get("adapt_ngb", 0.0))
    p.adapt_skin = float(d.get("adapt_skin", 1.25))
    p.eta_a = float(d.get("eta_a", 0.0))
    p.rungs = int(d.get("rungs", 0))
    return p


# ------------------------------------------------------------------ kernels
def kernel(r, h):
    """Return (W, K, dW/dh) of the Wendland C2 kernel at arrays r, h."""
    r, h = np.broadcast_arrays(_f64(r), _f64(h))
    r, h = _f64(r), _f64(h)
    n = r.size
    W, K, D = np.empty(n), np.empty(n), np.empty(n)
    lib().or_kernel_arr(C.c_int64(n), _p(r), _p(h), _p(W), _p(K), _p(D))
    return W.reshape(r.shape), K.reshape(r.shape), D.reshape(r.shape)


def tillotson(mat: dict, rho, u):
    """Return (P, c, dP/drho, dP/du) of the Tillotson EOS."""
    rho, u = np.broadcast_arrays(_f64(rho), _f64(u))
    rho, u = _f64(rho), _f64(u)
    n = rho.size
    P, c, dr, du = (np.empty(n) for _ in range(4))
    m = material(mat)
    lib().or_tillotson_arr(C.byref(m), C.c_int64(n), _p(rho), _p(u), _p(P), _p(c), _p(dr), _p(du))
    return P, c, dr, du


def eos(mat: dict, rho, u):
    """Return (P, c, T) of the material's EOS: its table when it has one,
    otherwise Tillotson with T = T_ref + u / cv."""
    rho, u = np.broadcast_arrays(_f64(rho), _f64(u))
    rho, u = _f64(rho), _f64(u)
    n = rho.size
    P, c, T = (np.empty(n) for _ in range(3))
    m = material(mat)
    lib().or_eos_arr(C.byref(m), C.c_int64(n), _p(rho), _p(u), _p(P), _p(c), _p(T))
    return P.reshape(rho.shape), c.reshape(rho.shape), T.reshape(rho.shape)


def yield_strength(mat: dict, P, T, rho=None):
    """Yield strength at pressure P, temperature T and density rho (rho only
    matters for a tabulated melting temperature; default rho0)."""
    P, T = np.broadcast_arrays(_f64(P), _f64(T))
    P, T = _f64(P), _f64(T)
    R = None if rho is None else _f64(np.broadcast_to(_f64(rho), P.shape))
    Y = np.empty(P.size)
    m = material(mat)
    lib().or_yield_arr(C.byref(m), C.c_int64(P.size), _p(R), _p(P), _p(T), _p(Y))
    return Y


def rung_step(rungs: int, tick: float, d: float, t: int, cur: int):
    """Individual step of a particle in ticks (reading T1): returns
    (step, clamped)."""
    k = C.c_int64(0)
    v = lib().or_rung_step(rungs, tick, d, t, cur, C.byref(k))
    return int(v), int(k.value)


def shear_modulus(mat: dict, rho: float, c: float) -> float:
    m = material(mat)
    return lib().or_shear_modulus(C.byref(m), rho, c)


def J2(s5) -> float:
    s5 = _f64(s5)
    return lib().or_J2(_p(s5))


def plastic_return_rows(S_rows, Y):
    """S_rows (n,5) entry-major; returns rescaled copy."""
    S = _f64(S_rows).copy()
    Y = _f64(Y)
    lib().or_plastic_return_rows(C.c_int64(S.shape[0]), _p(S), _p(Y))
    return S


def stress_rate_rows(G_rows, S_rows, Gam, rot_sign=1.0, printed=False):
    """G_rows (n,9), S_rows (n,5) entry-major; returns (dS (n,5), eps2 rate (n,))."""
    G, S, Gm = _f64(G_rows), _f64(S_rows), _f64(np.broadcast_to(Gam, (len(G_rows),)))
    n = G.shape[0]
    dS = np.empty((n, 5))
    e2 = np.empty(n)
    lib().or_stress_rate_rows(C.c_int64(n), _p(G), _p(S), _p(Gm), C.c_double(rot_sign),
                              C.c_int32(1 if printed else 0), _p(dS), _p(e2))
    return dS, e2


def predict(y, dy, dt, fixed=None):
    """y + dt/2 dy for non-fixed particles; y, dy of shape (ncomp, n) or (n,)."""
    y2, dy2 = np.atleast_2d(_f64(y)), np.atleast_2d(_f64(dy))
    nc, n = y2.shape
    out = np.empty_like(y2)
    fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
    lib().or_predict(C.c_int64(n), C.c_int32(nc), _p(fx, _U8), C.c_double(dt),
                     _p(y2), _p(dy2), _p(out))
    return out.reshape(np.shape(y))


# --------------------------------------------------------------- pair sweeps
def _targets(n, targets):
    if targets is None:
        return np.arange(n, dtype=np.int64)
    return np.ascontiguousarray(targets, dtype=np.int64)


def pair_counts(x, y, z, h, prm: dict, targets=None):
    """|N_i| for the targets by brute force (one sweep over all particles
    per target)."""
    x, y, z, h = map(_f64, (x, y, z, h))
    n = x.size
    tar = _targets(n, targets)
    p = params(prm)
    cnt = np.empty(tar.size, dtype=np.int64)
    lib().or_pair_counts(C.c_int64(n), _p(x), _p(y), _p(z), _p(h), C.byref(p),
                         C.c_int64(tar.size), _p(tar, _I64), _p(cnt, _I64))
    return cnt


def pair_lists(x, y, z, h, prm: dict, targets=None):
    """Brute-force pair sets N_i (ascending j) for the targets.

    Returns (offsets (nt+1,), nbr (int64), dflag (uint8))."""
    x, y, z, h = map(_f64, (x, y, z, h))
    n = x.size
    tar = _targets(n, targets)
    p = params(prm)
    cnt = np.empty(tar.size, dtype=np.int64)
    L = lib()
    L.or_pair_counts(C.c_int64(n), _p(x), _p(y), _p(z), _p(h), C.byref(p),
                     C.c_int64(tar.size), _p(tar, _I64), _p(cnt, _I64))
    off = np.zeros(tar.size + 1, dtype=np.int64)
    np.cumsum(cnt, out=off[1:])
    nbr = np.empty(int(off[-1]), dtype=np.int64)
    dfl = np.empty(int(off[-1]), dtype=np.uint8)
    L.or_pair_lists(C.c_int64(n), _p(x), _p(y), _p(z), _p(h), C.byref(p),
                    C.c_int64(tar.size), _p(tar, _I64), _p(off, _I64), _p(nbr, _I64), _p(dfl, _U8))
    return off, nbr, dfl


def density(x, y, z, m, h, prm: dict, targets=None, out=None):
    x, y, z, m, h = map(_f64, (x, y, z, m, h))
    n = x.size
    tar = _targets(n, targets)
    rho, om = (np.full(n, np.nan), np.full(n, np.nan)) if out is None else out
    p = params(prm)
    lib().or_density(C.c_int64(n), _p(x), _p(y), _p(z), _p(m), _p(h), C.byref(p),
                     C.c_int64(tar.size), _p(tar, _I64), _p(rho), _p(om))
    return rho, om


def state(rho, u, mat_id, mats: list, targets=None, out=None):
    """EOS, temperature, yield and shear modulus: returns (P, c, T, Y, Gamma)."""
    rho, u = _f64(rho), _f64(u)
    n = rho.size
    tar = _targets(n, targets)
    mid = np.ascontiguousarray(mat_id, dtype=np.int32)
    outs = tuple(np.full(n, np.nan) for _ in range(5)) if out is None else out
    arr = materials(mats)
    lib().or_state(C.c_int64(tar.size), _p(tar, _I64), _p(rho), _p(u), _p(mid, _I32), arr,
                   *[_p(o) for o in outs])
    return outs


def plastic_return(S, Y, targets=None):
    """Rescale component-major S (5,n) in a copy."""
    S = _f64(S).copy()
    n = S.shape[1]
    tar = _targets(n, targets)
    lib().or_plastic_return_all(C.c_int64(n), C.c_int64(tar.size), _p(tar, _I64), _p(S), _p(_f64(Y)))
    return S


def gradients(x, y, z, vx, vy, vz, m, h, rho, omega, prm: dict, targets=None,
              want_parts=False):
    """Corrected velocity gradient G (9,n); optionally also C^-1 and F."""
    arrs = list(map(_f64, (x, y, z, vx, vy, vz, m, h, rho, omega)))
    n = arrs[0].size
    tar = _targets(n, targets)
    G = np.full((9, n), np.nan)
    Ci = np.full((9, n), np.nan) if want_parts else None
    F = np.full((9, n), np.nan) if want_parts else None
    ns = C.c_int64(0)
    p = params(prm)
    lib().or_gradients(C.c_int64(n), *[_p(a) for a in arrs], C.byref(p),
                       C.c_int64(tar.size), _p(tar, _I64), _p(G), _p(Ci), _p(F), C.byref(ns))
    if want_parts:
        return G, Ci, F, ns.value
    return G, ns.value


def stress_rate(G, S, Gam, rot_sign, targets=None):
    G, S, Gam = _f64(G), _f64(S), _f64(Gam)
    n = G.shape[1]
    tar = _targets(n, targets)
    dS = np.full((5, n), np.nan)
    e2 = np.full(n, np.nan)
    lib().or_stress_rate(C.c_int64(n), C.c_int64(tar.size), _p(tar, _I64), _p(G), _p(S),
                         _p(Gam), C.c_double(rot_sign), _p(dS), _p(e2))
    return dS, e2


def forces(x, y, z, vx, vy, vz, m, h, rho, omega, P, cs, S, prm: dict, targets=None):
    """Returns (a (3,n), du/dt (n,), dt_CFL (n,))."""
    arrs = list(map(_f64, (x, y, z, vx, vy, vz, m, h, rho, omega, P, cs)))
    S = _f64(S)
    n = arrs[0].size
    tar = _targets(n, targets)
    a = np.full((3, n), np.nan)
    du = np.full(n, np.nan)
    dt = np.full(n, np.nan)
    p = params(prm)
    lib().or_forces(C.c_int64(n), *[_p(v) for v in arrs], _p(S), C.byref(p),
                    C.c_int64(tar.size), _p(tar, _I64), _p(a[0]), _p(a[1]), _p(a[2]),
                    _p(du), _p(dt))
    return a, du, dt


def term_scales(x, y, z, vx, vy, vz, m, h, rho, omega, P, cs, S, Gam, prm: dict,
                targets=None):
    """Per-particle scales of the pair sums (sum over the pair set of the
    magnitude of each pair's contribution): returns dict a, dudt, G, dS of
    (n,) arrays (NaN where not computed).  S is the rescaled predicted stress
    the passes use; Gam the shear modulus."""
    arrs = list(map(_f64, (x, y, z, vx, vy, vz, m, h, rho, omega, P, cs)))
    S, Gam = _f64(S), _f64(Gam)
    n = arrs[0].size
    tar = _targets(n, targets)
    out = {k: np.full(n, np.nan) for k in ("a", "dudt", "G", "dS")}
    p = params(prm)
    lib().or_term_scales(C.c_int64(n), *[_p(v) for v in arrs], _p(S), _p(Gam), C.byref(p),
                         C.c_int64(tar.size), _p(tar, _I64), _p(out["a"]), _p(out["dudt"]),
                         _p(out["G"]), _p(out["dS"]))
    return out


def closure(x, y, z, h, prm: dict, targets):
    """Targets together with every member of their pair sets (sorted)."""
    off, nbr, _ = pair_lists(x, y, z, h, prm, targets)
    return np.unique(np.concatenate([np.asarray(targets, dtype=np.int64), nbr]))


def derivs(st: dict, mats: list, prm: dict, targets=None, scales=False):
    """One derivative evaluation of the strength-SPH step.

    ``st`` holds x, y, z, m, h, mat, the predicted velocity vx, vy, vz, the
    predicted energy u and the predicted (not yet rescaled) stress S (5,n).
    The density, EOS, yield and rescaling run on the targets and their pair
    sets; gradients, stress rate and forces on the targets.  Returns a dict of
    full-length arrays (NaN where not computed); with ``scales`` also
    ``scale``, the per-particle scales of the pair sums (``term_scales``).
    """
    x, y, z, h = st["x"], st["y"], st["z"], st["h"]
    n = np.asarray(x).size
    tar = _targets(n, targets)
    near = tar if targets is None else closure(x, y, z, h, prm, tar)
    rho, om = density(x, y, z, st["m"], h, prm, near)
    P, c, T, Y, Gam = state(rho, st["u"], st["mat"], mats, near)
    Sp = plastic_return(st["S"], Y, near)
    G, nsing = gradients(x, y, z, st["vx"], st["vy"], st["vz"], st["m"], h, rho, om, prm, tar)
    dS, e2 = stress_rate(G, Sp, Gam, prm["rot_sign"], tar)
    a, du, dt = forces(x, y, z, st["vx"], st["vy"], st["vz"], st["m"], h, rho, om, P, c, Sp,
                       prm, tar)
    out = dict(rho=rho, omega=om, P=P, c=c, T=T, Y=Y, Gam=Gam, S_pred=Sp, G=G, dS=dS,
               eps2_rate=e2, a=a, dudt=du, dt=dt, n_singular=nsing, targets=tar)
    if scales:
        out["scale"] = term_scales(x, y, z, st["vx"], st["vy"], st["vz"], st["m"], h, rho, om,
                                   P, c, Sp, Gam, prm, tar)
    return out


class Integrator:
    """Multi-step FP64 integration of a particle set (kick-drift-kick with the
    predictor of the paper's sec. 2.4), for tests that follow a state in time.
    With ``prm["rungs"] > 0`` each ``step`` is one substep of the individual
    steps to the next end of a particle's step, and ``dt_fixed`` is the base
    step."""

    _FIELDS = ("rho", "omega", "P", "cs", "T", "Y", "Gam", "dt_i")

    def __init__(self, st: dict, mats: list, prm: dict, dt_fixed: float = 0.0):
        n = np.asarray(st["x"]).size
        self.n = n
        self.arr = {k: _f64(st[k]).copy() for k in ("x", "y", "z", "vx", "vy", "vz", "u")}
        self.arr["S"] = _f64(st["S"]).copy()
        self.arr["m"] = _f64(st["m"]).copy()
        self.arr["h"] = _f64(st["h"]).copy()
        for k in ("ax", "ay", "az", "dudt", "eps2"):
            self.arr[k] = np.zeros(n)
        self.arr["dS"] = np.zeros((5, n))
        self.arr["G"] = np.zeros((9, n))
        for k in self._FIELDS:
            self.arr[k] = np.zeros(n)
        self.mat = np.ascontiguousarray(st["mat"], dtype=np.int32)
        self.fixed = np.ascontiguousarray(st.get("fixed", np.zeros(n)), dtype=np.uint8)
        self._mats = materials(mats)
        self._prm = params(prm)
        self.dt_fixed = float(dt_fixed)
        s = _State()
        s.n = n
        for k in ("x", "y", "z", "vx", "vy", "vz", "u", "S", "ax", "ay", "az", "dudt", "dS",
                  "eps2", "m", "h", "G"):
            setattr(s, k, _p(self.arr[k]))
        for k in self._FIELDS:
            setattr(s, k, _p(self.arr[k]))
        s.mat = _p(self.mat, _I32)
        s.fixed = _p(self.fixed, _U8)
        self.arr["dtp"] = np.zeros(n, dtype=np.int64)   # ticks (individual steps)
        self.arr["el"] = np.zeros(n, dtype=np.int64)
        s.dtp = _p(self.arr["dtp"], _I64)
        s.el = _p(self.arr["el"], _I64)
        self._s = s
        lib().or_init(C.byref(s), self._mats, C.byref(self._prm), C.c_double(self.dt_fixed))

    @property
    def dt(self):
        return self._s.dt

    @property
    def pairs(self):
        return self._s.pairs

    @property
    def time(self):
        return self._s.time

    @property
    def ticks(self):
        return self._s.ticks

    @property
    def tick(self):
        return self._s.tick

    @property
    def n_clamped(self):
        return self._s.n_clamped

    def step(self, k: int = 1):
        for _ in range(k):
            lib().or_step(C.byref(self._s), self._mats, C.byref(self._prm),
                          C.c_double(self.dt_fixed))

    def __getitem__(self, k):
        return self.arr[k]


# ------------------------------------------------- self-gravity, bound mass
def _runs(n, run_start):
    if run_start is None:
        return 1, None
    rs = np.ascontiguousarray(run_start, dtype=np.int64)
    return len(rs) - 1, rs


def gravity(x, y, z, m, G, eps, active=None, run_start=None):
    """Direct-sum softened gravity (gravity_oracle.c, reading G1).
    Returns (ax, ay, az, phi)."""
    L = lib()
    x, y, z, m = _f64(x), _f64(y), _f64(z), _f64(m)
    n = x.size
    nr, rs = _runs(n, run_start)
    act = None if active is None else np.ascontiguousarray(active, dtype=np.int32)
    out = [np.zeros(n) for _ in range(4)]
    L.or_gravity(C.c_int64(n), _p(x), _p(y), _p(z), _p(m), _p(act, _I32), C.c_int32(nr),
                 _p(rs, _I64), C.c_double(G), C.c_double(eps), *[_p(o) for o in out])
    return tuple(out)


def bound_mass(x, y, z, vx, vy, vz, m, G, eps, run_start=None, max_iter=100):
    """Iterative removal of unbound particles per run (reading G2).
    Returns (bound flags int32, bound mass per run)."""
    L = lib()
    arrs = [_f64(a) for a in (x, y, z, vx, vy, vz, m)]
    n = arrs[0].size
    nr, rs = _runs(n, run_start)
    bound = np.zeros(n, dtype=np.int32)
    mb = np.zeros(nr)
    L.or_bound_mass.restype = C.c_int32
    L.or_bound_mass(C.c_int64(n), *[_p(a) for a in arrs], C.c_int32(nr), _p(rs, _I64),
                    C.c_double(G), C.c_double(eps), C.c_int32(max_iter), _p(bound, _I32),
                    _p(mb))
    return bound, mb


# ------------------------------------------------ adaptive smoothing length
def adapt_h(x, y, z, m, h, prm: dict, n_ngb: float, tol=1e-12, max_iter=50, h_cap=None,
            fixed=None):
    """Newton-Raphson smoothing lengths at constant kernel mass (reading H1),
    optionally capped per particle.  Returns (h, largest number of steps)."""
    L = lib()
    x, y, z, m, h = (_f64(a) for a in (x, y, z, m, h))
    cap = None if h_cap is None else _f64(h_cap)
    fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
    out = np.zeros_like(h)
    p = params(prm)
    L.or_adapt_h.restype = C.c_int32
    it = L.or_adapt_h(C.c_int64(x.size), _p(x), _p(y), _p(z), _p(m), _p(h), _p(cap),
                      _p(fx, _U8), C.byref(p), C.c_double(n_ngb), C.c_double(tol),
                      C.c_int32(max_iter), _p(out))
    return out, int(it)
