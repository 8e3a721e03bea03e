"""Python binding of the gfx950 strength-SPH library (``libsph.so``).

Argument marshalling only: every function forwards to the C entry point of
the same name declared in ``include/sph.h``; all arithmetic runs in the HIP
kernels.  Arrays are torch tensors on the GPU (float64 unless stated);
PyTorch is used for device memory and streams, nothing else.  Importing
this module fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsph.so")

SPH_OK, SPH_EINVAL, SPH_EHIP, SPH_ENOMEM, SPH_ECAPACITY, SPH_ENONFINITE, SPH_ESTATE = range(7)
SPH_FP64, SPH_FP32_CELLREL = 0, 1
SPH_STRESS_PREDICT, SPH_STRESS_RATE, SPH_STRESS_KICK, SPH_STRESS_OPEN = 1, 2, 4, 8
SPH_KD_DRIFT, SPH_KD_PREDICT, SPH_KD_KICK, SPH_KD_OPEN = 1, 2, 4, 8

# rows of the state buffers (must match include/sph.h)
SPH_X, SPH_Y, SPH_Z, SPH_VX, SPH_VY, SPH_VZ, SPH_U = range(7)
SPH_S, SPH_AX, SPH_AY, SPH_AZ, SPH_DUDT, SPH_SDOT, SPH_M, SPH_H, SPH_EPS2 = (
    7, 12, 13, 14, 15, 16, 21, 22, 23)
SPH_DTP, SPH_EL, SPH_NF64 = 24, 25, 26
SPH_MAT, SPH_ID, SPH_FIXED, SPH_RUN, SPH_NI32 = range(5)
(SPH_W_RHO, SPH_W_OMEGA, SPH_W_P, SPH_W_CS, SPH_W_T, SPH_W_Y, SPH_W_GMOD) = range(7)
SPH_W_VP, SPH_W_UP, SPH_W_SP, SPH_W_G, SPH_W_DT, SPH_W_PERM = 7, 10, 11, 16, 25, 26
SPH_W_TAU, SPH_W_ACT, SPH_NW = 27, 28, 29
SPH_T_BUILD, SPH_T_DENSITY, SPH_T_GRADIENTS, SPH_T_FORCES = range(4)
(SPH_TUNE_LANES_DENSITY, SPH_TUNE_LANES_GRADIENTS, SPH_TUNE_LANES_FORCES, SPH_TUNE_LANES_STEP,
 SPH_TUNE_CELL_SCALE, SPH_TUNE_BUILD_RANGE, SPH_TUNE_SWEEP_DEPTH, SPH_TUNE_BUILD_TILE) = range(8)


class SphError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sph status {code}: {msg}")
        self.code = code


class sph_material(C.Structure):
    _fields_ = [(k, C.c_double) for k in (
        "rho0", "A", "B", "E0", "Eiv", "Ecv", "a", "b", "alpha", "beta",
        "cv", "T_ref", "c_min", "shear_modulus", "nu",
        "Y0", "Ym", "mu_i", "mu_d", "xi", "T_melt")] + [
        ("strength_on", C.c_int32), ("thermal_softening_on", C.c_int32),
        ("tmelt_n", C.c_int32), ("tmelt_pad", C.c_int32),
        ("tmelt_rho", C.c_double * 8), ("tmelt_T", C.c_double * 8),
        ("eos_nrho", C.c_int32), ("eos_nu", C.c_int32)] + [
        (k, C.c_void_p) for k in ("eos_rho", "eos_u", "eos_P", "eos_c", "eos_T")] + [
        ("rho_limit", C.c_double)]


class sph_params(C.Structure):
    _fields_ = [("av_alpha", C.c_double), ("av_beta", C.c_double), ("av_eps", C.c_double),
                ("eta_C", C.c_double), ("rot_sign", C.c_double), ("g", C.c_double * 3),
                ("use_correction_tensor", C.c_int32), ("omega_one", C.c_int32),
                ("grav_G", C.c_double), ("grav_eps_over_h", C.c_double),
                ("grav_theta", C.c_double), ("adapt_ngb", C.c_double),
                ("adapt_skin", C.c_double), ("eta_a", C.c_double), ("rungs", C.c_int32),
                ("rungs_pad", C.c_int32), ("far_factor", C.c_double)]


class sph_state(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_cap", C.c_int64),
                ("f64", C.c_void_p * 2), ("i32", C.c_void_p * 2), ("work", C.c_void_p),
                ("dt", C.c_void_p), ("dt_next", C.c_void_p), ("n_singular", C.c_void_p),
                ("cur", C.c_int32), ("n_runs", C.c_int32), ("run_start", C.c_void_p),
                ("cell_min", C.c_double), ("dt_max", C.c_double), ("clock", C.c_void_p),
                ("time", C.c_void_p)]


_lib = None
_P = C.c_void_p


def lib():
    """Load ``libsph.so``; raises if it is missing (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        i32, i64, dbl = C.c_int32, C.c_int64, C.c_double
        sig = {
            "sph_create": [C.POINTER(_P), i64, i32, i64, i32, i32],
            "sph_destroy": [_P],
            "sph_sync_status": [_P, _P],
            "sph_build_cells": [_P, i64, _P, _P, _P, _P, i32, _P, dbl, _P, _P],
            "sph_reorder": [_P, i64, _P, i32, _P, _P, _P, _P, _P],
            "sph_neighbors_csr": [_P, _P, _P, _P, _P],
            "sph_pair_count": [_P, _P, _P],
            "sph_timing": [_P, i32],
            "sph_timing_read": [_P, i32, C.POINTER(dbl), C.POINTER(i64)],
            "sph_set_tuning": [_P, i32, i32, i32],
            "sph_gravity": [_P, i64, _P, _P, dbl, dbl, dbl, i32, _P, _P, _P, _P, _P],
            "sph_adapt_h": [_P, i64, _P, _P, dbl, dbl, i32, _P, _P, _P, _P],
            "sph_bound_mass": [_P, i64, _P, _P, _P, _P, dbl, dbl, dbl, i32, _P, _P, _P,
                               C.POINTER(i32), _P],
            "sph_get_tuning": [_P, i32, i32, C.POINTER(i32)],
            "sph_density": [_P, i64, _P, _P, _P, _P, C.POINTER(sph_material), i32,
                            C.POINTER(sph_params), i32] + [_P] * 8,
            "sph_gradients": [_P, i64] + [_P] * 7 + [C.POINTER(sph_params), i32, _P, _P, _P],
            "sph_stress_update": [_P, i32, i64] + [_P] * 6 + [C.POINTER(sph_params)] + [_P] * 5,
            "sph_forces_stress": [_P, i64] + [_P] * 10 + [C.POINTER(sph_params), i32] + [_P] * 6,
            "sph_kick_drift": [_P, i32, i64] + [_P] * 19,
            "sph_dt_min": [_P, i64, _P, _P, _P, _P],
            "sph_diagnostics": [_P, i64] + [_P] * 13,
            "sph_diagnostics_noalloc": [i64] + [_P] * 13,
            "sph_init": [_P, C.POINTER(sph_state), C.POINTER(sph_material), i32,
                         C.POINTER(sph_params), i32, _P],
            "sph_step": [_P, C.POINTER(sph_state), C.POINTER(sph_material), i32,
                         C.POINTER(sph_params), i32, _P],
        }
        sig.update({
            "sph_mlp_forward": [i32, _P, _P, _P, _P, _P, _P],
            "sph_mlp_backward": [i32, _P, _P, _P, _P, _P, _P, _P, _P, _P],
            "sph_mlp_adam": [_P, _P, _P, _P, i32, C.c_float, C.c_float, C.c_float, C.c_float, _P],
            "sph_mlp_loss": [i32, _P, _P, _P, _P],
        })
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.sph_mlp_num_params.argtypes = []
        L.sph_mlp_num_params.restype = C.c_int32
        L.sph_last_error.argtypes = [_P]
        L.sph_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return t.data_ptr()


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


# device copies of tabulated EOS, keyed by the table dict (kept for the life
# of the process: tables are small and their pointers go into kernels)
_EOS_DEVICE = {}


def device_eos_table(tab: dict):
    """Device float64 copies (rho, u, P, c, T) of a tabulated EOS given as a
    dict of node vectors ``rho`` (n_rho), ``u`` (n_u) and value grids ``P``,
    ``c``, ``T`` (n_rho x n_u).  The dict is treated as immutable: the copy
    is made once per dict and kept."""
    hit = _EOS_DEVICE.get(id(tab))
    if hit is None or hit[0] is not tab:
        r = np.ascontiguousarray(tab["rho"], dtype=np.float64).ravel()
        u = np.ascontiguousarray(tab["u"], dtype=np.float64).ravel()
        grids = [np.ascontiguousarray(tab[k], dtype=np.float64).reshape(r.size, u.size)
                 for k in ("P", "c", "T")]
        dev = tuple(torch.from_numpy(a.copy()).to("cuda") for a in [r, u] + grids)
        hit = (tab, dev)
        _EOS_DEVICE[id(tab)] = hit
    return hit[1]


def make_material(d: dict) -> sph_material:
    """Material block from a dict; optional ``tmelt_rho`` / ``tmelt_T`` (up to
    8 nodes, ascending density) give a tabulated melting temperature, and an
    optional ``eos_table`` (see ``device_eos_table``) a tabulated EOS."""
    m = sph_material()
    for k, _ in sph_material._fields_:
        if k.startswith("tmelt_") or k.startswith("eos_") or k == "rho_limit":
            continue
        setattr(m, k, d[k])
    m.rho_limit = float(d.get("rho_limit", 0.0))
    tab = d.get("eos_table")
    if tab is not None:
        dev = device_eos_table(tab)
        m.eos_nrho, m.eos_nu = dev[0].numel(), dev[1].numel()
        for k, t in zip(("eos_rho", "eos_u", "eos_P", "eos_c", "eos_T"), dev):
            setattr(m, k, t.data_ptr())
    tab_r, tab_t = d.get("tmelt_rho"), d.get("tmelt_T")
    if tab_r is not None:
        if len(tab_r) != len(tab_t) or len(tab_r) > 8:
            raise ValueError("tmelt_rho and tmelt_T must have the same length, at most 8")
        m.tmelt_n = len(tab_r)
        for k, (r, t) in enumerate(zip(tab_r, tab_t)):
            m.tmelt_rho[k], m.tmelt_T[k] = r, t
    return m


def make_materials(lst):
    arr = (sph_material * len(lst))()
    for i, d in enumerate(lst):
        arr[i] = make_material(d)
    return arr


def make_params(d: dict) -> sph_params:
    p = sph_params()
    p.av_alpha, p.av_beta, p.av_eps = d["av_alpha"], d["av_beta"], d["av_eps"]
    p.eta_C, p.rot_sign = d["eta_C"], d["rot_sign"]
    for k in range(3):
        p.g[k] = d["g"][k]
    p.use_correction_tensor = int(d["use_correction"])
    p.omega_one = int(d.get("omega_one", 0))
    p.grav_G = float(d.get("grav_G", 0.0))
    p.grav_eps_over_h = float(d.get("grav_eps_over_h", 0.5))
    p.grav_theta = float(d.get("grav_theta", 0.6))
    p.adapt_ngb = float(d.get("adapt_ngb", 0.0))
    p.adapt_skin = float(d.get("adapt_skin", 1.25))
    p.eta_a = float(d.get("eta_a", 0.0))
    p.rungs = int(d.get("rungs", 0))
    p.far_factor = float(d.get("far_factor", 0.0))
    return p


class Context:
    """Owner of an ``sph_ctx`` (internal scratch of the library)."""

    def __init__(self, capacity: int, max_neighbors: int = 128, max_cells: int = 1 << 23,
                 max_runs: int = 1, device: int = 0):
        self.h = _P()
        self.capacity = int(capacity)
        code = lib().sph_create(C.byref(self.h), int(capacity), int(max_neighbors),
                                int(max_cells), int(max_runs), int(device))
        if code != SPH_OK:
            raise SphError(code, "sph_create failed")
        self.max_neighbors = max_neighbors

    def close(self):
        if self.h:
            lib().sph_destroy(self.h)
            self.h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:  # pragma: no cover
            pass

    def check(self, code):
        if code != SPH_OK:
            raise SphError(code, (lib().sph_last_error(self.h) or b"").decode())


# ------------------------------------------------------- C entry points
def sph_build_cells(ctx: Context, x, y, z, h, perm_out, run_start=None, cell_min=0.0,
                    stream=None):
    n = x.numel()
    rs, nr = None, 1
    if run_start is not None:
        arr = (C.c_int64 * len(run_start))(*[int(v) for v in run_start])
        rs, nr = C.cast(arr, _P), len(run_start) - 1
    ctx.check(lib().sph_build_cells(ctx.h, n, _ptr(x), _ptr(y), _ptr(z), _ptr(h), nr, rs,
                                    float(cell_min), _ptr(perm_out), _stream(stream)))


def sph_reorder(ctx: Context, perm, src: list, dst: list, stream=None):
    n = perm.numel()
    nf = len(src)
    sp = (_P * nf)(*[_ptr(t) for t in src])
    dp = (_P * nf)(*[_ptr(t) for t in dst])
    eb = (C.c_int32 * nf)(*[t.element_size() for t in src])
    rows = (C.c_int32 * nf)(*[t.numel() // n if n else 1 for t in src])
    ctx.check(lib().sph_reorder(ctx.h, n, _ptr(perm), nf, sp, dp, eb, rows, _stream(stream)))


def sph_neighbors_csr(ctx: Context, n: int, stream=None):
    """Returns (offsets int64 (n+1,), nbr int32, dflag uint8) on the device."""
    off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    ctx.check(lib().sph_neighbors_csr(ctx.h, _ptr(off), None, None, _stream(stream)))
    tot = int(off[-1].item())
    nbr = torch.empty(max(tot, 1), dtype=torch.int32, device="cuda")
    dfl = torch.empty(max(tot, 1), dtype=torch.uint8, device="cuda")
    ctx.check(lib().sph_neighbors_csr(ctx.h, _ptr(off), _ptr(nbr), _ptr(dfl), _stream(stream)))
    return off, nbr[:tot], dfl[:tot]


def sph_pair_count(ctx: Context, stream=None) -> int:
    """Running total of ordered pairs over every neighbour search of ``ctx``."""
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    ctx.check(lib().sph_pair_count(ctx.h, _ptr(out), _stream(stream)))
    return int(out.item())


def sph_timing(ctx: Context, enable: bool):
    ctx.check(lib().sph_timing(ctx.h, 1 if enable else 0))


def sph_timing_read(ctx: Context, which: int):
    """(total ms, launches) of pass kernel ``which`` (0 build, 1 density,
    2 gradients, 3 forces) since timing was enabled."""
    ms, cnt = C.c_double(), C.c_int64()
    ctx.check(lib().sph_timing_read(ctx.h, int(which), C.byref(ms), C.byref(cnt)))
    return ms.value, cnt.value


def sph_gravity(ctx: Context, m, ax, ay, az, phi=None, active=None, G=6.674e-11,
                eps_over_h=0.5, theta=0.6, accumulate=False, stream=None):
    """Self-gravity of every run at the last neighbour search (sorted order)."""
    ctx.check(lib().sph_gravity(ctx.h, int(m.numel()), _ptr(m), _ptr(active), float(G),
                                float(eps_over_h), float(theta), 1 if accumulate else 0,
                                _ptr(ax), _ptr(ay), _ptr(az), _ptr(phi), _stream(stream)))


def sph_bound_mass(ctx: Context, vx, vy, vz, m, n_runs: int, G=6.674e-11, eps_over_h=0.5,
                   theta=0.6, max_iter=100, stream=None):
    """Bound mass per run at the last neighbour search (sorted order).
    Returns (bound flags int32 tensor, bound mass per run float64 tensor,
    passes done)."""
    n = int(m.numel())
    bound = torch.zeros(max(n, 1), dtype=torch.int32, device=m.device)
    mb = torch.zeros(max(n_runs, 1), dtype=torch.float64, device=m.device)
    work = torch.empty(max(4 * n, 1), dtype=torch.float64, device=m.device)
    it = C.c_int32()
    ctx.check(lib().sph_bound_mass(ctx.h, n, _ptr(vx), _ptr(vy), _ptr(vz), _ptr(m), float(G),
                                   float(eps_over_h), float(theta), int(max_iter), _ptr(bound),
                                   _ptr(mb), _ptr(work), C.byref(it), _stream(stream)))
    return bound[:n], mb[:n_runs], it.value


def sph_adapt_h(ctx: Context, m, h_start, h_out, n_ngb: float, tol=1e-12, max_iter=50,
                n_clamped=None, iterations=None, stream=None):
    """Smoothing lengths at constant kernel mass over the last build's lists."""
    ctx.check(lib().sph_adapt_h(ctx.h, int(m.numel()), _ptr(m), _ptr(h_start), float(n_ngb),
                                float(tol), int(max_iter), _ptr(h_out), _ptr(n_clamped),
                                _ptr(iterations), _stream(stream)))


def sph_set_tuning(ctx: Context, knob: int, prec: int, value: int):
    ctx.check(lib().sph_set_tuning(ctx.h, int(knob), int(prec), int(value)))


def sph_get_tuning(ctx: Context, knob: int, prec: int) -> int:
    v = C.c_int32()
    ctx.check(lib().sph_get_tuning(ctx.h, int(knob), int(prec), C.byref(v)))
    return v.value


def sph_density(ctx: Context, m, h, u, mat, mats, prm, prec, out: dict, stream=None):
    arr = make_materials(mats)
    p = make_params(prm)
    ctx.check(lib().sph_density(ctx.h, m.numel(), _ptr(m), _ptr(h), _ptr(u), _ptr(mat), arr,
                                len(mats), C.byref(p), int(prec),
                                *[_ptr(out[k]) for k in ("rho", "omega", "P", "cs", "T", "Y", "Gmod")],
                                _stream(stream)))


def sph_gradients(ctx: Context, vx, vy, vz, m, h, rho, omega, prm, prec, G, n_singular=None,
                  stream=None):
    p = make_params(prm)
    ctx.check(lib().sph_gradients(ctx.h, m.numel(), _ptr(vx), _ptr(vy), _ptr(vz), _ptr(m), _ptr(h),
                                  _ptr(rho), _ptr(omega), C.byref(p), int(prec), _ptr(G),
                                  _ptr(n_singular), _stream(stream)))


def sph_stress_update(ctx: Context, phase, n, prm, dt=None, dt_next=None, G=None, Y=None,
                      Gmod=None, fixed=None, S_half=None, S_pred=None, Sdot=None, eps2=None,
                      stream=None):
    p = make_params(prm)
    ctx.check(lib().sph_stress_update(ctx.h, int(phase), int(n), _ptr(dt), _ptr(dt_next), _ptr(G),
                                      _ptr(Y), _ptr(Gmod), _ptr(fixed), C.byref(p), _ptr(S_half),
                                      _ptr(S_pred), _ptr(Sdot), _ptr(eps2), _stream(stream)))


def sph_forces_stress(ctx: Context, vx, vy, vz, m, h, rho, omega, P, cs, S, prm, prec, out: dict,
                      stream=None):
    p = make_params(prm)
    ctx.check(lib().sph_forces_stress(ctx.h, m.numel(), _ptr(vx), _ptr(vy), _ptr(vz), _ptr(m),
                                      _ptr(h), _ptr(rho), _ptr(omega), _ptr(P), _ptr(cs), _ptr(S),
                                      C.byref(p), int(prec),
                                      *[_ptr(out[k]) for k in ("ax", "ay", "az", "dudt", "dt")],
                                      _stream(stream)))


def sph_kick_drift(ctx: Context, phase, n, dt=None, dt_next=None, fixed=None, x=None, y=None,
                   z=None, vx=None, vy=None, vz=None, u=None, ax=None, ay=None, az=None, dudt=None,
                   vpx=None, vpy=None, vpz=None, up=None, stream=None):
    ctx.check(lib().sph_kick_drift(ctx.h, int(phase), int(n), *[_ptr(t) for t in (
        dt, dt_next, fixed, x, y, z, vx, vy, vz, u, ax, ay, az, dudt, vpx, vpy, vpz, up)],
        _stream(stream)))


def sph_dt_min(ctx: Context, dt_cfl, fixed, dt_out, stream=None):
    ctx.check(lib().sph_dt_min(ctx.h, dt_cfl.numel(), _ptr(dt_cfl), _ptr(fixed), _ptr(dt_out),
                               _stream(stream)))


def sph_diagnostics(ctx: Context, x, y, z, vx, vy, vz, m, ax, ay, az, dudt, out13, stream=None):
    ctx.check(lib().sph_diagnostics(ctx.h, m.numel(), *[_ptr(t) for t in (
        x, y, z, vx, vy, vz, m, ax, ay, az, dudt, out13)], _stream(stream)))


def sph_diagnostics_noalloc(x, y, z, vx, vy, vz, m, ax, ay, az, dudt, out13, n=None,
                            stream=None):
    """sph_diagnostics without a context (no allocation by the library);
    ``n`` defaults to the length of ``m``."""
    n = m.numel() if n is None else int(n)
    code = lib().sph_diagnostics_noalloc(n, *[_ptr(t) for t in (
        x, y, z, vx, vy, vz, m, ax, ay, az, dudt, out13)], _stream(stream))
    if code != SPH_OK:
        raise SphError(code, (lib().sph_last_error(None) or b"").decode())


def sph_init(ctx: Context, st: "State", mats, prm, prec, stream=None):
    st._sync_in()
    ctx.check(lib().sph_init(ctx.h, C.byref(st.c), st.mats_c(mats), len(mats),
                             C.byref(make_params(prm)), int(prec), _stream(stream)))
    st._sync_out()


def sph_step(ctx: Context, st: "State", mats, prm, prec, stream=None):
    st._sync_in()
    ctx.check(lib().sph_step(ctx.h, C.byref(st.c), st.mats_c(mats), len(mats),
                             C.byref(make_params(prm)), int(prec), _stream(stream)))
    st._sync_out()


class State:
    """Device buffers of a particle state in the row layout of ``sph_state``."""

    def __init__(self, w: dict, device="cuda", run_start=None, cell_min=0.0, dt_max=0.0):
        n = int(w["x"].size)
        self.n = n
        self.n_cap = max(n, 1)
        dd = dict(dtype=torch.float64, device=device)
        self.f64 = torch.zeros((2, SPH_NF64, self.n_cap), **dd)
        self.i32 = torch.zeros((2, SPH_NI32, self.n_cap), dtype=torch.int32, device=device)
        self.work = torch.zeros((SPH_NW, self.n_cap), **dd)
        # the library swaps the two step scalars after every step
        n_dt = 1 if run_start is None else len(run_start) - 1
        self._dt_pair = (torch.zeros(n_dt, **dd), torch.zeros(n_dt, **dd))
        self.clock = torch.zeros(n_dt, **dd)   # per run, ticks (individual steps)
        self.time = torch.zeros(n_dt, **dd)    # per run, simulated time since sph_init
        self.n_singular = torch.zeros(1, dtype=torch.int64, device=device)
        F = self.f64[0]
        for k, row in (("x", SPH_X), ("y", SPH_Y), ("z", SPH_Z), ("vx", SPH_VX), ("vy", SPH_VY),
                       ("vz", SPH_VZ), ("u", SPH_U), ("m", SPH_M), ("h", SPH_H)):
            F[row, :n] = torch.as_tensor(w[k], dtype=torch.float64)
        F[SPH_S:SPH_S + 5, :n] = torch.as_tensor(w["S"], dtype=torch.float64)
        I = self.i32[0]
        I[SPH_MAT, :n] = torch.as_tensor(w["mat"], dtype=torch.int32)
        I[SPH_ID, :n] = torch.arange(n, dtype=torch.int32)
        I[SPH_FIXED, :n] = torch.as_tensor(w["fixed"], dtype=torch.int32)
        self.run_start = None
        self._rs = None
        if run_start is not None:
            self._rs = (C.c_int64 * len(run_start))(*[int(v) for v in run_start])
            self.run_start = list(run_start)
            for r in range(len(run_start) - 1):
                I[SPH_RUN, run_start[r]:run_start[r + 1]] = r
        c = sph_state()
        c.n, c.n_cap = n, self.n_cap
        c.f64[0], c.f64[1] = self.f64[0].data_ptr(), self.f64[1].data_ptr()
        c.i32[0], c.i32[1] = self.i32[0].data_ptr(), self.i32[1].data_ptr()
        c.work = self.work.data_ptr()
        c.dt, c.dt_next = self._dt_pair[0].data_ptr(), self._dt_pair[1].data_ptr()
        c.n_singular = self.n_singular.data_ptr()
        c.cur = 0
        c.n_runs = 1 if run_start is None else len(run_start) - 1
        c.run_start = None if self._rs is None else C.cast(self._rs, _P).value
        c.cell_min = float(cell_min)
        c.dt_max = float(dt_max)
        c.clock = self.clock.data_ptr()
        c.time = self.time.data_ptr()
        self.c = c
        self._mats_cache = None

    def mats_c(self, mats):
        key = id(mats)
        if self._mats_cache is None or self._mats_cache[0] != key:
            self._mats_cache = (key, make_materials(mats))
        return self._mats_cache[1]

    def _sync_in(self):
        pass

    def _sync_out(self):
        pass

    @property
    def cur(self):
        return self.c.cur

    @property
    def dt(self):
        """Device scalar holding the step of the coming drift."""
        a, b = self._dt_pair
        return a if self.c.dt == a.data_ptr() else b

    def row(self, k):
        return self.f64[self.cur, k, :self.n]

    def irow(self, k):
        return self.i32[self.cur, k, :self.n]

    def wrow(self, k):
        return self.work[k, :self.n]

    def to_host(self, by_id=True) -> dict:
        """Current state as numpy arrays, in the caller's original particle
        order (by the ID row) when ``by_id``."""
        F = self.f64[self.cur, :, :self.n].cpu().numpy()
        I = self.i32[self.cur, :, :self.n].cpu().numpy()
        W = self.work[:, :self.n].cpu().numpy()
        order = slice(None)
        if by_id:
            inv = I[SPH_ID].argsort(kind="stable")
            order = inv
        out = dict(x=F[SPH_X][order], y=F[SPH_Y][order], z=F[SPH_Z][order],
                   vx=F[SPH_VX][order], vy=F[SPH_VY][order], vz=F[SPH_VZ][order],
                   u=F[SPH_U][order], S=F[SPH_S:SPH_S + 5][:, order],
                   a=F[SPH_AX:SPH_AX + 3][:, order], dudt=F[SPH_DUDT][order],
                   dS=F[SPH_SDOT:SPH_SDOT + 5][:, order], eps2=F[SPH_EPS2][order],
                   rho=W[SPH_W_RHO][order], omega=W[SPH_W_OMEGA][order], P=W[SPH_W_P][order],
                   c=W[SPH_W_CS][order], T=W[SPH_W_T][order], Y=W[SPH_W_Y][order],
                   Gam=W[SPH_W_GMOD][order], S_pred=W[SPH_W_SP:SPH_W_SP + 5][:, order],
                   G=W[SPH_W_G:SPH_W_G + 9][:, order], dt=W[SPH_W_DT][order],
                   id=I[SPH_ID][order], step_ticks=F[SPH_DTP][order],
                   elapsed_ticks=F[SPH_EL][order])
        return out


# ------------------------------------------------------ proposal network
def _mlp_check(code):
    if code != SPH_OK:
        raise SphError(code, "network kernel launch failed")


def sph_mlp_forward(X, params, out, h1=None, h2=None, stream=None):
    _mlp_check(lib().sph_mlp_forward(X.shape[0], _ptr(X), _ptr(params), _ptr(out), _ptr(h1),
                                     _ptr(h2), _stream(stream)))


def sph_mlp_backward(X, Y, params, out, h1, h2, work, grads, stream=None):
    _mlp_check(lib().sph_mlp_backward(X.shape[0], _ptr(X), _ptr(Y), _ptr(params), _ptr(out),
                                      _ptr(h1), _ptr(h2), _ptr(work), _ptr(grads),
                                      _stream(stream)))


def sph_mlp_loss(out, Y, loss, stream=None):
    """loss[0] = mean of (out - Y)^2 (float32 device tensors)."""
    _mlp_check(lib().sph_mlp_loss(int(out.numel()), _ptr(out), _ptr(Y), _ptr(loss),
                                  _stream(stream)))


def sph_mlp_adam(params, grads, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                 stream=None):
    _mlp_check(lib().sph_mlp_adam(_ptr(params), _ptr(grads), _ptr(m), _ptr(v), int(step),
                                  float(lr), float(beta1), float(beta2), float(eps),
                                  _stream(stream)))
