"""Benchmark of the strength-SPH step on one MI355X.

Headline workload: the two-sphere impact of about 1.1M particles (granite
target of radius 50 km with 1,000,162 particles and a projectile of equal
particle mass with 100,090, relaxed glass-like packings, h = 1.3 spacing,
projectile at 45 deg and 3 km/s, Collins yield with thermal softening,
Poisson-route shear modulus, gravity excluded), advanced by whole strength
steps with the FP32 cell-relative pair arithmetic; the plain FP64 path is
timed on the same workload beside it.  One step = drift, neighbour search
(cell sort + pair sets), reorder of the state, predictor, density + EOS +
yield, stress predict and rescale, corrected gradients, stress rate,
forces, CFL minimum, closing and opening kicks.  Metric: ordered neighbour
pairs per second, sum over the timed steps of sum_i |N_i| / wall time,
inputs resident in HBM.

Prints one JSON line (progress goes to stderr).  ``--gpus N`` with N > 1 is
not supported: one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SPH strength-step pair interactions/s (FP32 vs FP64 plain, 1 GPU) at 1e-5 rel err"
PEAK_FP32_VALU = 157.3e12   # MI355X FP32 vector, published (packed instructions)
PEAK_FP32_UNPACKED = 78.6e12  # the same pipes without packed FP32 (the library is compiled so)
PEAK_FP64_VALU = 78.6e12
PEAK_HBM = 8.0e12

# Algorithmic flops per ordered pair of the fused gradient + force sweep.
# Estimates per pass (FMA = 2, sqrt and division 1 each): gradients ~60
# (the corrected velocity-gradient sums), forces ~110 plus ~25 when the pair
# approaches (the AV term); both passes' work is credited, each with its own
# separation, square root and kernel factors, as a two-pass code would do it.
EST_GRADIENTS, EST_FORCES, EST_AV = 60.0, 110.0, 25.0
# The same work counted from the fused pair term, shared parts once:
# separation 3, r^2 5, sqrt 1, kernel factors t_i^3, t_j^3 with Kn 10, v_ij 3;
# gradient weight 8, C^-1 sums 12, F sums 18; (K A)_i x and (K A)_j x 30,
# their combination into the momentum sum 15, energy term 8, v_ij . x_ij 5
# -> 118; the viscosity of an approaching pair adds 40 (two means, the
# softened mu with one division, Pi with one division, mean kernel
# gradient, momentum and energy updates, the CFL maximum).
RECOUNT, RECOUNT_AV = 118.0, 40.0

# Measured HBM traffic of the dominant pair kernel (rocprofv3 FETCH_SIZE and
# WRITE_SIZE per dispatch, scaled by the same counters on a plain copy of
# known size).  Valid only for the kernel source it was taken on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_grad_forces_c3_fp32_traffic.md")
TRAFFIC_SOURCES = ("paper_2603_19764_amd/csrc/pairs.hip", "paper_2603_19764_amd/csrc/device_util.h",
                   "paper_2603_19764_amd/csrc/records.h", "paper_2603_19764_amd/csrc/sph_internal.h")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel: str):
    """Bytes per launch of ``kernel`` (e.g. "k_grad_forces<8,fp32,2>") from the
    committed counter summary, or None when it is missing, does not list that
    instantiation, or was taken on another version of the kernel source."""
    import re
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    sha = re.search(r"source_sha256:\s*([0-9a-f]{64})", text)
    val = re.search(r"traffic_bytes_per_launch\[" + re.escape(kernel) + r"\]:\s*([0-9.eE+]+)",
                    text)
    if not sha or not val or sha.group(1) != kernel_source_sha256():
        return None
    return float(val.group(1))


def copy_calibration(mib: int):
    """A plain device-to-device copy of known size, for scaling the HBM
    byte counters (profiled together with the workload)."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy calibration: 3 copies of {mib} MiB ({n * 8} bytes read and written each)")
    del a, b


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


# ------------------------------------------------------------- GPU steps
def run_steps(w, prec, steps, warmup, use_graph=False, timing=True, tuned=None, keep=False,
              max_neighbors=128):
    """Whole steps of workload ``w``: sph_init, ``warmup`` steps, then exactly
    ``steps`` timed steps (HIP events around each step on the launch stream,
    wall clock around all of them, synchronised on both sides).  With
    ``timing`` the library's event timers record the pass kernels over the
    timed region."""
    import torch
    from paper_2603_19764_amd import autotune, sph

    n = int(w["x"].size)
    ctx = sph.Context(n, max_neighbors=max_neighbors, max_cells=1 << 22)
    if tuned:
        autotune.apply(ctx, prec, tuned)
    st = sph.State(w)
    mats, prm = w["mats"], w["params"]
    sph.sph_init(ctx, st, mats, prm, prec)
    for _ in range(warmup):
        sph.sph_step(ctx, st, mats, prm, prec)
    torch.cuda.synchronize()
    ctx.check(sph.lib().sph_sync_status(ctx.h, None))
    graph = None
    if use_graph:
        # the state buffers flip every step: capture two steps per replay
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            sph.sph_step(ctx, st, mats, prm, prec)
            sph.sph_step(ctx, st, mats, prm, prec)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            sph.sph_step(ctx, st, mats, prm, prec)
            sph.sph_step(ctx, st, mats, prm, prec)
        graph.replay()
        torch.cuda.synchronize()
    if timing and not use_graph:
        sph.sph_timing(ctx, True)
    p0 = sph.sph_pair_count(ctx)
    reps = steps // 2 if use_graph else steps
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(reps):
        if use_graph:
            graph.replay()
        else:
            sph.sph_step(ctx, st, mats, prm, prec)
        ev[k + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    p1 = sph.sph_pair_count(ctx)
    ctx.check(sph.lib().sph_sync_status(ctx.h, None))
    k_steps = reps * 2 if use_graph else steps
    per = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(reps)]) / (2 if use_graph else 1)
    kern = {}
    if timing and not use_graph:
        for name, kid in (("build", sph.SPH_T_BUILD), ("density", sph.SPH_T_DENSITY),
                          ("grad_forces", sph.SPH_T_FORCES)):
            kern[name] = sph.sph_timing_read(ctx, kid)
        sph.sph_timing(ctx, False)
    out = dict(seconds=t1 - t0, steps=k_steps, pairs=p1 - p0, kernels=kern, n=n,
               ms_median=float(np.median(per)) if per.size else None)
    if keep:
        out["state"], out["ctx"] = st, ctx
    else:
        ctx.close()
    del graph
    return out


def approaching_fraction(st, h_max, sample=20000, seed=3):
    """Fraction of ordered pairs (r < max(H_i, H_j), H = 2h) that approach,
    v_ij . x_ij < 0, at the state of the last evaluation (positions and the
    predicted velocities the sweep used), on a random sample of particles."""
    from scipy.spatial import cKDTree
    from paper_2603_19764_amd import sph
    n = st.n
    x = np.stack([st.row(k).cpu().numpy() for k in (sph.SPH_X, sph.SPH_Y, sph.SPH_Z)], 1)
    v = np.stack([st.wrow(sph.SPH_W_VP + k).cpu().numpy() for k in range(3)], 1)
    h = st.row(sph.SPH_H).cpu().numpy()
    rng = np.random.default_rng(seed)
    idx = rng.choice(n, min(sample, n), replace=False)
    tree = cKDTree(x)
    lists = tree.query_ball_point(x[idx], 2.0 * h_max)
    app = tot = 0
    for i, js in zip(idx, lists):
        js = np.asarray(js)
        js = js[js != i]
        d = x[i] - x[js]
        r2 = np.einsum("ij,ij->i", d, d)
        H = np.maximum(2.0 * h[i], 2.0 * h[js])
        ok = r2 < H * H
        vr = np.einsum("ij,ij->i", v[i] - v[js][ok], d[ok])
        app += int((vr < 0.0).sum())
        tot += int(ok.sum())
    return app / max(tot, 1)


def stir(w, seed, v0, s0, length):
    """A smooth velocity field of amplitude v0 (wavelength `length`) on the
    mobile particles and random deviatoric stresses of scale s0, so that every
    derivative is non-zero at t = 0 (accuracy sample)."""
    rng = np.random.default_rng(seed)
    k = 2.0 * np.pi / length
    mob = w["fixed"] == 0
    w = dict(w)
    w["vx"] = w["vx"] + np.where(mob, v0 * np.sin(k * w["y"] + 0.3), 0.0)
    w["vy"] = w["vy"] + np.where(mob, v0 * np.sin(k * w["z"] + 1.1), 0.0)
    w["vz"] = w["vz"] + np.where(mob, v0 * np.sin(k * w["x"] + 2.3), 0.0)
    w["S"] = w["S"] + np.where(mob, s0 * rng.standard_normal(w["S"].shape), 0.0)
    return w


def gpu_evaluation(w, prec, tuned):
    """One derivative evaluation in the benchmark's launch configuration (the
    fused path of sph_init with the tuned shapes); fields in input order."""
    import torch
    from paper_2603_19764_amd import autotune, sph
    n = int(w["x"].size)
    ctx = sph.Context(n, 128, max_cells=1 << 22)
    if tuned:
        autotune.apply(ctx, prec, tuned)
    st = sph.State(w)
    sph.sph_init(ctx, st, w["mats"], w["params"], prec)
    torch.cuda.synchronize()
    ctx.check(sph.lib().sph_sync_status(ctx.h, None))
    g = st.to_host()
    ctx.close()
    return g


# ------------------------------------------------------ oracle on the host
def oracle_sample(w, targets):
    """The FP64 oracle's full derivative chain (brute-force O(N^2) pair sets
    against all particles, density + EOS of the pair-set closure, gradients,
    stress rate, forces) for ``targets``; returns (reference dict, seconds)."""
    from oracle import oracle
    st = {k: w[k] for k in ("x", "y", "z", "m", "h", "mat", "vx", "vy", "vz", "u", "S")}
    t0 = time.perf_counter()
    ref = oracle.derivs(st, w["mats"], w["params"], targets)
    return ref, time.perf_counter() - t0


def search_seconds(w, targets):
    """Time of the brute-force neighbour search alone, as the oracle's chain
    performs it: a sweep over all particles per target in each of the two
    passes of the pair-set closure, the gradients and the forces, and per
    member of the closure in the density (each sweep timed as the count of
    the pair set, which tests every particle once).  Returns (seconds,
    ordered pairs of the targets, closure size)."""
    from oracle import oracle
    x, y, z, h, prm = w["x"], w["y"], w["z"], w["h"], w["params"]
    off, nbr, _ = oracle.pair_lists(x, y, z, h, prm, targets)
    near = np.unique(np.concatenate([np.asarray(targets, dtype=np.int64), nbr]))
    t0 = time.perf_counter()
    oracle.pair_counts(x, y, z, h, prm, targets)
    t_tar = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.pair_counts(x, y, z, h, prm, near)
    t_near = time.perf_counter() - t0
    return 4.0 * t_tar + t_near, int(off[-1]), int(near.size)


class _Sampler:
    """Compact samples of a workload: the k particles nearest a random
    particle (their pair-set closure stays close to the sample), and the
    sub-volume around a sample that holds everything its derivatives read
    (particles within two supports of it: pair sets, and the pair sets of
    their members for the densities)."""

    def __init__(self, w, seed):
        from scipy.spatial import cKDTree
        self.w = w
        self.x = np.stack([w["x"], w["y"], w["z"]], 1)
        self.tree = cKDTree(self.x)
        self.rng = np.random.default_rng(seed)
        self.c = self.x[self.rng.integers(self.x.shape[0])]
        self.H = 2.0 * float(np.max(w["h"]))

    def targets(self, k, c=None):
        c = self.c if c is None else c
        d, idx = self.tree.query(c, k=min(k, self.x.shape[0]))
        idx = np.atleast_1d(idx)
        return np.sort(idx).astype(np.int64), float(np.max(d))

    def new_centre(self):
        return self.x[self.rng.integers(self.x.shape[0])]

    def sub(self, radius, c=None):
        """(sub-workload, index map sub -> full) of the particles within
        radius + 2 H (+5%) of the centre."""
        c = self.c if c is None else c
        keep = np.sort(np.asarray(self.tree.query_ball_point(c, radius + 2.1 * self.H),
                                  dtype=np.int64))
        n = self.x.shape[0]
        sub = {k: (v[..., keep] if isinstance(v, np.ndarray) and v.shape[-1] == n else v)
               for k, v in self.w.items()}
        return sub, keep


def _omp():
    """Handle to the OpenMP runtime the oracle uses (to run it on one core)."""
    import ctypes
    g = ctypes.CDLL("libgomp.so.1")
    g.omp_get_max_threads.restype = ctypes.c_int
    g.omp_set_num_threads.argtypes = [ctypes.c_int]
    return g


def _scaled(measure, budget_s, k0=32, n_max=None):
    """Grow the sample size k until one measurement takes about
    0.3-0.6 of ``budget_s``; returns the last (k, result, seconds)."""
    k = k0
    while True:
        res, t = measure(k)
        if t > 0.3 * budget_s or (n_max is not None and k >= n_max):
            return k, res, t
        k = int(k * max(2.0, min(8.0, 0.6 * budget_s / max(t, 1e-3))))


def cpu_baseline(w, budget_s=6.0, ball=300):
    """The oracle as it stands, timed on the host on compact samples of the
    workload (each measurement about half of ``budget_s``): all threads, then
    one thread.  Rate = ordered pairs of the sample / time of the FP64
    derivative chain.  Two figures per thread count: the chain as the oracle
    runs it on the whole workload, its brute-force O(N^2) search against all
    particles; and the chain on small sub-volumes (``ball`` particles nearest
    a random particle, with everything their derivatives read: same results
    for them, a brute-force search over a few thousand particles only), with
    the time of that search measured alone and subtracted for the
    search-excluded rate."""
    from oracle import oracle
    oracle.lib()
    omp = _omp()
    threads = omp.omp_get_max_threads()
    smp = _Sampler(w, seed=17)
    n = int(w["x"].size)
    out = {}
    for leg, nthr in (("all", threads), ("one", 1)):
        omp.omp_set_num_threads(nthr)

        def full(k):
            tar, _ = smp.targets(k)
            _, t = oracle_sample(w, tar)
            return tar, t

        k, tar, t = _scaled(full, budget_s, n_max=n)
        off, _, _ = oracle.pair_lists(w["x"], w["y"], w["z"], w["h"], w["params"], tar)
        pairs = int(off[-1])
        # sub-volumes until about half the budget is spent in their chains
        t_sub = s_sub = 0.0
        p_sub = m_sub = nb = 0
        while t_sub < 0.5 * budget_s and nb < 4096:
            c = smp.new_centre()
            tar_k, rad = smp.targets(ball, c)
            sub, keep = smp.sub(rad, c)
            tar_s = np.searchsorted(keep, tar_k)
            _, ts = oracle_sample(sub, tar_s)
            ss, ps, _ = search_seconds(sub, tar_s)
            t_sub += ts
            s_sub += ss
            p_sub += ps
            m_sub += int(keep.size)
            nb += 1
        phys = t_sub - s_sub
        out[leg] = dict(threads=nthr, targets=int(tar.size), pairs=pairs, chain_s=t,
                        value=pairs / t, sub_volumes=nb, sub_particles=m_sub // max(nb, 1),
                        sub_pairs=p_sub, sub_chain_s=t_sub, sub_search_s=s_sub,
                        value_sub=p_sub / t_sub,
                        value_search_excluded=(p_sub / phys) if phys > 0.0 else None)
        log(f"cpu baseline ({leg}, {nthr} threads): {tar.size} targets, {pairs} pairs, chain "
            f"{t:.2f} s; {nb} sub-volumes of ~{m_sub // max(nb, 1)} with {ball} targets: "
            f"chains {t_sub:.2f} s, their search {s_sub:.2f} s")
    omp.omp_set_num_threads(threads)
    a, o = out["all"], out["one"]
    return dict(value=a["value"], unit="pairs/s", cores=a["threads"], kind="oracle",
                sample=f"{cpu_model()}, {a['threads']} threads: the {a['targets']} particles "
                       f"nearest a random particle of the {n}-particle impact ({a['pairs']} "
                       f"ordered pairs), full FP64 derivative chain with brute-force O(N^2) "
                       f"neighbour search over all particles, {a['chain_s']:.2f} s",
                search_restricted=dict(
                    value=a["value_sub"], value_search_excluded=a["value_search_excluded"],
                    sub_volumes=a["sub_volumes"], targets_each=ball,
                    particles_each=a["sub_particles"], pairs=a["sub_pairs"],
                    chain_s=a["sub_chain_s"], search_s=a["sub_search_s"]),
                single_core=dict(
                    value=o["value"], targets=o["targets"], pairs=o["pairs"],
                    chain_s=o["chain_s"], value_search_restricted=o["value_sub"],
                    value_search_excluded=o["value_search_excluded"],
                    sub_volumes=o["sub_volumes"], sub_chain_s=o["sub_chain_s"],
                    sub_search_s=o["sub_search_s"]))


def accuracy(w, tuned, ntar=200, seed=9):
    """FP32 form against the FP64 oracle on a stirred copy of the workload
    (smooth velocities of 30 m/s, random stresses of 10 MPa): per field the
    normwise error max_i |dX_i| / max_i |X_i| and the median and 99th
    percentile of the per-particle error |dX_i| / (|X_i| + s_i), s_i the
    summed magnitudes of the pair contributions, on random particles."""
    from oracle import oracle
    ws = stir(w, 11, 30.0, 1.0e7, 1.0e5)
    n = int(ws["x"].size)
    rng = np.random.default_rng(seed)
    tar = np.unique(rng.choice(n, ntar, replace=False))
    st = {k: ws[k] for k in ("x", "y", "z", "m", "h", "mat", "vx", "vy", "vz", "u", "S")}
    ref = oracle.derivs(st, ws["mats"], ws["params"], tar, scales=True)
    g = gpu_evaluation(ws, 1, tuned)
    out = {}
    for k in ("a", "dS", "G", "dudt", "rho"):
        r, x = ref[k][..., tar], g[k][..., tar]
        rr = np.atleast_2d(r)
        d = np.sqrt(((np.atleast_2d(x) - rr) ** 2).sum(0))
        e = dict(normwise=float(d.max() / np.sqrt((rr ** 2).sum(0)).max()))
        if k in ref["scale"]:
            den = np.sqrt((rr ** 2).sum(0)) + ref["scale"][k][tar]
            pe = np.where(den > 0, d / np.where(den > 0, den, 1.0), np.where(d > 0, np.inf, 0.0))
            e.update(median=float(np.median(pe)), p99=float(np.percentile(pe, 99)),
                     max=float(pe.max()))
        out[k] = e
    out["sample"] = (f"{tar.size} random particles of the stirred workload, FP32 evaluation "
                     "in the benchmark's launch configuration against the FP64 oracle")
    log(f"accuracy: {out}")
    return out


# ------------------------------------------------------------ extra legs
def run_batch(steps, warmup, gravity=True, tune=True):
    """The batched Q_RD* scan: 64 head-on impacts of uneven sizes (targets
    20k-300k particles, ~7.2M in all) in one set of buffers, FP32 pair
    arithmetic, self-gravity on, per-run time steps, two steps captured in a
    hipGraph and replayed.  Rate = ordered pairs of all runs per second."""
    import torch
    from paper_2603_19764_amd import autotune, inputs, sph

    b = inputs.scan_batch(64, seed=5)
    if gravity:
        b["params"] = inputs.default_params(grav_G=inputs.G_NEWTON)
    rs = [int(v) for v in b["run_start"]]
    n = int(b["x"].size)
    tuned = None
    if tune:
        tuned = autotune.tune(b, 1, steps=2, run_start=rs, max_neighbors=256,
                              max_cells=1 << 24)["settings"]
        log(f"batch autotune: {tuned}")
    # colliding bodies compress: room for twice the neighbours of the lattice
    ctx = sph.Context(n, max_neighbors=256, max_cells=1 << 24, max_runs=64)
    if tuned:
        autotune.apply(ctx, 1, tuned)
    st = sph.State(b, run_start=rs)
    mats, prm = b["mats"], b["params"]
    sph.sph_init(ctx, st, mats, prm, 1)
    for _ in range(warmup):
        sph.sph_step(ctx, st, mats, prm, 1)
    torch.cuda.synchronize()
    ctx.check(sph.lib().sph_sync_status(ctx.h, None))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sph.sph_step(ctx, st, mats, prm, 1)
        sph.sph_step(ctx, st, mats, prm, 1)
    g.replay()  # first replay outside the timed region
    torch.cuda.synchronize()
    p0 = sph.sph_pair_count(ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps // 2):
        g.replay()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    p1 = sph.sph_pair_count(ctx)
    ctx.check(sph.lib().sph_sync_status(ctx.h, None))
    k = (steps // 2) * 2
    dt = st.dt.cpu().numpy()
    del g
    ctx.close()
    return {"workload": f"batched Q_RD* scan: 64 head-on impacts, {n} particles, targets "
                        f"{min(np.diff(rs))}-{max(np.diff(rs))} per run (incl. projectiles), "
                        "FP32 pair loop, self-gravity " + ("on" if gravity else "off"),
            "value": (p1 - p0) / (t1 - t0), "unit": "pairs/s", "steps": k,
            "ms_per_step": 1e3 * (t1 - t0) / k, "pairs_per_step": (p1 - p0) / k,
            "graph": True, "launch_shapes": tuned,
            "dt_spread": float(dt.max() / dt.min())}


def run_batch_outcomes(max_steps=12000, check_every=10, seed=5, scale=1.0, far_factor=3.0,
                       t_end_sound=6.0):
    """The 64-impact batch (FP32, self-gravity on; particle counts times
    ``scale``; each run in its centre-of-mass frame) run to every run's t_end
    (the crossing time plus the shorter of ``t_end_sound`` sound-crossing
    times of the target and two free-fall times), ejecta beyond the run's far
    cube (``far_factor``) counted unbound: each run's largest-remnant
    fraction f_lr when it passes t_end/2 and t_end, and whether it changed
    by less than 1% of the run's mass between the two (converged)."""
    from paper_2603_19764_amd import inputs, scan
    b = inputs.scan_batch(64, seed=seed, scale=scale, cm_frame=True)
    t_end = scan.end_times(b["cases"], t_end_sound=t_end_sound)
    r = scan.run_to_end(b, t_end, (0.5, 1.0), max_steps=max_steps, check_every=check_every,
                        log=log, max_cells=1 << 26, far_factor=far_factor)
    f1, f2 = r["f"][0.5], r["f"][1.0]
    d = np.abs(f2 - f1)
    runs = [{"n_particles": int(b["run_start"][k + 1] - b["run_start"][k]),
             "v_over_vesc": c["v"] / c["v_esc"], "strength": c["strength"],
             "m_tot": c["m_tot"], "t_end_s": float(t_end[k]),
             "f_lr_half": None if np.isnan(f1[k]) else float(f1[k]),
             "f_lr_end": None if np.isnan(f2[k]) else float(f2[k])}
            for k, c in enumerate(b["cases"])]
    ok = ~np.isnan(d)
    return {"workload": f"the 64-impact batch ({int(b['x'].size)} particles, target counts x "
                        f"{scale}) run to t_end (crossing time + min({t_end_sound} sound "
                        f"crossings, 2 free-fall times)) with self-gravity, FP32, far cube "
                        f"{far_factor}", "steps": r["steps"], "seconds": r["seconds"],
            "runs_reaching_t_end": int(r["reached"].sum()),
            "converged_runs": int((d[ok] < 0.01).sum()), "compared_runs": int(ok.sum()),
            "max_change": float(d[ok].max()) if ok.any() else None, "runs": runs}


def run_column(steps, warmup, tune=True):
    """The granular column (196,794 mobile particles on a floor of 29,928
    fixed ones, FP32 and FP64 whole steps)."""
    from paper_2603_19764_amd import autotune, inputs
    w = inputs.c2_column()
    row = {"workload": "granular column, 196794 mobile + 29928 fixed particles, Drucker-Prager "
                       "tan 30, g = 9.81", "particles": int(w["x"].size)}
    for prec, name in ((1, "fp32"), (0, "fp64")):
        tuned = autotune.tune(w, prec, steps=3)["settings"] if tune else None
        r = run_steps(w, prec, steps, warmup, timing=False, tuned=tuned)
        row[name] = {"pairs_per_s": r["pairs"] / r["seconds"],
                     "ms_per_step": 1e3 * r["seconds"] / r["steps"],
                     "pairs_per_step": r["pairs"] / r["steps"], "launch_shapes": tuned}
    log(f"column: {row}")
    return row


def run_curve(sizes=(32, 64, 128, 160), steps=40, warmup=3):
    """Throughput against size: the single-step block workload (16^3 lattice,
    spacing 1 m, jitter, shear flow) scaled to n_side^3 particles, FP32 and
    FP64 whole steps."""
    from paper_2603_19764_amd import inputs
    out = []
    for k in sizes:
        w = inputs.c1_block(k)
        row = {"n_side": k, "particles": int(w["x"].size)}
        for prec, name in ((1, "fp32"), (0, "fp64")):
            r = run_steps(w, prec, steps, warmup, timing=False)
            row[name] = {"pairs_per_s": r["pairs"] / r["seconds"],
                         "ms_per_step": 1e3 * r["seconds"] / r["steps"]}
        log(f"curve {k}^3: {row}")
        out.append(row)
    return out


def _conserved(st, mats):
    """Total momentum and energy (kinetic + internal, half-step velocities
    and energies) of a state, in FP64 on the host."""
    from paper_2603_19764_amd import sph
    m = st.row(sph.SPH_M).cpu().numpy()
    v = np.stack([st.row(k).cpu().numpy() for k in (sph.SPH_VX, sph.SPH_VY, sph.SPH_VZ)])
    u = st.row(sph.SPH_U).cpu().numpy()
    return (m * v).sum(1), float((m * (0.5 * (v * v).sum(0) + u)).sum())


def run_hsteps(n_side=64, prec=1, shared_steps=600):
    """Individual time steps against one shared step on a block with a hot
    core: a 64^3 lattice block (the spacing, jitter and shear flow of the
    single-step block) whose central sphere of a fifth of its edge carries
    u = 3e6 J/kg.  The shared step runs ``shared_steps`` steps (it follows
    the particle with the shortest CFL step); the rungs (base step: the
    longest CFL step at the start) then run to the same simulated time.
    Figure of merit: wall time to that simulated time; accuracy: the drift
    of total momentum and energy in each run and the difference of the
    final states (positions, velocities, energies) between the two."""
    import torch
    from paper_2603_19764_amd import inputs, sph
    w = inputs.c1_block(n_side)
    c = np.array([w[k].mean() for k in ("x", "y", "z")])
    r = np.sqrt((w["x"] - c[0]) ** 2 + (w["y"] - c[1]) ** 2 + (w["z"] - c[2]) ** 2)
    hot = r < 0.2 * n_side
    w["u"] = np.where(hot, 3.0e6, w["u"])
    n = int(w["x"].size)
    out = {"workload": f"{n_side}^3 block with a hot core ({int(hot.sum())} of {n} particles "
                       "at u = 3e6 J/kg)", "precision": "fp32" if prec else "fp64"}
    t_target = None
    dt0 = None
    final = {}
    for mode in ("shared", "rungs"):
        prm = dict(w["params"])
        if mode == "rungs":
            prm["rungs"] = 8
        ctx = sph.Context(n, 128, max_cells=1 << 22)
        st = sph.State(w, dt_max=dt0 if mode == "rungs" else 0.0)
        sph.sph_init(ctx, st, w["mats"], prm, prec)
        torch.cuda.synchronize()
        if mode == "shared":
            dt0 = float(st.wrow(sph.SPH_W_DT).max()) * 1.01
        p0, e0 = _conserved(st, w["mats"])
        k = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while True:
            for _ in range(20):
                sph.sph_step(ctx, st, w["mats"], prm, prec)   # advances st.time
            k += 20
            if mode == "shared" and k >= shared_steps:
                break
            if mode == "rungs" and float(st.time.item()) >= t_target:
                break
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sim = float(st.time.item())
        ctx.check(sph.lib().sph_sync_status(ctx.h, None))
        p1, e1 = _conserved(st, w["mats"])
        pscale = float((st.row(sph.SPH_M).cpu().numpy() * np.abs(
            st.row(sph.SPH_VX).cpu().numpy())).sum()) + 1e-300
        row = {"steps": k, "wall_s": t1 - t0, "ms_per_step": 1e3 * (t1 - t0) / k,
               "simulated_s": sim, "energy_drift": (e1 - e0) / abs(e0),
               "momentum_drift": float(np.abs(p1 - p0).max() / pscale)}
        if mode == "shared":
            t_target = sim
        else:
            steps = st.row(sph.SPH_DTP).cpu().numpy()
            vals, cnt = np.unique(steps, return_counts=True)
            row["base_step_s"] = dt0
            row["particles_per_step_ticks"] = {str(int(v)): int(q) for v, q in zip(vals, cnt)}
        final[mode] = st.to_host()
        out[mode] = row
        ctx.close()
    # the two runs end at slightly different times (the rungs stop at the
    # first substep at or past the shared run's time): compare the states
    a, b = final["shared"], final["rungs"]
    disp = np.stack([a[k] - w[k] for k in "xyz"])
    out["state_difference"] = {
        "position": float(np.abs(np.stack([b[k] - a[k] for k in "xyz"])).max()
                          / np.abs(disp).max()),
        "velocity": float(np.abs(np.stack([b[k] - a[k] for k in ("vx", "vy", "vz")])).max()
                          / np.abs(np.stack([a[k] for k in ("vx", "vy", "vz")])).max()),
        "energy": float(np.abs(b["u"] - a["u"]).max() / np.abs(a["u"] - w["u"]).max()),
        "time_difference": (out["rungs"]["simulated_s"] - t_target) / t_target}
    out["speedup"] = (out["shared"]["wall_s"] / out["shared"]["simulated_s"]) / (
        out["rungs"]["wall_s"] / out["rungs"]["simulated_s"])
    log(f"individual steps: {out}")
    return out


CAMPAIGN_FILE = os.path.join(ROOT, "profiles", "qrd_campaign_c5.md")


def recorded_campaign():
    """Figures of the production-size Q_RD* campaign (simulations per held-out
    case for bisection and for the network, thresholds, GPU time), as the
    campaign driver recorded them in the committed summary; None when the
    summary is missing.  The campaign runs for tens of GPU minutes, so the
    benchmark reports the record rather than rerunning it."""
    import re
    try:
        text = open(CAMPAIGN_FILE).read()
    except OSError:
        return None
    m = re.search(r"campaign_summary:\s*(\{.*\})\s*$", text, re.M)
    if not m:
        return None
    out = json.loads(m.group(1))
    out["source"] = os.path.relpath(CAMPAIGN_FILE, ROOT)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--graph", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-curve", action="store_true",
                    help="skip the size curve (block workload, 32^3 to 160^3)")
    ap.add_argument("--no-column", action="store_true", help="skip the granular column")
    ap.add_argument("--no-hsteps", action="store_true",
                    help="skip the individual-step comparison on the hot-core block")
    ap.add_argument("--batch-steps", type=int, default=20,
                    help="steps of the batched 64-impact scan (0: skip it)")
    ap.add_argument("--batch-outcomes", type=float, default=0.0, metavar="SCALE",
                    help="also run the 64-impact batch with target counts times SCALE to "
                         "t_end (minutes) for each run's largest-remnant fraction at t_end/2 "
                         "and t_end (0: skip)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default launch shapes (no autotuning before the warmup)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the timed FP32 steps of the headline workload (profiling)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device to device (counter calibration)")
    ap.add_argument("--batch-only", type=int, default=0, metavar="STEPS",
                    help="only the batched 64-impact scan, STEPS graph-replayed steps "
                         "(profiling)")
    ap.add_argument("--outcomes-only", type=float, default=0.0, metavar="SCALE",
                    help="only the 64-impact batch run to t_end (see --batch-outcomes)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2603_19764_amd import inputs

    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
    if args.batch_only:
        print(json.dumps(run_batch(args.batch_only, 4, tune=not args.no_tune)), flush=True)
        return
    if args.outcomes_only > 0:
        print(json.dumps(run_batch_outcomes(scale=args.outcomes_only)), flush=True)
        return
    w = inputs.c3_impact()
    n = int(w["x"].size)
    log(f"workload {w['name']}: n={n}")
    tuned = {0: None, 1: None}
    if not args.no_tune:
        from paper_2603_19764_amd import autotune
        for prec in ((1,) if args.no_fp64 else (1, 0)):
            t = autotune.tune(w, prec, steps=3)
            tuned[prec] = t["settings"]
            log(f"autotune prec {prec}: {t['settings']} {t['times_ms']}")
    r32 = run_steps(w, 1, args.steps, args.warmup, bool(args.graph), tuned=tuned[1], keep=True)
    log(f"fp32: {r32['seconds']:.4f} s for {r32['steps']} steps, {r32['pairs']} pairs")
    if args.headline_only:
        r32["ctx"].close()
        line = {"metric": METRIC, "value": r32["pairs"] / r32["seconds"],
                "ms_per_step": 1e3 * r32["seconds"] / r32["steps"]}
        if not args.no_fp64:
            r64 = run_steps(w, 0, args.steps, args.warmup, bool(args.graph), tuned=tuned[0])
            line["fp64_plain"] = {"value": r64["pairs"] / r64["seconds"],
                                  "ms_per_step": 1e3 * r64["seconds"] / r64["steps"]}
        print(json.dumps(line), flush=True)
        return
    f_av = approaching_fraction(r32["state"], float(w["h"].max()))
    r32["ctx"].close()
    del r32["state"], r32["ctx"]
    r64 = None
    if not args.no_fp64:
        r64 = run_steps(w, 0, args.steps, args.warmup, bool(args.graph), tuned=tuned[0])
        log(f"fp64: {r64['seconds']:.4f} s for {r64['steps']} steps, {r64['pairs']} pairs")
    value = r32["pairs"] / r32["seconds"]
    ms_step = 1e3 * r32["seconds"] / r32["steps"]
    roof = None
    if r32["kernels"]:
        ms, cnt = r32["kernels"]["grad_forces"]
        avg_s = ms / cnt * 1e-3
        ppl = r32["pairs"] / r32["steps"]
        fl_est = EST_GRADIENTS + EST_FORCES + EST_AV * f_av
        fl_recount = RECOUNT + RECOUNT_AV * f_av
        achieved = fl_est * ppl / avg_s
        lanes = (tuned[1] or {}).get("lanes_step", 8)
        depth = (tuned[1] or {}).get("sweep_depth", 2)
        kname = f"k_grad_forces<{lanes},fp32,{depth}>"
        roof = dict(bound="alu", achieved=achieved / 1e12, peak=PEAK_FP32_VALU / 1e12,
                    unit="TFLOP/s", frac=achieved / PEAK_FP32_VALU,
                    frac_unpacked=achieved / PEAK_FP32_UNPACKED,
                    traffic=measured_traffic(kname), kernel=kname, avg_launch_us=avg_s * 1e6,
                    pairs_per_launch=ppl, flops_per_pair=fl_est,
                    flops_per_pair_recount=fl_recount,
                    frac_recount=fl_recount * ppl / avg_s / PEAK_FP32_VALU,
                    approaching_pair_fraction=f_av,
                    kernels_us={k: (v[0] / v[1] * 1e3 if v[1] else None)
                                for k, v in r32["kernels"].items()})
    acc = None if args.no_accuracy else accuracy(w, tuned[1])
    column = None if args.no_column else run_column(max(args.steps, 20), args.warmup,
                                                    tune=not args.no_tune)
    curve = None if args.no_curve else run_curve()
    hsteps = None if args.no_hsteps else run_hsteps()
    batch = None
    if args.batch_steps > 0:
        batch = run_batch(args.batch_steps, 4, tune=not args.no_tune)
        log(f"batch: {batch['ms_per_step']:.3f} ms/step, {batch['value']:.3e} pairs/s")
    outcomes = run_batch_outcomes(scale=args.batch_outcomes) if args.batch_outcomes > 0 else None
    cpu = None if args.no_cpu_baseline else cpu_baseline(w)
    line = {
        "metric": METRIC, "value": value, "unit": "pairs/s", "n_gpus": 1,
        "steps": r32["steps"], "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 pair terms, f64 state", "data": "synthetic",
        "config": {"workload": f"two-sphere impact: granite target {w['n_target']} + projectile "
                               f"{n - w['n_target']} particles (relaxed glass, h = 1.3 spacing), "
                               "45 deg, 3 km/s, Collins yield with thermal softening, gravity "
                               "excluded; whole strength steps, FP32 cell-relative pair loop",
                   "particles": n, "pairs_per_step": r32["pairs"] / r32["steps"],
                   "ms_per_step_median": r32["ms_median"], "graph": bool(args.graph),
                   "launch_shapes": tuned[1]},
        "fp64_plain": None if r64 is None else {
            "value": r64["pairs"] / r64["seconds"],
            "ms_per_step": 1e3 * r64["seconds"] / r64["steps"],
            "ms_per_step_median": r64["ms_median"], "steps": r64["steps"],
            "launch_shapes": tuned[0],
            "fp32_speedup": (r64["seconds"] / r64["steps"]) / (r32["seconds"] / r32["steps"])},
        "accuracy": acc,
        "roofline": roof,
        "cpu_baseline": cpu,
        "granular_column": column,
        "size_curve": curve,
        "individual_steps": hsteps,
        "batch_scan": batch,
        "batch_outcomes": outcomes,
        "qrd_campaign": recorded_campaign(),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
