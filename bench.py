"""Benchmark of the strength-SPH step on one MI355X.

Workload: the granular column (196,794 mobile particles in a 0.2 x 0.1 x 0.05 m
block on a 4-layer floor of 29,928 fixed particles, cubic lattice spacing
1.70998 mm, h = 1.3 spacing, Drucker-Prager friction tan 30 deg, g = 9.81),
advanced with the FP32 cell-relative pair arithmetic; the same steps in the
plain FP64 path are timed next to it.  One step = neighbour search (cell
sort + pair sets), reorder of the state, predictor, density + EOS + yield,
stress predict and rescale, corrected gradients, stress rate, forces, CFL
minimum, kicks.  Metric: ordered neighbour pairs per second,
sum_steps sum_i |N_i| / wall time.

Prints one JSON line.  ``--gpus N`` with N > 1 is not supported (one GPU).
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

PEAK_FP32_VALU = 157.3e12   # MI355X FP32 vector, published
PEAK_FP64_VALU = 78.6e12    # MI355X FP64 vector, published
PEAK_HBM = 8.0e12

# Algorithmic flops per ordered pair of the fused gradient + force sweep of
# the step (FMA = 2, sqrt = 1), counted from the pair term without the
# artificial-viscosity branch: separation (9 in float incl. the cell shift,
# 3 in double), r^2 (5), sqrt (1), kernel factors t_i^3, t_j^3 (8), v_ij (3);
# force part: (K A)_i x and (K A)_j x (30), momentum sum (15), energy term
# (8), v_ij . x_ij (5); gradient part: pair weight (5), w x_ij (3),
# C^-1 sums (12), F sums (18).
FLOPS_PAIR = {1: 122, 0: 116}


# Measured HBM traffic of the dominant pair kernel (rocprofv3 FETCH_SIZE and
# WRITE_SIZE per dispatch, scaled by the same counters on a plain copy of
# known size).  Valid only for the kernel source it was taken on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_grad_forces_c2_fp32_traffic.md")
TRAFFIC_SOURCES = ("paper_2603_19764_amd/csrc/pairs.hip", "paper_2603_19764_amd/csrc/device_util.h",
                   "paper_2603_19764_amd/csrc/records.h")


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
    """Bytes per launch of ``kernel`` (e.g. "k_grad_forces<4,fp32>") from the
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


def run_steps(w, prec, steps, warmup, use_graph, timing=True, tuned=None):
    import torch
    from paper_2603_19764_amd import autotune, sph

    n = int(w["x"].size)
    ctx = sph.Context(n, max_neighbors=128, max_cells=1 << 22)
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
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if use_graph:
        for _ in range(steps // 2):
            graph.replay()
    else:
        for _ in range(steps):
            sph.sph_step(ctx, st, mats, prm, prec)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    p1 = sph.sph_pair_count(ctx)
    ctx.check(sph.lib().sph_sync_status(ctx.h, None))
    k_steps = (steps // 2) * 2 if use_graph else steps
    kern = {}
    if timing and not use_graph:
        for name, kid in (("build", 0), ("density", 1), ("grad_forces", 3)):
            kern[name] = sph.sph_timing_read(ctx, kid)
        sph.sph_timing(ctx, False)
    out = dict(seconds=t1 - t0, steps=k_steps, pairs=p1 - p0, kernels=kern, n=n)
    del graph
    ctx.close()
    return out


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
            r = run_steps(w, prec, steps, warmup, False, timing=False)
            row[name] = {"pairs_per_s": r["pairs"] / r["seconds"],
                         "ms_per_step": 1e3 * r["seconds"] / r["steps"]}
        log(f"curve {k}^3: {row}")
        out.append(row)
    return out


def run_impact_step(steps=4, warmup=2):
    """The two-sphere impact (about 1.1M particles, glass-like bodies, 45 deg,
    3 km/s, gravity excluded): whole steps in FP32 and in FP64."""
    from paper_2603_19764_amd import inputs
    w = inputs.c3_impact()
    row = {"particles": int(w["x"].size)}
    for prec, name in ((1, "fp32"), (0, "fp64")):
        r = run_steps(w, prec, steps, warmup, False, timing=False)
        row[name] = {"pairs_per_s": r["pairs"] / r["seconds"],
                     "ms_per_step": 1e3 * r["seconds"] / r["steps"],
                     "pairs_per_step": r["pairs"] / r["steps"]}
    log(f"impact: {row}")
    return row


def run_hsteps(n_side=64, prec=1, shared_steps=600):
    """Individual time steps against one shared step on a block with a hot
    core: a 64^3 lattice block (the spacing, jitter and shear flow of the
    single-step block) whose central sphere of a fifth of its edge carries
    u = 3e6 J/kg.  The shared step runs ``shared_steps`` steps (it follows
    the particle with the shortest CFL step); the rungs (base step: the
    longest CFL step at the start) then run to the same simulated time.
    Figure of merit: wall time to that simulated time."""
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
    for mode in ("shared", "rungs"):
        prm = dict(w["params"])
        if mode == "rungs":
            prm["rungs"] = 8
        ctx = sph.Context(n, 128, max_cells=1 << 22)
        st = sph.State(w, dt_max=dt0 if mode == "rungs" else 0.0)
        sph.sph_init(ctx, st, w["mats"], prm, prec)
        if mode == "shared":
            torch.cuda.synchronize()
            dt0 = float(st.wrow(sph.SPH_W_DT).max()) * 1.01
        sim = torch.zeros(1, dtype=torch.float64, device="cuda")
        k = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while True:
            for _ in range(20):
                sim += st.dt
                sph.sph_step(ctx, st, w["mats"], prm, prec)
            k += 20
            if mode == "shared" and k >= shared_steps:
                break
            if mode == "rungs" and float(sim.item()) >= t_target:
                break
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.check(sph.lib().sph_sync_status(ctx.h, None))
        row = {"steps": k, "wall_s": t1 - t0, "ms_per_step": 1e3 * (t1 - t0) / k,
               "simulated_s": float(sim.item())}
        if mode == "shared":
            t_target = row["simulated_s"]
        else:
            steps = st.row(sph.SPH_DTP).cpu().numpy()
            vals, cnt = np.unique(steps, return_counts=True)
            row["base_step_s"] = dt0
            row["particles_per_step_ticks"] = {str(int(v)): int(q) for v, q in zip(vals, cnt)}
        out[mode] = row
        ctx.close()
    out["speedup"] = (out["shared"]["wall_s"] / out["shared"]["simulated_s"]) / (
        out["rungs"]["wall_s"] / out["rungs"]["simulated_s"])
    log(f"individual steps: {out}")
    return out


def cpu_baseline(w, budget_s=15.0):
    """The FP64 oracle on a bounded sample of the same workload: the full
    derivative chain (brute-force pair sets, density + EOS for the pair-set
    closure, gradients, stress rate, forces) for randomly chosen target
    particles.  Rate = ordered pairs of the targets per second."""
    from oracle import oracle

    st = {k: w[k] for k in ("x", "y", "z", "m", "h", "mat", "vx", "vy", "vz", "u", "S")}
    n = w["x"].size
    rng = np.random.default_rng(123)
    oracle.lib()
    ntar = 8
    t_used = 0.0
    while True:
        tar = np.sort(rng.choice(n, ntar, replace=False))
        t0 = time.perf_counter()
        oracle.derivs(st, w["mats"], w["params"], tar)
        dt = time.perf_counter() - t0
        if dt > 0.25 * budget_s or ntar >= n:
            break
        t_used += dt
        ntar = int(min(n, ntar * max(2.0, min(8.0, 0.5 * budget_s / max(dt, 1e-3)))))
    off, _, _ = oracle.pair_lists(w["x"], w["y"], w["z"], w["h"], w["params"], tar)
    pairs = int(off[-1])
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    model = "unknown CPU"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(value=pairs / dt, unit="pairs/s", cores=threads, kind="oracle",
                sample=f"{model}, {threads} threads: "
                       f"{ntar} random targets of the {n}-particle column, full FP64 derivative "
                       f"chain with brute-force O(N^2) neighbour search, {pairs} target pairs in "
                       f"{dt:.2f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--graph", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-curve", action="store_true",
                    help="skip the size curve (block workload, 32^3 to 160^3)")
    ap.add_argument("--no-hsteps", action="store_true",
                    help="skip the individual-step comparison on the hot-core block")
    ap.add_argument("--no-impact", action="store_true",
                    help="skip the 1.1M-particle two-sphere impact steps")
    ap.add_argument("--batch-steps", type=int, default=20,
                    help="steps of the batched 64-impact scan (0: skip it)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default launch shapes (no autotuning before the warmup)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device to device (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2603_19764_amd import inputs

    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
    w = inputs.c2_column()
    log(f"workload {w['name']}: n={w['x'].size}")
    tuned = {0: None, 1: None}
    if not args.no_tune:
        from paper_2603_19764_amd import autotune
        for prec in ((1,) if args.no_fp64 else (1, 0)):
            t = autotune.tune(w, prec, steps=3)
            tuned[prec] = t["settings"]
            log(f"autotune prec {prec}: {t['settings']} {t['times_ms']}")
    r32 = run_steps(w, 1, args.steps, args.warmup, bool(args.graph), tuned=tuned[1])
    log(f"fp32: {r32['seconds']:.3f} s for {r32['steps']} steps, {r32['pairs']} pairs")
    r64 = None
    if not args.no_fp64:
        r64 = run_steps(w, 0, max(args.steps // 4, 2), args.warmup, bool(args.graph),
                        tuned=tuned[0])
        log(f"fp64: {r64['seconds']:.3f} s for {r64['steps']} steps, {r64['pairs']} pairs")
    value = r32["pairs"] / r32["seconds"]
    ms_step = 1e3 * r32["seconds"] / r32["steps"]
    roof = None
    if r32["kernels"]:
        ms, cnt = r32["kernels"]["grad_forces"]
        avg_s = ms / cnt * 1e-3
        pairs_per_launch = r32["pairs"] / r32["steps"]
        achieved = FLOPS_PAIR[1] * pairs_per_launch / avg_s
        kname = f"k_grad_forces<{(tuned[1] or {}).get('lanes_step', 8)},fp32>"
        roof = dict(bound="alu", achieved=achieved / 1e12, peak=PEAK_FP32_VALU / 1e12,
                    unit="TFLOP/s", frac=achieved / PEAK_FP32_VALU,
                    traffic=measured_traffic(kname), kernel=kname,
                    avg_launch_us=avg_s * 1e6,
                    kernels_us={k: (v[0] / v[1] * 1e3 if v[1] else None)
                                for k, v in r32["kernels"].items()})
    curve = None if args.no_curve else run_curve()
    impact = None if args.no_impact else run_impact_step()
    hsteps = None if args.no_hsteps else run_hsteps()
    batch = None
    if args.batch_steps > 0:
        batch = run_batch(args.batch_steps, 4, tune=not args.no_tune)
        log(f"batch: {batch['ms_per_step']:.3f} ms/step, {batch['value']:.3e} pairs/s")
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w)
    line = {
        "metric": "SPH strength-step pair interactions/s (FP32 vs FP64 plain, 1 GPU) at 1e-5 rel err",
        "value": value, "unit": "pairs/s", "n_gpus": 1, "steps": r32["steps"],
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 pair terms, f64 state",
        "data": "synthetic",
        "config": {"workload": "granular column collapse, 196794 mobile + 29928 fixed particles, "
                               "FP32 cell-relative pair loop, Drucker-Prager tan 30, g = 9.81",
                   "particles": r32["n"], "pairs_per_step": r32["pairs"] / r32["steps"],
                   "graph": bool(args.graph), "launch_shapes": tuned[1]},
        "fp64_plain": None if r64 is None else {
            "value": r64["pairs"] / r64["seconds"], "ms_per_step": 1e3 * r64["seconds"] / r64["steps"],
            "steps": r64["steps"], "launch_shapes": tuned[0]},
        "size_curve": curve,
        "impact_1p1M": impact,
        "individual_steps": hsteps,
        "batch_scan": batch,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
