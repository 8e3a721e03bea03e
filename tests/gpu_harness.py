"""Shared helpers of the GPU parity tests: run one derivative evaluation of
the strength-SPH step through the C-ABI and bring the results back in the
caller's particle order; error metrics."""
from __future__ import annotations

import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def norm_err(got, ref):
    """max_i |got_i - ref_i| / max_i |ref_i| with per-particle vector norms
    (rows = components)."""
    g = np.atleast_2d(np.asarray(got, dtype=np.float64))
    r = np.atleast_2d(np.asarray(ref, dtype=np.float64))
    d = np.sqrt(((g - r) ** 2).sum(0))
    s = np.sqrt((r ** 2).sum(0)).max()
    if s == 0:
        return float(d.max())
    return float(d.max() / s)


def particle_err(got, ref, scale):
    """Per-particle relative errors |got_i - ref_i| / (|ref_i| + s_i) with
    vector norms over the rows and s_i the oracle's scale of the pair sum
    (the summed magnitudes of its pair contributions).  Returns (median,
    99th percentile, max)."""
    g = np.atleast_2d(np.asarray(got, dtype=np.float64))
    r = np.atleast_2d(np.asarray(ref, dtype=np.float64))
    d = np.sqrt(((g - r) ** 2).sum(0))
    den = np.sqrt((r ** 2).sum(0)) + np.asarray(scale, dtype=np.float64)
    # a particle with no contribution at all (a fixed particle among fixed
    # ones) counts as exact when the result is exactly zero
    e = np.where(den > 0, d / np.where(den > 0, den, 1.0), np.where(d > 0, np.inf, 0.0))
    return float(np.median(e)), float(np.percentile(e, 99)), float(e.max())


def gpu_pair_sets_of(ctx, perm: np.ndarray, targets):
    """Pair sets of the given input indices from the last build, as
    {input index: (sorted input indices j, density flags)}; only the CSR
    rows of the targets are mapped."""
    from paper_2603_19764_amd import sph

    n = perm.size
    off, nbr, dfl = sph.sph_neighbors_csr(ctx, n)
    off = off.cpu().numpy()
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    nbr_d, dfl_d = nbr, dfl
    out = {}
    for t in targets:
        k = int(inv[int(t)])
        a, b = int(off[k]), int(off[k + 1])
        js = perm[nbr_d[a:b].cpu().numpy()]
        fl = dfl_d[a:b].cpu().numpy()
        o = np.argsort(js, kind="stable")
        out[int(t)] = (js[o], fl[o])
    return out


def gpu_derivs(w: dict, prec: int, ctx=None, max_neighbors: int = 128, state=None):
    """One derivative evaluation (neighbour search, density + EOS, stress
    predict with dt = 0, gradients, stress rate, forces) via the C-ABI.

    ``state`` overrides the velocity / energy / stress of ``w`` (predicted
    values).  Returns (dict of numpy arrays in input order, ctx, perm)."""
    import torch
    from paper_2603_19764_amd import sph

    st = dict(w) if state is None else dict(w, **state)
    n = int(np.asarray(st["x"]).size)
    dev = "cuda"
    if ctx is None:
        ctx = sph.Context(max(n, 1), max_neighbors=max_neighbors)
    T = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    x, y, z, h = T(st["x"]), T(st["y"]), T(st["z"]), T(st["h"])
    perm = torch.empty(max(n, 1), dtype=torch.int32, device=dev)[:n]
    sph.sph_build_cells(ctx, x, y, z, h, perm)
    src = [x, y, z, T(st["m"]), h, T(st["u"]), T(st["vx"]), T(st["vy"]), T(st["vz"]),
           T(st["S"]), T(st["mat"], torch.int32), T(st["fixed"], torch.int32)]
    dst = [torch.empty_like(t) for t in src]
    if n:
        sph.sph_reorder(ctx, perm, src, dst)
    sx, sy, sz, sm, sh, su, svx, svy, svz, sS, smat, sfix = dst
    z1 = lambda: torch.zeros(n, dtype=torch.float64, device=dev)
    out = {k: z1() for k in ("rho", "omega", "P", "cs", "T", "Y", "Gmod")}
    sph.sph_density(ctx, sm, sh, su, smat, st["mats"], st["params"], prec, out)
    dt0 = torch.zeros(1, dtype=torch.float64, device=dev)
    Sp = torch.zeros((5, n), dtype=torch.float64, device=dev)
    Sdot = torch.zeros((5, n), dtype=torch.float64, device=dev)
    sph.sph_stress_update(ctx, sph.SPH_STRESS_PREDICT, n, st["params"], dt=dt0, Y=out["Y"],
                          fixed=sfix, S_half=sS, S_pred=Sp, Sdot=Sdot)
    G = torch.zeros((9, n), dtype=torch.float64, device=dev)
    nsing = torch.zeros(1, dtype=torch.int64, device=dev)
    sph.sph_gradients(ctx, svx, svy, svz, sm, sh, out["rho"], out["omega"], st["params"], prec, G,
                      nsing)
    sph.sph_stress_update(ctx, sph.SPH_STRESS_RATE, n, st["params"], G=G, Gmod=out["Gmod"],
                          S_pred=Sp, Sdot=Sdot)
    f = {k: z1() for k in ("ax", "ay", "az", "dudt", "dt")}
    sph.sph_forces_stress(ctx, svx, svy, svz, sm, sh, out["rho"], out["omega"], out["P"],
                          out["cs"], Sp, st["params"], prec, f)
    torch.cuda.synchronize()
    ctx.check(sph.lib().sph_sync_status(ctx.h, None))
    p = perm.cpu().numpy().astype(np.int64)

    def back(t):
        a = t.cpu().numpy()
        o = np.empty_like(a)
        o[..., p] = a
        return o

    res = {k: back(v) for k, v in out.items()}
    res.update(S_pred=back(Sp), dS=back(Sdot), G=back(G), a=back(torch.stack([f["ax"], f["ay"], f["az"]])),
               dudt=back(f["dudt"]), dt=back(f["dt"]), n_singular=int(nsing.item()))
    return res, ctx, p


def gpu_neighbour_sets(ctx, perm: np.ndarray, n: int):
    """Pair sets of the last build as {input index i: (sorted input indices j, dflags)}."""
    from paper_2603_19764_amd import sph

    off, nbr, dfl = sph.sph_neighbors_csr(ctx, n)
    off, nbr, dfl = off.cpu().numpy(), nbr.cpu().numpy(), dfl.cpu().numpy()
    sets = {}
    for k in range(n):
        js = perm[nbr[off[k]:off[k + 1]]]
        fl = dfl[off[k]:off[k + 1]]
        o = np.argsort(js, kind="stable")
        sets[int(perm[k])] = (js[o], fl[o])
    return sets
