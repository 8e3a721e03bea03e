"""The context-free diagnostics entry point (no allocation by the library)
against sph_diagnostics on the same inputs: two calls in a row, the second
on a smaller input, equal bit for bit (same kernels, same partial sums)."""
import numpy as np
import pytest

from paper_2603_19764_amd import inputs
from tests.gpu_harness import say

pytestmark = pytest.mark.gpu


def _fields(n_side, seed):
    w = inputs.c1_block(n_side, variant="s")
    rng = np.random.default_rng(seed)
    n = w["x"].size
    a = rng.normal(0.0, 1e3, (3, n))
    du = rng.normal(0.0, 1e4, n)
    return [w["x"], w["y"], w["z"], w["vx"], w["vy"], w["vz"], w["m"], a[0], a[1], a[2], du]


def test_noalloc_diagnostics_equals_context_diagnostics():
    import torch
    from paper_2603_19764_amd import sph
    out_ctx = torch.zeros(13, dtype=torch.float64, device="cuda")
    out_na = torch.full((13,), np.nan, dtype=torch.float64, device="cuda")
    ctx = sph.Context(20 ** 3, 64)
    for n_side, seed in ((20, 1), (7, 2)):      # the second input is smaller
        say(f"[noalloc diagnostics n={n_side ** 3}]")
        f = [torch.as_tensor(a, dtype=torch.float64, device="cuda") for a in _fields(n_side, seed)]
        sph.sph_diagnostics(ctx, *f, out_ctx)
        sph.sph_diagnostics_noalloc(*f, out_na)
        torch.cuda.synchronize()
        a, b = out_ctx.cpu().numpy(), out_na.cpu().numpy()
        assert np.array_equal(a, b), (a, b)
        assert np.all(np.isfinite(b)) and np.any(b != 0.0)
    # n = 0: all sums zero
    sph.sph_diagnostics_noalloc(*f, out_na, n=0)
    torch.cuda.synchronize()
    assert np.array_equal(out_na.cpu().numpy(), np.zeros(13))
    ctx.check(sph.lib().sph_sync_status(ctx.h, None))


def test_noalloc_rejects_sizes_beyond_the_limit():
    import torch
    from paper_2603_19764_amd import sph
    say("[noalloc limits]")
    f = [torch.zeros(4, dtype=torch.float64, device="cuda") for _ in range(11)]
    out = torch.zeros(13, dtype=torch.float64, device="cuda")
    for n in ((1 << 26) + 1, -1):
        with pytest.raises(sph.SphError) as ei:
            sph.sph_diagnostics_noalloc(*f, out, n=n)
        assert ei.value.code == sph.SPH_EINVAL
        assert "outside" in str(ei.value)
    with pytest.raises(sph.SphError):
        sph.sph_diagnostics_noalloc(*f[:10], None, out)
