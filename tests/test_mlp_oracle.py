"""Pins of the FP64 network oracle: the analytic backward pass against central
finite differences, and the Adam step against its closed form."""
import numpy as np

from oracle import mlp_oracle as mo


def test_parameter_count():
    assert mo.N_PARAMS == 4545
    assert mo.init_params(0).size == 4545


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = mo.init_params(3) + rng.normal(0, 0.05, mo.N_PARAMS)
    X = rng.normal(0, 1, (37, 4))
    Y = rng.uniform(0, 1, 37)
    g = mo.backward(p, X, Y)
    idx = np.concatenate([rng.choice(mo.N_PARAMS, 60, replace=False), [mo.N_PARAMS - 1, 0, 256]])
    for k in idx:
        e = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[k] += e
        pm[k] -= e
        fd = (mo.loss(pp, X, Y) - mo.loss(pm, X, Y)) / (2 * e)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (k, fd, g[k])


def test_adam_first_step_closed_form():
    """With zero moments the first bias-corrected step is lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p = np.zeros(4)
    p1, m, v = mo.adam_step(p, g, np.zeros(4), np.zeros(4), 1, lr=0.01, eps=1e-8)
    np.testing.assert_allclose(p1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_forward_output_range_and_saturation():
    p = mo.init_params(0)
    w = mo.unpack(p)
    w["b3"][0] = 50.0  # view into p
    out, h1, h2 = mo.forward(p, np.zeros((3, 4)))
    assert np.all(out > 1 - 1e-12)
    assert h1.shape == (3, 64) and h2.shape == (3, 64)
