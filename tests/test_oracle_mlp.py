"""Pins of the oracle's gate network: its analytic gradient against central
finite differences (float64, no rounding), BF16 rounding against exact cases,
GELU against its closed form at known points, and Adam on a quadratic."""
import math

import numpy as np
import pytest

from oracle import mlp


@pytest.mark.parametrize("n_in", [25, 33])
def test_gradient_matches_finite_differences(n_in):
    rng = np.random.default_rng(1)
    p = mlp.init_params(n_in, seed=3).astype(np.float64)
    p[-1] = 0.3
    X = rng.uniform(-1, 1, size=(40, n_in))
    y = (rng.random(40) < 0.3).astype(float)
    g = mlp.backward(p, X, y, pos_weight=4.0, bf16=False)
    idx = rng.choice(len(p), 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        lp = mlp.loss(mlp.forward(p + e, X, bf16=False)[0], y, 4.0)
        lm = mlp.loss(mlp.forward(p - e, X, bf16=False)[0], y, 4.0)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(fd), (i, fd, g[i])


def test_bf16_rounding():
    # exactly representable values stay; halfway cases round to even
    assert mlp.bf16_round(1.0) == 1.0
    assert mlp.bf16_round(-0.15625) == -0.15625
    one_plus = 1.0 + 2.0 ** -8             # halfway between 1 and 1 + 2^-7
    assert mlp.bf16_round(one_plus) == 1.0
    assert mlp.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2 * 2.0 ** -7
    x = np.random.default_rng(0).normal(size=1000)
    r = mlp.bf16_round(x)
    # 8 significant bits: half an ulp is at most 2^-8 of the value
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x) * (1 + 1e-12))


def test_gelu_known_values():
    assert mlp.gelu(0.0) == 0.0
    # large arguments: identity / zero
    assert abs(mlp.gelu(10.0) - 10.0) < 1e-12 and abs(mlp.gelu(-10.0)) < 1e-12
    # tanh form at x = 1: 0.5 (1 + tanh(sqrt(2/pi) * 1.044715))
    want = 0.5 * (1 + math.tanh(math.sqrt(2 / math.pi) * 1.044715))
    assert abs(mlp.gelu(1.0) - want) < 1e-15
    z = np.linspace(-3, 3, 13)
    fd = (mlp.gelu(z + 1e-6) - mlp.gelu(z - 1e-6)) / 2e-6
    assert np.allclose(mlp.gelu_grad(z), fd, atol=1e-8)


def test_adam_minimises_a_quadratic():
    p = np.array([3.0, -2.0])
    m = v = np.zeros(2)
    for t in range(1, 3001):
        p, m, v = mlp.adam_step(p, 2 * p, m, v, t, lr=0.01)
    assert np.abs(p).max() < 1e-2


def test_gelu_curvature_and_slope_bounds():
    """The constants the GPU gate tests use to bound an approximate GELU's effect
    on the logit: |gelu''| <= 2 phi(0) = 0.7979 (the maximum sits at z = 0) and
    |gelu'| <= 1.13, both of the tanh form, from central differences."""
    z = np.linspace(-12.0, 12.0, 480001)
    h = 1e-4
    g2 = (mlp.gelu(z + h) - 2 * mlp.gelu(z) + mlp.gelu(z - h)) / h ** 2
    assert np.abs(g2).max() <= 2.0 / np.sqrt(2.0 * np.pi) + 1e-5
    assert abs(np.abs(g2).max() - 2.0 / np.sqrt(2.0 * np.pi)) <= 1e-3
    assert np.abs(mlp.gelu_grad(z)).max() <= 1.13
