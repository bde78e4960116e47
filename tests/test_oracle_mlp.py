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


def test_gelu_chords_interpolate_gelu():
    """The inference GELU: exact at the nodes -6 + k/64, linear between them (the
    midpoint is the mean of its ends), within the chord bound h^2/8 max|gelu''|
    (h = 1/64, |gelu''| <= 2 phi(0) = 0.798) of gelu on [-6, 6], and the end
    chords continue outside it (GELU is 0 and z there to 1e-8 at |z| = 6)."""
    k = np.arange(769)
    nodes = -6.0 + k / 64.0
    assert np.abs(mlp.gelu_chords(nodes) - mlp.gelu(nodes)).max() <= 1e-15
    mids = nodes[:-1] + 1.0 / 128.0
    assert np.abs(mlp.gelu_chords(mids) - 0.5 * (mlp.gelu(nodes[:-1]) + mlp.gelu(nodes[1:]))).max() <= 1e-15
    z = np.linspace(-6.0, 6.0, 200001)
    err = np.abs(mlp.gelu_chords(z) - mlp.gelu(z)).max()
    assert err <= (1.0 / 64.0) ** 2 / 8.0 * 2.0 / np.sqrt(2.0 * np.pi) and err > 1e-6
    far = np.array([-40.0, -9.0, 7.0, 30.0])
    assert np.abs(mlp.gelu_chords(far) - np.maximum(far, 0.0)).max() <= 1e-6
    # a network evaluated with chords stays within the chord error's reach of the exact one
    rng = np.random.default_rng(2)
    p = mlp.init_params(25, seed=4)
    X = rng.normal(0.0, 0.3, (512, 25))
    z_exact = mlp.forward(p, X, bf16=False)[0]
    z_chord = mlp.forward(p, X, bf16=False, chords=True)[0]
    w3 = mlp.unpack(p, 25)[4]
    assert 0.0 < np.abs(z_chord - z_exact).max() <= 4 * err * (1.0 + np.abs(w3).sum())
