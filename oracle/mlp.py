"""Oracle: the troubled-cell gate network in float64 (numpy).

TEST INFRASTRUCTURE ONLY: tests/, the smoke check and the benchmark's CPU
baseline may import it; the product path never does.

Network (one per dimension): n_in -> 32 -> 32 -> 1, GELU (tanh form,
Hendrycks & Gimpel 2016) after both hidden layers, a logit out: the network as
trained.  (How the GPU's inference evaluates GELU is its own choice; the tests
bound its effect on the logit.)  n_in = 25 in 2D
(the 5 x 5 window of one reconstruction variable around the cell) and 33 in 3D
(the radius-2 sphere S0).  Inputs are the increments W_h - W_c of that variable,
divided by the power of two 2^(e+1) with max|W_h - W_c| in [2^e, 2^(e+1)).

Parameters, one flat float32 vector: W1 [32][n_in], b1 [32], W2 [32][32],
b2 [32], w3 [32], b3 [1].

The GPU runs the two hidden layers as BF16 matrix products with float32
accumulation: inputs, W1, W2 and the first hidden activations are rounded to
BF16.  `bf16=True` applies the same roundings here (round to nearest even);
everything else is float64.  Loss: binary cross-entropy on the logit with a
weight on the positive (troubled) class.
"""
from __future__ import annotations

import numpy as np

H = 32
SQRT_2_OVER_PI = np.sqrt(2.0 / np.pi)


def n_params(n_in: int) -> int:
    return H * n_in + H + H * H + H + H + 1


def unpack(p, n_in):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + H * n_in].reshape(H, n_in); o += H * n_in
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def bf16_round(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(SQRT_2_OVER_PI * (z + 0.044715 * z ** 3)))


def gelu_grad(z):
    t = np.tanh(SQRT_2_OVER_PI * (z + 0.044715 * z ** 3))
    dt = (1.0 - t * t) * SQRT_2_OVER_PI * (1.0 + 3 * 0.044715 * z * z)
    return 0.5 * (1.0 + t) + 0.5 * z * dt


def forward(p, X, bf16=True):
    """Logits [B] and the intermediates needed by backward."""
    X = np.asarray(X, dtype=np.float64)
    n_in = X.shape[1]
    W1, b1, W2, b2, w3, b3 = unpack(p, n_in)
    r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    xr, W1r, W2r = r(X), r(W1), r(W2)
    z1 = xr @ W1r.T + b1
    h1 = gelu(z1)
    h1r = r(h1)
    z2 = h1r @ W2r.T + b2
    h2 = gelu(z2)
    z3 = h2 @ w3 + b3
    return z3, dict(xr=xr, W1r=W1r, W2r=W2r, z1=z1, h1r=h1r, z2=z2, h2=h2, w3=w3)


def loss(z3, y, pos_weight=1.0):
    """Mean weighted BCE with logits: pw y softplus(-z) + (1 - y) softplus(z)."""
    y = np.asarray(y, dtype=np.float64)
    sp_pos = np.logaddexp(0.0, z3)      # softplus(z)
    sp_neg = np.logaddexp(0.0, -z3)     # softplus(-z)
    return float(np.mean(pos_weight * y * sp_neg + (1.0 - y) * sp_pos))


def backward(p, X, y, pos_weight=1.0, bf16=True):
    """Gradient of `loss` with respect to the flat parameters (straight-through
    the BF16 roundings)."""
    z3, c = forward(p, X, bf16)
    B = len(z3)
    y = np.asarray(y, dtype=np.float64)
    s = 1.0 / (1.0 + np.exp(-z3))
    dz3 = (-pos_weight * y * (1.0 - s) + (1.0 - y) * s) / B
    dw3 = c["h2"].T @ dz3
    db3 = dz3.sum()
    dz2 = np.outer(dz3, c["w3"]) * gelu_grad(c["z2"])
    dW2 = dz2.T @ c["h1r"]
    db2 = dz2.sum(0)
    dz1 = (dz2 @ c["W2r"]) * gelu_grad(c["z1"])
    dW1 = dz1.T @ c["xr"]
    db1 = dz1.sum(0)
    return np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dw3, [db3]])


def init_params(n_in: int, seed: int = 0) -> np.ndarray:
    """Glorot-uniform weights, zero biases (float32)."""
    rng = np.random.default_rng(seed)

    def glorot(fan_out, fan_in):
        a = np.sqrt(6.0 / (fan_in + fan_out))
        return rng.uniform(-a, a, size=(fan_out, fan_in))

    p = np.concatenate([glorot(H, n_in).ravel(), np.zeros(H), glorot(H, H).ravel(), np.zeros(H),
                        glorot(1, H).ravel(), [0.0]])
    return p.astype(np.float32)


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba), bias-corrected; returns new (p, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
