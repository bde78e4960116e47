"""The learned troubled-cell gate on the GPU against the oracle.

* training kernels: gradients and logits against oracle.mlp (same BF16
  roundings, float64 arithmetic), one Adam step against the oracle's, and loss
  reduction on a synthetic task;
* sample export: network inputs and omega_0 / gamma_0 against the oracle;
* fused inference in the split-precision reconstruction: decisions against
  the oracle network as trained (exact tanh GELU) on the oracle's inputs,
  disagreements allowed only where the exact logit lies within a per-sample
  bound of the threshold (logit_bound: the inference's approximate GELU and
  its float32 arithmetic), and the gated right-hand side against the oracle
  replaying the same decisions.
"""
import numpy as np
import pytest
import torch

from oracle import mlp
from paper_2401_16543_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def K():
    from paper_2401_16543_amd import kfvm
    kfvm.load_library()
    return kfvm


# The inference evaluates GELU approximately: piecewise linear between nodes
# 1/64 apart, the bins centred on k/64 for k = -384 .. 383 (the chord bound
# h^2/8 max|gelu''|, with max|gelu''| = 2 phi(0) <= 0.798 pinned in
# test_oracle_mlp) from float32 node values, the end chords extended beyond
# (GELU is 0 or z there to 1e-8).
GELU_APPROX = (1.0 / 64.0) ** 2 / 8.0 * 0.7979 + 1e-6
GELU_SLOPE = 1.13            # max |gelu'|, pinned in test_oracle_mlp


def _flip_range(v, tol):
    """Largest change of bf16_round(v') over |v' - v| <= tol: zero unless a BF16
    rounding boundary lies within tol of v."""
    return np.abs(mlp.bf16_round(v + tol) - mlp.bf16_round(v - tol))


def logit_bound(p, X):
    """Exact logits (the network as trained, oracle.mlp) and, per sample, a bound
    on how far the GPU's inference logit can lie from them.  Sources: the float32
    rounding of the inputs before their BF16 rounding (a flip moves an input by
    one BF16 step), float32 sums, the approximate GELU of both hidden layers, and
    the BF16 rounding of the first hidden layer, which absorbs a small change
    unless it straddles a rounding boundary.  Each term is carried through
    |W| sums and the GELU slope bound."""
    X = np.asarray(X, dtype=np.float64)
    n_in = X.shape[1]
    z3, c = mlp.forward(p, X, bf16=True)
    W1, b1, W2, b2, w3, b3 = mlp.unpack(p, n_in)
    aW1, aW2, aw3 = np.abs(mlp.bf16_round(W1)), np.abs(c["W2r"]), np.abs(w3)
    dx = _flip_range(X, 1e-7 * np.abs(X) + 1e-12)
    dz1 = dx @ aW1.T + 1e-6 * (1.0 + np.abs(c["xr"]) @ aW1.T + np.abs(b1))
    h1 = mlp.gelu(c["z1"])
    dh1 = GELU_SLOPE * dz1 + GELU_APPROX + 1e-7 * np.abs(c["z1"])
    dh1r = np.maximum(_flip_range(h1, dh1), 0.0)
    dz2 = dh1r @ aW2.T + 1e-6 * (1.0 + np.abs(c["h1r"]) @ aW2.T + np.abs(b2))
    dh2 = GELU_SLOPE * dz2 + GELU_APPROX + 1e-7 * np.abs(c["z2"])
    dz3 = dh2 @ aw3 + 1e-6 * (1.0 + np.abs(c["h2"]) @ aw3 + abs(b3))
    return z3, dz3


def _params(n_in, seed, scale=1.0):
    p = mlp.init_params(n_in, seed=seed).astype(np.float64)
    rng = np.random.default_rng(seed + 1)
    p += 0.05 * rng.normal(size=p.shape)        # nonzero biases
    return (scale * p).astype(np.float32)


@pytest.mark.parametrize("d", [2, 3])
def test_mlp_gradient_matches_oracle(K, d):
    say(f"case mlp gradient d={d}")
    dev = K.KFVM(d, (8,) * d, order=5)
    n_in, P = dev.mlp_sizes()
    assert P == mlp.n_params(n_in)
    rng = np.random.default_rng(7)
    p = _params(n_in, 3)
    # the same BF16-rounded operands on both sides: keep the samples whose first
    # hidden layer lies clear of BF16 rounding boundaries by more than the GPU's
    # float32 arithmetic can move it (the inputs are BF16 values already).  That
    # bound: a float32 chain of n_in + 1 fused multiply-adds errs by at most
    # (n_in + 1) 2^-24 of the sum of its absolute terms (2e-6 covers 33 terms),
    # carried through the GELU slope, plus a few float32 ulps of the GELU itself.
    X = mlp.bf16_round(rng.uniform(-1, 1, size=(4000, n_in))).astype(np.float32)
    c = mlp.forward(p, X, bf16=True)[1]
    W1, b1 = mlp.unpack(p, n_in)[:2]
    h1 = mlp.gelu(c["z1"])
    dz1 = 2e-6 * (np.abs(c["xr"]) @ np.abs(mlp.bf16_round(W1)).T + np.abs(b1))
    keep = np.all(_flip_range(h1, GELU_SLOPE * dz1 + 1e-6 * np.abs(h1)) == 0.0, axis=1)
    X = X[keep][:1000]
    B = len(X)
    assert B >= 800, B
    y = (rng.random(B) < 0.3).astype(np.float32)
    loss, g, logits = dev.mlp_train_step(torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda(),
                                         torch.from_numpy(p).cuda(), lr=0.0, pos_weight=4.0, want_grad=True,
                                         want_logits=True)
    z_ref, _ = mlp.forward(p, X, bf16=True)
    g_ref = mlp.backward(p, X, y, pos_weight=4.0, bf16=True)
    l_ref = mlp.loss(z_ref, y, 4.0)
    ez = np.abs(logits.cpu().numpy() - z_ref).max() / np.abs(z_ref).max()
    eg = np.abs(g.cpu().numpy() - g_ref).max() / np.abs(g_ref).max()
    say(f"  {B} samples: logits rel {ez:.2e}  grad rel {eg:.2e}  loss {loss.item():.6f} vs {l_ref:.6f}")
    assert ez <= 1e-5 and eg <= 1e-5
    assert abs(loss.item() - l_ref) <= 1e-5 * abs(l_ref)


def test_adam_step_and_training(K):
    say("case adam + training")
    d = 2
    dev = K.KFVM(d, (8, 8), order=5)
    n_in, P = dev.mlp_sizes()
    rng = np.random.default_rng(11)
    B = 4096
    X = rng.uniform(-1, 1, size=(B, n_in)).astype(np.float32)
    y = ((X[:, 0] * X[:, 7] > 0.1) | (np.abs(X).max(1) > 0.995)).astype(np.float32)
    p0 = _params(n_in, 5)
    Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    # one Adam step against the oracle's update rule applied to the same gradient
    pd = torch.from_numpy(p0).cuda()
    m, v = torch.zeros_like(pd), torch.zeros_like(pd)
    _, g, _ = dev.mlp_train_step(Xd, yd, pd, lr=0.0, pos_weight=2.0, want_grad=True)
    dev.mlp_train_step(Xd, yd, pd, m, v, t=1, lr=1e-2, pos_weight=2.0)
    p1, _, _ = mlp.adam_step(p0.astype(np.float64), g.cpu().numpy().astype(np.float64), 0.0, 0.0, 1, 1e-2)
    e = np.abs(pd.cpu().numpy() - p1).max()
    say(f"  adam step max diff {e:.2e}")
    assert e <= 2e-5
    # a few hundred steps lower the loss
    first = None
    for t in range(2, 400):
        loss, _, _ = dev.mlp_train_step(Xd, yd, pd, m, v, t=t, lr=3e-3, pos_weight=2.0)
        if first is None:
            first = loss.item()
    last = loss.item()
    say(f"  loss {first:.4f} -> {last:.4f}")
    assert last < 0.6 * first


@pytest.mark.parametrize("d,n", [(2, 24), (3, 10)])
def test_gate_samples_match_oracle(K, oracle_mod, d, n):
    say(f"case samples d={d}")
    U = inputs.cell_averages(inputs.discontinuous(21, d, 4, 10.0, 100.0), n, 1.4, rule="midpoint", q=4)
    orc = oracle_mod.Oracle(d, 2, (n,) * d)
    dev = K.KFVM(d, (n,) * d, order=5)
    x, r = dev.gate_samples(U.cuda())
    x_ref, r_ref = orc.gate_inputs(U.numpy()), orc.omega_ratio(U.numpy())
    ex = np.abs(x.cpu().numpy() - x_ref).max()
    er = np.abs(r.cpu().numpy() - r_ref).max()
    say(f"  x max diff {ex:.2e}  ratio max diff {er:.2e}  troubled frac {(1 - r_ref > 0.5).mean():.3f}")
    assert ex <= 1e-6
    assert er <= 1e-5
    # the labels alone (no input buffer): the same ratios
    x2, r2 = dev.gate_samples(U.cuda(), inputs=False)
    assert x2 is None and torch.equal(r2, r)


@pytest.mark.parametrize("d,R,n", [(2, 2, 48), (2, 3, 48), (3, 2, 16)])
def test_fused_gate_decisions_and_replay(K, oracle_mod, d, R, n):
    say(f"case fused gate d={d} R={R}")
    U = inputs.cell_averages(inputs.discontinuous(23, d, 6 if d == 2 else 4, 10.0, 100.0), n, 1.4,
                             rule="midpoint", q=4)
    orc = oracle_mod.Oracle(d, R, (n,) * d)
    dev = K.KFVM(d, (n,) * d, order=2 * R + 1)
    n_in, _ = dev.mlp_sizes()
    p = _params(n_in, 9, scale=2.0)
    x_ref = orc.gate_inputs(U.numpy()).reshape(-1, n_in)
    z_ref, band = logit_bound(p, x_ref)
    z_ref, band = z_ref.reshape(d + 2, -1), band.reshape(d + 2, -1)
    # S0 increments at rounding level are smooth by definition; these fields have none
    flat = np.zeros((d + 2, x_ref.shape[0] // (d + 2)), dtype=bool)
    thr = float(np.median(z_ref))
    dev.set_precision("split_f16")
    dev.set_gate(torch.from_numpy(p).cuda(), thr)
    dev.set_checking(True)
    Ud = U.cuda()
    L = dev.rhs(Ud).cpu().numpy()
    flags = dev.get_flags().cpu().numpy()
    want = ((z_ref > thr) & ~flat).astype(np.uint8)
    bad = flags != want
    near = np.abs(z_ref - thr) <= band
    say(f"  flagged {flags.mean():.3f}  disagreements {int(bad.sum())} (all within the bound of the threshold: "
        f"{bool(np.all(near[bad]))}; median bound {np.median(band):.1e})")
    assert np.all(near[bad]) and bad.mean() <= 0.01
    # the oracle replaying the GPU's decisions
    orc.set_flags(flags)
    ref = orc.rhs(U.numpy())
    nv = d + 2
    e = max(np.abs(L[k] - ref[k]).max() / np.abs(ref[k]).max() for k in range(nv))
    say(f"  gated rhs rel err {e:.2e}")
    assert e <= 2e-5


# (case, largest fraction of (variable, cell) pairs left on WENO-AO): the 64^2
# vortex is resolved by ~3 cells per core radius and keeps most of its core
# pairs on WENO-AO; variables at rounding level (the wave's velocity and
# pressure) count as smooth
@pytest.mark.parametrize("case,max_weno", [("3d_density_wave", 0.1), ("2d_vortex", 0.75)])
def test_gate_gain_on_exact_solution(K, case, max_weno):
    """What the trained gate gains over the method without it, on problems with
    an exact solution: the cells it marks smooth skip the WENO-AO work, and the
    density error against the exact cell averages stays at or below that of
    the plain FP64 WENO-AO path."""
    from paper_2401_16543_amd import gate
    say(f"case gate gain {case}")
    if case == "3d_density_wave":
        d, n, gamma, steps, vel = 3, 64, 5.0 / 3.0, 40, (0.5, 0.3, -0.2)
        spec = lambda t: inputs.density_wave(31, d, 6, vel, t)
        dx = 1.0 / n
    else:
        d, n, gamma, steps = 2, 64, 1.4, 80
        spec = lambda t: inputs.isentropic_vortex(gamma, t)
        dx = 20.0 / n
    U0 = inputs.cell_averages(spec(0.0), n, gamma, rule="gauss", q=4, device="cuda")
    plain = K.KFVM(d, (n,) * d, dx=[dx] * d, order=5, gamma=gamma)
    gated = K.KFVM(d, (n,) * d, dx=[dx] * d, order=5, gamma=gamma)
    gated.set_precision("split_f16")
    params, thr, _ = gate.load(d)
    gated.set_gate(torch.from_numpy(params).cuda(), thr)
    dt = plain.cfl_dt(U0, 0.4)
    Up, Ug = U0.clone(), U0.clone()
    flagged = 0.0
    for _ in range(steps):
        plain.step(Up, dt)
        gated.step(Ug, dt)
        flagged += float(gated.get_flags().float().mean()) / steps
    Ue = inputs.cell_averages(spec(steps * dt), n, gamma, rule="gauss", q=4, device="cuda")
    ep = float((Up[0] - Ue[0]).abs().mean())
    eg = float((Ug[0] - Ue[0]).abs().mean())
    say(f"  t={steps * dt:.4f}: L1 rho error plain FP64 {ep:.3e}, mixed+gate {eg:.3e}, "
        f"WENO-AO on {flagged:.4f} of (variable, cell) pairs")
    assert gated.status() == K.KFVM_OK and plain.status() == K.KFVM_OK
    assert eg <= 1.05 * ep
    assert flagged < max_weno


def test_gate_dilated_for_3d_order7(K, oracle_mod):
    """3D order 7: the network runs in its own kernel on the radius-2 sphere and a
    variable takes WENO-AO where any cell of the 3^3 block is marked troubled (the
    radius-3 stencil reaches one cell past the inputs).  Decisions against the
    oracle network as trained, dilated the same way (disagreements only next to
    exact logits within logit_bound of the threshold); the RHS against the oracle
    replaying the GPU's decisions."""
    say("case gate 3D order 7")
    d, R, n = 3, 3, (16, 16, 12)
    U = inputs.cell_averages(inputs.discontinuous(29, d, 4, 10.0, 100.0), 16, 1.4, rule="midpoint", q=4)
    U = U[:, :n[2], :n[1], :n[0]].contiguous()
    dx = [1.0 / 16] * d
    orc = oracle_mod.Oracle(d, R, n, dx=dx)
    dev = K.KFVM(d, n, dx=dx, order=7)
    n_in, _ = dev.mlp_sizes()
    p = _params(n_in, 13, scale=2.0)
    x_ref = orc.gate_inputs(U.numpy()).reshape(-1, n_in)
    z, band = logit_bound(p, x_ref)
    z, band = z.reshape(d + 2, n[2], n[1], n[0]), band.reshape(d + 2, n[2], n[1], n[0])
    thr = float(np.quantile(z, 0.85))
    near = np.abs(z - thr) <= band
    want = np.zeros(z.shape, dtype=bool)
    close = np.zeros(z.shape, dtype=bool)
    for oz in (-1, 0, 1):
        for oy in (-1, 0, 1):
            for ox in (-1, 0, 1):
                want |= np.roll(z > thr, (oz, oy, ox), axis=(1, 2, 3))
                close |= np.roll(near, (oz, oy, ox), axis=(1, 2, 3))
    dev.set_precision("split_f16")
    dev.set_gate(torch.from_numpy(p).cuda(), thr)
    dev.set_checking(True)
    L = dev.rhs(U.cuda()).cpu().numpy()
    flags = dev.get_flags().cpu().numpy().reshape(z.shape)
    bad = flags.astype(bool) != want
    say(f"  WENO-AO on {flags.mean():.3f}  disagreements {int(bad.sum())} (all next to near-threshold logits: "
        f"{bool(np.all(close[bad]))})")
    assert np.all(close[bad]) and bad.mean() <= 0.02
    orc.set_flags(flags.reshape(d + 2, -1))
    ref = orc.rhs(U.numpy())
    e = max(np.abs(L[k] - ref[k]).max() / np.abs(ref[k]).max() for k in range(d + 2))
    say(f"  gated rhs rel err {e:.2e}")
    assert e <= 2e-5
