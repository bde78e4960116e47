"""The split-precision (matrix-core) path against the FP64 oracle.

Its bar is accuracy, not bit parity: the contractions run on FP16/BF16 hi/lo
operands with FP32 accumulation.  Right-hand sides are compared relative to the
largest magnitude per variable; trajectories by the L1 density difference."""

import numpy as np
import pytest
import torch

from paper_2401_16543_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def rel_err(a, b):
    nv = a.shape[0]
    a, b = np.asarray(a).reshape(nv, -1), np.asarray(b).reshape(nv, -1)
    return max(float(np.abs(a[k] - b[k]).max() / np.abs(b[k]).max()) for k in range(nv))


@pytest.fixture(scope="module")
def K():
    from paper_2401_16543_amd import kfvm
    kfvm.load_library()
    return kfvm


def _U(kind, d, n, seed):
    if kind == "smooth":
        return inputs.cell_averages(inputs.smooth(seed, d, 8), n, 1.4, rule="gauss", q=3)
    return inputs.cell_averages(inputs.discontinuous(seed, d, 6 if d == 2 else 4, 10.0, 100.0), n, 1.4,
                                rule="midpoint", q=4)


# (d, R, n, kind, mode, rhs tolerance, states tolerance): a hi/lo pair of FP16
# values carries ~22 significant bits (BF16: ~16) of each operand, relative to
# the largest increment of the cell; the 122-point rows of 3D R = 3 cancel more
# (sum |w delta| over |sum w delta|), so their smooth-data bound is wider
MIXED = [
    (2, 2, (64, 64), "smooth", "split_f16", 2e-6, 2e-7),
    (2, 2, (37, 29), "jumps", "split_f16", 2e-5, 2e-6),
    (2, 2, (48, 40), "jumps", "split_bf16", 2e-2, 2e-3),
    (2, 3, (40, 36), "jumps", "split_f16", 2e-5, 2e-6),
    (3, 2, (16, 16, 16), "smooth", "split_f16", 2e-6, 5e-7),
    (3, 2, (13, 11, 9), "jumps", "split_f16", 2e-5, 2e-6),
    (3, 2, (16, 12, 10), "jumps", "split_bf16", 2e-2, 2e-3),
    (3, 3, (16, 16, 16), "smooth", "split_f16", 5e-6, 5e-6),
    (3, 3, (13, 11, 10), "jumps", "split_f16", 2e-5, 1e-5),
    (3, 3, (16, 12, 9), "jumps", "split_bf16", 2e-2, 2e-3),
]


@pytest.mark.parametrize("d,R,n,kind,mode,tol_rhs,tol_st", MIXED)
def test_mixed_rhs_close_to_oracle(K, oracle_mod, d, R, n, kind, mode, tol_rhs, tol_st):
    say(f"case mixed d={d} R={R} n={n} {kind} {mode}")
    U = _U(kind, d, max(n), 300 + d * 10 + R)
    sl = (slice(None),) + tuple(slice(0, x) for x in reversed(n))
    U = U[sl].contiguous()
    dx = [1.0 / max(n)] * d
    orc = oracle_mod.Oracle(d, R, n, dx=dx)
    ref, ref_st = orc.rhs(U.numpy()), orc.states(U.numpy())
    dev = K.KFVM(d, n, dx=dx, order=2 * R + 1)
    dev.set_precision(mode)
    dev.set_checking(True)
    Ud = U.cuda()
    got = dev.rhs(Ud).cpu().numpy()
    st = dev.face_states(Ud).cpu().numpy()
    e_st = rel_err(np.moveaxis(st, -1, 0), np.moveaxis(ref_st, -1, 0))
    e_rhs = rel_err(got, ref)
    say(f"  states rel err {e_st:.3e}  rhs rel err {e_rhs:.3e}")
    assert e_st <= tol_st
    assert e_rhs <= tol_rhs


@pytest.mark.parametrize("d,R,mode", [(2, 2, "fp64"), (2, 2, "split_f16"), (3, 3, "fp64"), (3, 3, "split_f16")])
def test_gate_flags_replay(K, oracle_mod, d, R, mode):
    """Flags choose WENO-AO or the linear S0 value per (variable, cell); the oracle
    replays the same decisions.  Whole waves (and, in 3D, whole blocks) are linear
    or WENO-AO, the rest mixed at random."""
    say(f"case flags d={d} R={R} {mode}")
    n = (48, 48) if d == 2 else (16, 16, 12)
    ncell = int(np.prod(n))
    U = _U("jumps", d, max(n), 17)
    U = U[(slice(None),) + tuple(slice(0, x) for x in reversed(n))].contiguous()
    rng = np.random.default_rng(2)
    flags = (rng.random((d + 2, ncell)) < 0.3).astype(np.uint8)
    plane = n[0] * n[1] if d == 3 else n[0]
    flags[:, : 4 * plane] = 0                   # whole waves (3D: whole blocks) linear
    flags[:, 4 * plane: 8 * plane] = 1          # whole waves WENO
    dx = [1.0 / max(n)] * d
    orc = oracle_mod.Oracle(d, R, n, dx=dx)
    orc.set_flags(flags)
    ref = orc.rhs(U.numpy())
    dev = K.KFVM(d, n, dx=dx, order=2 * R + 1)
    dev.set_precision(mode)
    dev.set_checking(True)
    fl = torch.from_numpy(flags).cuda()
    dev.set_flags(fl)
    got = dev.rhs(U.cuda()).cpu().numpy()
    e = rel_err(got, ref)
    say(f"  rel err {e:.3e}")
    assert e <= (1e-12 if mode == "fp64" else 1e-5)


@pytest.mark.parametrize("name,mode,tol,gated", [("3d_smooth_256", "split_f16", 2e-6, False),
                                                  ("3d_smooth_256", "split_f16", 2e-6, True),
                                                  ("2d_jumps_1024", "split_bf16", 2e-2, False),
                                                  ("2d_jumps_1024", "split_f16", 2e-5, True)])
def test_mixed_full_size_sampled(K, oracle_mod, name, mode, tol, gated):
    """Full-size workloads in the benchmark's launch configuration: the
    split-precision RHS over the whole grid (with the trained gate, the oracle
    replaying its decisions) against the oracle at sampled cells, and
    conservation.  Face-buffer offsets pass 2^31 bytes here."""
    from paper_2401_16543_amd import gate
    say(f"case mixed full-size {name} {mode} gated={gated}")
    U, cfg = inputs.config_state(name, device="cuda")
    d, n, R, gamma = cfg["d"], cfg["n"], cfg["R"], cfg["gamma"]
    dev = K.KFVM(d, (n,) * d, order=2 * R + 1, gamma=gamma)
    dev.set_precision(mode)
    dev.set_checking(True)
    if gated:
        params, thr, _ = gate.load(d)
        dev.set_gate(torch.from_numpy(params).cuda(), thr)
    L = dev.rhs(U)
    torch.cuda.synchronize()
    Lh = L.cpu().numpy().reshape(d + 2, -1)
    Uh = U.cpu().numpy()
    ncell = n ** d
    rng = np.random.default_rng(8)
    cells = np.concatenate([[0, ncell - 1, n - 1, ncell - n], rng.integers(0, ncell, 160 if d == 3 else 600)])
    orc = oracle_mod.Oracle(d, R, (n,) * d, gamma=gamma)
    if gated:
        flags = dev.get_flags().cpu().numpy()
        say(f"  flagged {flags.mean():.4f}")
        orc.set_flags(flags)
    ref = orc.rhs_cells(Uh, cells)
    err = (np.abs(Lh[:, cells].T - ref) / np.abs(Lh).max(axis=1)).max()
    say(f"  sampled rel err {err:.3e}")
    assert err <= tol
    tot = np.abs(Lh.sum(axis=1)) / np.abs(Lh).sum(axis=1)
    assert np.all(tot <= 1e-13)


def test_mixed_trajectory_smooth_l1(K):
    """10 SSP-RK3 steps of the 64^2 smooth workload: L1 density difference between
    the split-FP16 and FP64 paths stays far below 1e-8."""
    say("case mixed trajectory")
    U0, cfg = inputs.config_state("2d_smooth_64")
    d, n = cfg["d"], cfg["n"]
    a = K.KFVM(d, (n, n), order=5, gamma=cfg["gamma"])
    b = K.KFVM(d, (n, n), order=5, gamma=cfg["gamma"])
    b.set_precision("split_f16")
    Ua, Ub = U0.cuda(), U0.cuda().clone()
    for _ in range(cfg["steps"]):
        dt = a.cfl_dt(Ua, cfg["cfl"])
        a.step(Ua, dt)
        b.step(Ub, dt)
    l1 = float((Ua[0] - Ub[0]).abs().mean())
    say(f"  L1 rho diff {l1:.3e}")
    assert l1 <= 1e-9


@pytest.mark.parametrize("d,R,n", [(2, 3, (32, 32)), (3, 2, (16, 16, 16)), (3, 3, (16, 16, 12))])
def test_mixed_limiter_engaged(K, oracle_mod, d, R, n):
    """Strong jumps (density ratios to 100, pressure ratios to 1000) and kappa =
    0.1 so the positivity limiter acts: the split path's running-bound limiter
    (exact per-point fallback) against the oracle's per-point limiter."""
    say(f"case mixed limiter d={d} R={R} n={n}")
    gamma = 1.4
    U = inputs.cell_averages(inputs.discontinuous(9, d, 6 if d == 2 else 4, 100.0, 1000.0), max(n), gamma,
                             rule="midpoint", q=4 if d == 2 else 2)
    U = U[(slice(None),) + tuple(slice(0, x) for x in reversed(n))].contiguous()
    dx = [1.0 / max(n)] * d
    orc = oracle_mod.Oracle(d, R, n, dx=dx, gamma=gamma, kappa=0.1)
    free = oracle_mod.Oracle(d, R, n, dx=dx, gamma=gamma, limiter=False).states(U.numpy())
    ref_states = orc.states(U.numpy())
    assert np.abs(free - ref_states).max() > 1e-6          # the limiter acted
    dev = K.KFVM(d, n, dx=dx, order=2 * R + 1, gamma=gamma)
    dev.set_precision("split_f16")
    dev.set_limiter(True, 0.1)
    dev.set_checking(True)
    Ud = U.cuda()
    st = dev.face_states(Ud).cpu().numpy()
    e_st = rel_err(np.moveaxis(st, -1, 0), np.moveaxis(ref_states, -1, 0))
    e_rhs = rel_err(dev.rhs(Ud).cpu().numpy(), orc.rhs(U.numpy()))
    say(f"  states rel err {e_st:.3e}  rhs rel err {e_rhs:.3e}")
    assert e_st <= 2e-5 and e_rhs <= 2e-5


def test_mixed_hll(K, oracle_mod):
    """The HLL option in the split path (the Riemann solver itself is float64)."""
    say("case mixed hll")
    d, R, n = 2, 2, (40, 36)
    U = _U("jumps", d, 40, 23)[:, :n[1], :n[0]].contiguous()
    dx = [1.0 / 40] * d
    orc = oracle_mod.Oracle(d, R, n, dx=dx, riemann="hll")
    dev = K.KFVM(d, n, dx=dx, order=5)
    dev.set_precision("split_f16")
    dev.set_riemann("hll")
    dev.set_checking(True)
    e = rel_err(dev.rhs(U.cuda()).cpu().numpy(), orc.rhs(U.numpy()))
    say(f"  rhs rel err {e:.3e}")
    assert e <= 2e-5


@pytest.mark.parametrize("d,R,mode,gated", [(2, 2, "split_f16", False), (2, 2, "split_f16", True),
                                              (3, 2, "split_f16", False), (3, 2, "split_bf16", True),
                                              (3, 3, "split_f16", False), (3, 3, "split_f16", True)])
def test_mixed_tiny_increments_stay_finite(K, oracle_mod, d, R, mode, gated):
    """Ahead of a wave front the increments of a quiescent state decay to float64
    denormals (seen on the tilted Sod tube: 6e-314 in the momentum).  The per-cell
    scale 2^(SB - e) must stay finite there: a uniform state at rest with
    momentum perturbations of 1e-36 (below float32's normal range) and 6e-314 in a
    few cells gives a finite RHS equal to the FP64 one to the path's tolerance."""
    from paper_2401_16543_amd import gate
    say(f"case tiny increments d={d} R={R} {mode} gated={gated}")
    n = (16,) * d
    U = np.zeros((d + 2,) + n)
    U[0] = 0.125
    U[d + 1] = 0.25
    idx = tuple(slice(3, 6) for _ in range(d))
    U[(1,) + idx] = 6e-314
    U[(d,) + tuple(slice(9, 12) for _ in range(d))] = -1e-36
    U = torch.from_numpy(U)
    ref = oracle_mod.Oracle(d, R, n).rhs(U.numpy())
    dev = K.KFVM(d, n, order=2 * R + 1)
    dev.set_precision(mode)
    dev.set_checking(True)
    if gated:
        params, thr, _ = gate.load(d)
        dev.set_gate(torch.from_numpy(params).cuda(), thr)
    got = dev.rhs(U.cuda()).cpu().numpy()
    assert np.isfinite(got).all()
    # the RHS is at rounding level of the state (1e-16 x 0.25 / dx), the tiny
    # momenta below it: compare absolutely
    err = np.abs(got - ref).max()
    say(f"  max |rhs - oracle| {err:.3e}")
    assert err <= 1e-12
