"""Every workload at its full size and step count: the L1 density difference
between the reduced-precision paths and the FP64 path, against the targets
(at most 1e-8 on smooth data, at most 1e-4 on discontinuous data).

The FP64 GPU path is the reference of these trajectories: it matches the CPU
oracle to 1e-12 per right-hand side on every workload at full size (sampled
cells, test_gpu_parity.py::test_full_size_sampled), and the oracle is far too
slow for the trajectories themselves.  All runs start from the same state and
take the FP64 path's dt sequence (CFL 0.4).

With the learned gate two figures are taken:
* same decisions: the FP64 path replays the gated run's decisions at every
  stage (accuracy.replay_l1), so the difference is the precision error alone;
  the targets bind this one;
* against FP64 WENO-AO everywhere: precision plus the scheme change of the
  decisions (linear S0 where the gate says smooth), reported, and held to the
  discontinuous-data bar where the workload has jumps.
The gated right-hand sides at full size are also checked against the oracle
replaying the gate's decisions, at sampled cells.
"""
import numpy as np
import pytest
import torch

from paper_2401_16543_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def K():
    from paper_2401_16543_amd import kfvm
    kfvm.load_library()
    return kfvm


def _ctx(K, cfg, mode="fp64", gated=False):
    from paper_2401_16543_amd import gate
    d, n, R = cfg["d"], cfg["n"], cfg["R"]
    dev = K.KFVM(d, (n,) * d, order=2 * R + 1, gamma=cfg["gamma"])
    dev.set_precision(mode)
    if gated:
        params, thr, _ = gate.load(d)
        dev.set_gate(torch.from_numpy(params).cuda(), thr)
    return dev


def _trajectories(K, name, runs, steps=None):
    """FP64 and each (mode, gated) of `runs` advanced by kfvm_step from the
    workload's state; returns (L1 of rho per run, FP64 dt sequence, FP64 state)."""
    U0, cfg = inputs.config_state(name, device="cuda")
    steps = steps or cfg["steps"]
    ref = _ctx(K, cfg)
    devs = [_ctx(K, cfg, m, g) for m, g in runs]
    Ur, Us = U0.clone(), [U0.clone() for _ in runs]
    dts = []
    for it in range(steps):
        dt = ref.cfl_dt(Ur, cfg["cfl"])
        dts.append(dt)
        ref.step(Ur, dt)
        for dev, U in zip(devs, Us):
            dev.step(U, dt)
        if (it + 1) % max(1, steps // 5) == 0:
            torch.cuda.synchronize()
            say(f"  {name}: step {it + 1}/{steps}")
    torch.cuda.synchronize()
    assert ref.status() == K.KFVM_OK
    l1 = []
    for dev, U in zip(devs, Us):
        assert dev.status() == K.KFVM_OK
        l1.append(float((U[0] - Ur[0]).abs().mean()))
        dev.close()
    ref.close()
    return l1, dts, U0, cfg


def _replay(K, name, cfg, U0, dts, mode="split_f16"):
    from paper_2401_16543_amd.accuracy import replay_l1
    gated, plain = _ctx(K, cfg, mode, gated=True), _ctx(K, cfg)
    l1, Ug = replay_l1(gated, plain, U0, dts)
    torch.cuda.synchronize()
    assert gated.status() == K.KFVM_OK and plain.status() == K.KFVM_OK
    gated.close()
    plain.close()
    return l1


def _sampled_gated_rhs(K, oracle_mod, name, nsample, tol, mode="split_f16"):
    """Gated RHS over the whole grid against the oracle at sampled cells, the
    oracle replaying the gate's decisions; plus periodic conservation."""
    U, cfg = inputs.config_state(name, device="cuda")
    d, n, R = cfg["d"], cfg["n"], cfg["R"]
    dev = _ctx(K, cfg, mode, gated=True)
    dev.set_checking(True)
    L = dev.rhs(U)
    flags = dev.get_flags().cpu().numpy()
    torch.cuda.synchronize()
    Lh = L.cpu().numpy().reshape(d + 2, -1)
    Uh = U.cpu().numpy()
    dev.close()
    del L, U
    ncell = n ** d
    rng = np.random.default_rng(11)
    # sample troubled cells as well as random ones
    troubled = np.flatnonzero(flags.any(axis=0))
    cells = np.concatenate([[0, ncell - 1, n - 1, ncell - n], rng.integers(0, ncell, nsample),
                            rng.choice(troubled, min(len(troubled), nsample // 2), replace=False)])
    orc = oracle_mod.Oracle(d, R, (n,) * d, gamma=cfg["gamma"])
    orc.set_flags(flags)
    ref = orc.rhs_cells(Uh, cells)
    err = (np.abs(Lh[:, cells].T - ref) / np.abs(Lh).max(axis=1)).max()
    say(f"  {name}: WENO-AO on {flags.mean():.4f} of pairs; sampled rel err {err:.3e} "
        f"({len(cells)} cells, {min(len(troubled), nsample // 2)} of them troubled)")
    assert err <= tol
    tot = np.abs(Lh.sum(axis=1)) / np.abs(Lh).sum(axis=1)
    assert np.all(tot <= 1e-13)


def test_2d_jumps_1024_split_bf16_200_steps(K):
    """Discontinuous 2D workload, 1024^2, R = 2: split BF16 (and split FP16)
    over its 200 steps, L1 of rho at most 1e-4."""
    say("case 2d_jumps_1024: 200 steps split_bf16, split_f16")
    (l1_bf, l1_f), _, _, _ = _trajectories(K, "2d_jumps_1024", [("split_bf16", False), ("split_f16", False)])
    say(f"  L1 rho vs FP64: split_bf16 {l1_bf:.3e}, split_f16 {l1_f:.3e}")
    assert l1_bf <= 1e-4 and l1_f <= 1e-4


def test_3d_smooth_256_split_f16_50_steps(K):
    """Smooth 3D workload, 256^3, R = 2: split FP16 with WENO-AO everywhere
    over its 50 steps, L1 at most 1e-8; with the learned gate, the same
    decisions replayed in FP64 over the first 10 steps, L1 at most 1e-8, and
    the gated run against WENO-AO everywhere (the scheme change) reported."""
    say("case 3d_smooth_256: 50 steps split_f16 (ungated, gated)")
    (l1_ung, l1_gate), dts, U0, cfg = _trajectories(K, "3d_smooth_256", [("split_f16", False),
                                                                          ("split_f16", True)])
    say(f"  L1 rho vs FP64 after 50 steps: split_f16 {l1_ung:.3e}; gated (incl. scheme change) {l1_gate:.3e}")
    assert l1_ung <= 1e-8
    l1_same = _replay(K, "3d_smooth_256", cfg, U0, dts[:10])
    say(f"  gated, same decisions, 10 steps: L1 rho {l1_same:.3e}")
    assert l1_same <= 1e-8


def test_2d_jumps_2048_gated_100_steps(K, oracle_mod):
    """The learned gate's 2D workload, 2048^2, R = 2, over its 100 steps: L1 at
    most 1e-4 both with the same decisions and against WENO-AO everywhere; the
    gated RHS at full size against the oracle replaying the decisions."""
    say("case 2d_jumps_2048: 100 steps split_f16 + gate")
    (l1_gate,), dts, U0, cfg = _trajectories(K, "2d_jumps_2048", [("split_f16", True)])
    l1_same = _replay(K, "2d_jumps_2048", cfg, U0, dts)
    say(f"  L1 rho vs FP64: same decisions {l1_same:.3e}; against WENO-AO everywhere {l1_gate:.3e}")
    assert l1_same <= 1e-4 and l1_gate <= 1e-4
    _sampled_gated_rhs(K, oracle_mod, "2d_jumps_2048", 600, 2e-5)


def test_3d_jumps_384_r3_gated_30_steps(K, oracle_mod):
    """Discontinuous 3D workload, 384^3, R = 3, split FP16 with the learned gate
    over its 30 steps: L1 at most 1e-4 against WENO-AO everywhere, and with the
    same decisions over the first 3 steps; the gated RHS at full size against
    the oracle replaying the decisions."""
    say("case 3d_jumps_384_r3: 30 steps split_f16 + gate")
    torch.cuda.empty_cache()
    (l1_gate,), dts, U0, cfg = _trajectories(K, "3d_jumps_384_r3", [("split_f16", True)])
    say(f"  L1 rho vs FP64 WENO-AO everywhere after 30 steps: {l1_gate:.3e}")
    assert l1_gate <= 1e-4
    l1_same = _replay(K, "3d_jumps_384_r3", cfg, U0, dts[:3])
    say(f"  same decisions, 3 steps: L1 rho {l1_same:.3e}")
    assert l1_same <= 1e-4
    del U0
    torch.cuda.empty_cache()
    _sampled_gated_rhs(K, oracle_mod, "3d_jumps_384_r3", 40, 2e-5)
